"""Algorithmic bytes per ray of the BVH method (roofline accounting).

B_alg = 32 B x (ray-box tests) + 40 B x (ray-triangle tests: 36 B of vertices
+ 4 B id) + 8 B of output (depth + label), with the test counts taken from a
canonical traversal (``canon_bvh.c``: full-sweep SAH BVH2, leaves <= 4,
nearest-first with a shrinking interval) over a seeded sample of each
workload.  The counts are a property of the method and the scene, not of the
GPU code; they are frozen in ``bytes_model.json`` by running this module:

    python -m bytemodel.bytemodel
"""
from __future__ import annotations

import ctypes as C
import json
import math
import os
import subprocess
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
JSON = os.path.join(HERE, "bytes_model.json")
SAMPLES = {1: None, 2: 12, 3: 32, 4: 24}  # environments per workload (None = all)


def _lib():
    so = os.path.join(HERE, "libcanon.so")
    src = os.path.join(HERE, "canon_bvh.c")
    if not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", so, src, "-lm"])
    L = C.CDLL(so)
    f32 = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
    L.canon_counts.argtypes = [C.c_int64, f32, C.c_int64, f32, f32, f32, f32, C.POINTER(C.c_double),
                               C.POINTER(C.c_double), C.POINTER(C.c_int32)]
    return L


def _world(scene, e):
    """World triangles of environment e (float64 affine, stored as float32)."""
    out = []
    for j in range(scene.inst_offsets[e], scene.inst_offsets[e + 1]):
        v, t = scene.protos[scene.inst_mesh[j]]
        A = scene.inst_T[j].astype(np.float64).reshape(3, 4)
        w = v.astype(np.float64) @ A[:, :3].T + A[:, 3]
        out.append(w[t].reshape(-1, 9))
    return np.concatenate(out).astype(np.float32) if out else np.zeros((0, 9), np.float32)


def _rays(scene, s):
    desc = scene.sensors[int(scene.sensor_ids[s])]
    W, H = desc.width, desc.height
    r = np.arange(W * H)
    row, col = r // W, r % W
    if desc.kind == 0:
        sc = math.tan(desc.hfov / 2) / (W / 2)
        dl = np.stack([np.ones(W * H), -(col + 0.5 - W / 2) * sc, -(row + 0.5 - H / 2) * sc], 1)
    elif desc.kind == 1:
        el = desc.vmax - row * (desc.vmax - desc.vmin) / max(H - 1, 1)
        az = desc.hmin + col * (desc.hmax - desc.hmin) / W
        dl = np.stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)], 1)
    else:
        dl = desc.dir_table.astype(np.float64)
    P = scene.sensor_T[s].astype(np.float64).reshape(3, 4)
    d = dl @ P[:, :3].T
    o = np.broadcast_to(P[:, 3], d.shape)
    n = len(d)
    return (np.ascontiguousarray(o, np.float32), np.ascontiguousarray(d, np.float32),
            np.full(n, desc.near, np.float32), np.full(n, desc.far, np.float32))


def measure(cfg: int, n_envs=None, seed: int = 0) -> dict:
    sys.path.insert(0, ROOT)
    from paper_2503_01471_amd import scenes as S
    L = _lib()
    if cfg == 1:
        scene = S.make_cfg1(seed)
    else:
        scene = S.make(cfg, env_ids=list(range(n_envs)), seed=seed)
    box, tri = C.c_double(0), C.c_double(0)
    depth = C.c_int32(0)
    rays = 0
    for e in range(scene.n_envs):
        w = np.ascontiguousarray(_world(scene, e))
        for s in range(scene.sens_offsets[e], scene.sens_offsets[e + 1]):
            o, d, tn, tf = _rays(scene, s)
            L.canon_counts(len(w), w, len(o), o, d, tn, tf, C.byref(box), C.byref(tri), C.byref(depth))
            rays += len(o)
    bpr, tpr = box.value / rays, tri.value / rays
    return {"box_tests_per_ray": bpr, "tri_tests_per_ray": tpr, "bytes_per_ray": 32 * bpr + 40 * tpr + 8,
            "sample": f"envs 0..{scene.n_envs - 1} of cfg{cfg} (seed {seed}), all {rays} rays",
            "max_stack": depth.value}


def load() -> dict:
    with open(JSON) as f:
        return json.load(f)


def main():
    res = {"definition": "32 B per ray-box test + 40 B per ray-triangle test + 8 B output; counts from a "
                         "full-sweep SAH BVH2 (leaf <= 4) traversed nearest-first with a shrinking interval"}
    for cfg, n in SAMPLES.items():
        res[f"cfg{cfg}"] = measure(cfg, n)
        print(cfg, res[f"cfg{cfg}"], flush=True)
    with open(JSON, "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
