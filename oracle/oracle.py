"""Python front end of the brute-force CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It loads ``liboracle.so`` (built from ``rc_oracle.c`` with
gcc, see :func:`build`) and never touches the HIP renderer; the only thing it
shares with the renderer is the scene object produced by the seeded input
generators, which it reads attribute by attribute.

What the oracle computes is the brute-force nearest hit over every triangle of
a ray's own environment (paper, Sec. III-D "Exteroceptive Sensors": sub-meshes
moved by their transforms, one ray per pixel or beam, depth for cameras and
range for LiDARs).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rc_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

HIT, B_BARY, B_GAP, B_RANGE, B_GRAZE, B_NEARMISS = 1, 2, 4, 8, 16, 32
BORDER_MASK = B_BARY | B_GAP | B_RANGE | B_GRAZE | B_NEARMISS

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (IEEE arithmetic: no contraction, no fast-math)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-o", tmp, SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


def load(path: str):
    """Open an oracle build at ``path`` and declare its entry points."""
    L = C.CDLL(path)
    f32, f64, i32, i64 = (np.ctypeslib.ndpointer(t, flags="C_CONTIGUOUS")
                          for t in (np.float32, np.float64, np.int32, np.int64))
    L.orc_transform.argtypes = [C.c_int64, f32, i32, f32, f32]
    L.orc_transform.restype = None
    L.orc_rays.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_float, C.c_float, C.c_float,
                           C.c_float, C.c_float, C.c_void_p, f32, C.c_int64, i64, f32, f32, C.c_void_p]
    L.orc_rays.restype = None
    L.orc_cast.argtypes = [f32, i64, C.c_int64, i32, f32, f32, f32, f32, C.c_int32,
                           f64, i32, f64, f64, f64, f64, f64, f64, i32]
    L.orc_cast.restype = None
    L.orc_transform64.argtypes = [C.c_int64, f32, i32, f32, f64]
    L.orc_transform64.restype = None
    L.orc_cast64.argtypes = [f64, i64, C.c_int64, i32, f32, f32, f32, f32, C.c_int32,
                             f64, i32, f64, f64, f64, f64, f64, f64, i32]
    L.orc_cast64.restype = None
    L.orc_move.argtypes = [C.c_int64, f32, f32, np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS"),
                           C.c_int32, C.c_float, f32]
    L.orc_move.restype = None
    L.orc_extras.argtypes = [f32, i64, C.c_int64, i32, i32, f32, f32, f64, f32, f32]
    L.orc_extras.restype = None
    L.orc_shadow.argtypes = [f32, i64, C.c_int64, i32, i32, f32, f32, f32, C.c_int32,
                             np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS"), i32]
    L.orc_shadow.restype = None
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = load(LIB)
    return _lib


# --------------------------------------------------------------------------
# world mesh
# --------------------------------------------------------------------------
@dataclass
class World:
    tris: np.ndarray  # float32 [N,9] (float64 from world64)
    env_off: np.ndarray  # int64 [E+1]
    tri_inst: np.ndarray  # int32 [N] global instance index
    tri_seg: np.ndarray  # int32 [N]


def world_corners(scene, inst_T=None):
    """Prototype corner coordinates and owning instance of every world triangle,
    env-local order = instances in CSR order, then prototype triangle order."""
    counts = np.array([len(t) for _, t in scene.protos], np.int64)
    per_inst = counts[scene.inst_mesh]
    tri_inst = np.repeat(np.arange(scene.n_inst, dtype=np.int32), per_inst)
    corners = np.empty((len(tri_inst), 9), np.float32)
    pos = 0
    # instances of the same prototype share the corner block; fill instance by instance
    proto_corners = [v[t].reshape(-1, 9) for v, t in scene.protos]
    starts = np.concatenate([[0], np.cumsum(per_inst)])
    for m, pc in enumerate(proto_corners):
        idx = np.nonzero(scene.inst_mesh == m)[0]
        if len(idx) == 0:
            continue
        rows = (starts[idx][:, None] + np.arange(len(pc))[None, :]).reshape(-1)
        corners[rows] = np.tile(pc, (len(idx), 1))
    pos = starts[-1]
    assert pos == len(tri_inst)
    inst_tri_cs = np.concatenate([[0], np.cumsum(per_inst)])
    env_off = inst_tri_cs[scene.inst_offsets].astype(np.int64)
    return corners, tri_inst, env_off


def world(scene, inst_T=None) -> World:
    """World triangles of every environment (FP32 fused-multiply-add transform)."""
    T = np.ascontiguousarray(scene.inst_T if inst_T is None else inst_T, np.float32)
    corners, tri_inst, env_off = world_corners(scene)
    out = np.empty_like(corners)
    lib().orc_transform(len(corners), corners, tri_inst, T, out)
    return World(out, env_off, tri_inst, scene.inst_seg[tri_inst].astype(np.int32))


def world64(scene, inst_T=None) -> World:
    """World triangles with the moved vertices kept in FP64, unrounded
    (``orc_transform64``): the composition of each sub-mesh with its transform
    that a renderer intersecting in each sub-mesh's own frame computes."""
    T = np.ascontiguousarray(scene.inst_T if inst_T is None else inst_T, np.float32)
    corners, tri_inst, env_off = world_corners(scene)
    out = np.empty(corners.shape, np.float64)
    lib().orc_transform64(len(corners), corners, tri_inst, T, out)
    return World(out, env_off, tri_inst, scene.inst_seg[tri_inst].astype(np.int32))


def moved_poses(scene, step: int) -> np.ndarray:
    """Instance poses after ``step`` steps of constant velocity (``orc_move``)."""
    T = np.empty_like(np.ascontiguousarray(scene.inst_T, np.float32))
    lib().orc_move(scene.n_inst, np.ascontiguousarray(scene.inst_T, np.float32),
                   np.ascontiguousarray(scene.inst_vel, np.float32),
                   np.ascontiguousarray(scene.inst_dynamic, np.uint8), int(step), float(scene.dt), T)
    return T


# --------------------------------------------------------------------------
# rays
# --------------------------------------------------------------------------
def sensor_rays(scene, s: int, ray_idx=None, local=False):
    """World rays (FP32 origin and direction) of sensor instance ``s``; with
    ``local`` also the sensor-frame directions."""
    desc = scene.sensors[int(scene.sensor_ids[s])]
    n_all = desc.width * desc.height
    idx = np.arange(n_all, dtype=np.int64) if ray_idx is None else np.ascontiguousarray(ray_idx, np.int64)
    o = np.empty((len(idx), 3), np.float32)
    d = np.empty((len(idx), 3), np.float32)
    table = None
    if desc.kind == 2:
        table = np.ascontiguousarray(desc.dir_table, np.float32)
    pose = np.ascontiguousarray(scene.sensor_T[s], np.float32)
    dl = np.empty((len(idx), 3), np.float32)
    lib().orc_rays(desc.kind, desc.width, desc.height, desc.hfov, desc.vmin, desc.vmax, desc.hmin,
                   desc.hmax, None if table is None else table.ctypes.data_as(C.c_void_p), pose,
                   len(idx), idx, o, d, dl.ctypes.data_as(C.c_void_p))
    return (o, d, dl) if local else (o, d)


def sensor_env(scene) -> np.ndarray:
    return np.repeat(np.arange(scene.n_envs, dtype=np.int32), np.diff(scene.sens_offsets))


# --------------------------------------------------------------------------
# nearest hit
# --------------------------------------------------------------------------
def cast(w: World, ray_env, o, d, near, far, nthreads: int = 0) -> dict:
    """Brute-force FP64 nearest hit of explicit rays (see ``orc_cast``)."""
    n = len(ray_env)
    ray_env = np.ascontiguousarray(ray_env, np.int32)
    o = np.ascontiguousarray(o, np.float32).reshape(n, 3)
    d = np.ascontiguousarray(d, np.float32).reshape(n, 3)
    near = np.ascontiguousarray(np.broadcast_to(np.float32(near) if np.isscalar(near) else near, (n,)), np.float32)
    far = np.ascontiguousarray(np.broadcast_to(np.float32(far) if np.isscalar(far) else far, (n,)), np.float32)
    out = dict(t=np.empty(n), tri=np.empty(n, np.int32), u=np.empty(n), v=np.empty(n),
               hit=np.empty((n, 3)), mb=np.empty(n), md=np.empty(n), g=np.empty(n),
               cls=np.empty(n, np.int32))
    if nthreads <= 0:
        nthreads = len(os.sched_getaffinity(0))
    if w.tris.dtype == np.float64:
        fn, tris = lib().orc_cast64, np.ascontiguousarray(w.tris, np.float64)
    else:
        fn, tris = lib().orc_cast, np.ascontiguousarray(w.tris, np.float32)
    fn(tris, np.ascontiguousarray(w.env_off, np.int64), n, ray_env, o, d, near, far, nthreads, out["t"],
       out["tri"], out["u"], out["v"], out["hit"], out["mb"], out["md"], out["g"], out["cls"])
    return out


@dataclass
class Render:
    """Oracle outputs for a list of (sensor instance, ray) pairs."""
    depth: np.ndarray  # float32, -1 on miss
    seg: np.ndarray  # int32, -1 on miss
    tri: np.ndarray  # int32 env-local, -1 on miss
    hit: np.ndarray  # float32 [n,3], NaN on miss
    t: np.ndarray  # float64
    cls: np.ndarray  # classification bits
    raw: dict
    normal: np.ndarray = None  # float32 [n,3] unit, facing the sensor; NaN on miss
    bary: np.ndarray = None    # float32 [n,2] (u, v) of the winner; NaN on miss
    point: np.ndarray = None   # float32 [n,3] sensor frame; NaN on miss
    vert: np.ndarray = None    # int32 [n,3] global prototype vertex ids; -1 on miss
    shadow: np.ndarray = None  # uint8 [n] 1 = hidden from the stereo pair's second camera
    shadow_cls: np.ndarray = None  # int32 [n] bit 1 occluded, bit 2 borderline


def render(scene, w: World = None, sensor_inst=None, ray_idx=None, nthreads: int = 0) -> Render:
    """Oracle render.  With no selection, every ray of every sensor instance in
    ray-major order (sensor instance, then ray); otherwise the given pairs."""
    if w is None:
        w = world(scene)
    S = len(scene.sensor_ids)
    if sensor_inst is None:
        sensor_inst = np.repeat(np.arange(S), scene.rays_per_sensor_inst())
        ray_idx = np.concatenate([np.arange(scene.sensors[int(k)].n_rays) for k in scene.sensor_ids])
    sensor_inst = np.asarray(sensor_inst, np.int64)
    ray_idx = np.asarray(ray_idx, np.int64)
    n = len(sensor_inst)
    o = np.empty((n, 3), np.float32)
    d = np.empty((n, 3), np.float32)
    dl = np.empty((n, 3), np.float32)
    near = np.empty(n, np.float32)
    far = np.empty(n, np.float32)
    senv = sensor_env(scene)
    for s in np.unique(sensor_inst):
        sel = np.nonzero(sensor_inst == s)[0]
        o[sel], d[sel], dl[sel] = sensor_rays(scene, int(s), ray_idx[sel], local=True)
        desc = scene.sensors[int(scene.sensor_ids[s])]
        near[sel], far[sel] = desc.near, desc.far
    ray_env = senv[sensor_inst]
    r = cast(w, ray_env, o, d, near, far, nthreads)
    hitm = r["tri"] >= 0
    depth = np.where(hitm, r["t"], -1.0).astype(np.float32)
    glob = w.env_off[ray_env] + np.maximum(r["tri"], 0)
    seg = np.where(hitm, w.tri_seg[glob], -1).astype(np.int32)
    hit = np.where(hitm[:, None], r["hit"], np.nan).astype(np.float32)
    # further data types of the same hit (Sec. III-D): normal and point cloud
    # (orc_extras), barycentric coordinates (the winner's u, v) and the
    # winner's prototype vertex ids for vertex-level annotations
    normal = np.empty((n, 3), np.float32)
    point = np.empty((n, 3), np.float32)
    lib().orc_extras(np.ascontiguousarray(w.tris, np.float32), np.ascontiguousarray(w.env_off, np.int64), n,
                     np.ascontiguousarray(ray_env, np.int32), np.ascontiguousarray(r["tri"], np.int32), d, dl,
                     np.ascontiguousarray(r["t"]), normal, point)
    bary = np.where(hitm[:, None], np.stack([r["u"], r["v"]], 1), np.nan).astype(np.float32)
    vert = np.where(hitm[:, None], tri_vertex_ids(scene)[glob], -1).astype(np.int32)
    # stereo shadows: segments from the FP32 hit points back to the second
    # camera of sensors that have one (orc_shadow)
    base = np.array([scene.sensors[int(k)].stereo for k in scene.sensor_ids], np.float32).reshape(-1, 3)
    has = np.any(base != 0, 1)[sensor_inst]
    shadow = np.zeros(n, np.uint8)
    shadow_cls = np.zeros(n, np.int32)
    sel = np.nonzero(has & hitm)[0]
    if len(sel):
        occ = np.zeros(len(sel), np.uint8)
        cls = np.zeros(len(sel), np.int32)
        lib().orc_shadow(np.ascontiguousarray(w.tris, np.float32), np.ascontiguousarray(w.env_off, np.int64),
                         len(sel), np.ascontiguousarray(ray_env[sel], np.int32),
                         np.ascontiguousarray(r["tri"][sel], np.int32), np.ascontiguousarray(hit[sel]),
                         np.ascontiguousarray(np.asarray(scene.sensor_T, np.float32)[sensor_inst[sel]]),
                         np.ascontiguousarray(base[sensor_inst[sel]]), nthreads if nthreads > 0 else
                         len(os.sched_getaffinity(0)), occ, cls)
        shadow[sel] = occ
        shadow_cls[sel] = cls
    return Render(depth, seg, r["tri"].copy(), hit, r["t"], r["cls"], r, normal, bary, point, vert, shadow,
                  shadow_cls)


def tri_vertex_ids(scene) -> np.ndarray:
    """Global vertex ids (prototypes' vertices numbered in prototype order) of
    the three corners of every world triangle, in world-triangle order."""
    vbase = np.concatenate([[0], np.cumsum([len(v) for v, _ in scene.protos])]).astype(np.int64)
    per = [np.asarray(t, np.int64) + vbase[m] for m, (_, t) in enumerate(scene.protos)]
    return np.concatenate([per[m] for m in scene.inst_mesh]) if scene.n_inst else np.zeros((0, 3), np.int64)
