"""Pins of the CPU oracle: checks against facts that do not come from the oracle.

Each ``pin_*`` function runs one family of checks against the oracle library
currently loaded by ``oracle.oracle`` and returns a list of failure messages
(empty = pinned).  The pin tests assert emptiness; the mutation test swaps in
deliberately broken oracle builds and asserts that every one of them is caught
by at least one pin.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import exact
from oracle import oracle as O
from paper_2503_01471_amd import scenes as S

F32 = np.float32


def _world_of(tris):
    tris = np.ascontiguousarray(np.asarray(tris, np.float32).reshape(-1, 9))
    n = len(tris)
    return O.World(tris, np.array([0, n], np.int64), np.zeros(n, np.int32), np.zeros(n, np.int32))


# --------------------------------------------------------------------------
# 1. exact rational arithmetic on tiny adversarial scenes
# --------------------------------------------------------------------------
def tiny_scene(seed: int):
    """1-4 triangles and 64 rays; the family rotates over random triangles,
    shared edges, coplanar overlaps, axis-aligned faces and degenerate triangles."""
    rng = np.random.default_rng(seed)
    kind = seed % 5
    if kind == 0:
        tris = rng.uniform(-1, 1, (int(rng.integers(1, 5)), 9))
    elif kind == 1:  # quad split along a diagonal + one random triangle
        p = rng.uniform(-1, 1, (4, 3))
        p[3] = p[0] + (p[2] - p[1])  # planar parallelogram
        tris = [np.r_[p[0], p[1], p[2]], np.r_[p[0], p[2], p[3]], rng.uniform(-1, 1, 9)]
    elif kind == 2:  # coplanar overlapping triangles in z = c
        c = rng.uniform(-0.5, 0.5)
        tris = []
        for _ in range(3):
            xy = rng.uniform(-1, 1, (3, 2))
            tris.append(np.c_[xy, np.full(3, c)].reshape(9))
    elif kind == 3:  # axis-aligned box faces with representable coordinates
        lo = np.round(rng.uniform(-1, 0, 3) * 8) / 8
        hi = lo + np.round(rng.uniform(0.25, 1, 3) * 8) / 8
        v = np.array([[x, y, z] for z in (lo[2], hi[2]) for y in (lo[1], hi[1]) for x in (lo[0], hi[0])])
        tris = [np.r_[v[0], v[2], v[3]], np.r_[v[0], v[3], v[1]], np.r_[v[1], v[3], v[7]],
                np.r_[v[1], v[7], v[5]]]
    else:  # degenerate: collinear and repeated vertices, plus a proper triangle
        a, b = rng.uniform(-1, 1, (2, 3))
        tris = [np.r_[a, b, 0.5 * (a + b)], np.r_[a, a, b], rng.uniform(-1, 1, 9)]
    tris = np.asarray(tris, np.float64).reshape(-1, 9).astype(np.float32)
    o = rng.uniform(-3, 3, 3)
    o[2] = 2.5 + rng.uniform(0, 1)
    # aim at an 8x8 grid over the triangles' bounding box, plus edge points
    lo, hi = tris.reshape(-1, 3).min(0), tris.reshape(-1, 3).max(0)
    g = np.linspace(0, 1, 8)
    targets = [lo + (hi - lo) * np.array([a, b, rng.random()]) for a in g for b in g]
    for k in range(min(len(tris), 4)):
        t = tris[k].reshape(3, 3).astype(np.float64)
        targets[k] = 0.5 * (t[0] + t[1])
        targets[8 + k] = 0.5 * (t[1] + t[2])
        targets[16 + k] = t[0]
    d = (np.array(targets) - o).astype(np.float32)
    o = np.tile(o.astype(np.float32), (len(d), 1))
    return tris, o, d


def _t_tol(tri, o, d, t):
    """FP64 error bound for t of a Moller-Trumbore solve: a few ulps times the
    conditioning |e1||e2||d| / |det| of the 3x3 system (large for slivers and
    grazing rays), scaled by how far the origin is from the triangle."""
    a, b, c = (np.asarray(tri[3 * i:3 * i + 3], float) for i in range(3))
    d = np.asarray(d, float)
    e1, e2 = b - a, c - a
    det = abs(np.dot(e1, np.cross(d, e2)))
    kappa = np.linalg.norm(e1) * np.linalg.norm(e2) * np.linalg.norm(d) / det
    reach = max(1.0, np.linalg.norm(np.asarray(o, float) - a) / (abs(t) * np.linalg.norm(d)))
    return 1e-14 * abs(t) * max(1.0, kappa) * reach


def pin_exact(seeds=range(200), near=0.05, far=50.0, margin_tol=1e-12):
    fails = []
    for seed in seeds:
        tris, o, d = tiny_scene(seed)
        r = O.cast(_world_of(tris), np.zeros(len(o), np.int32), o, d, near, far, nthreads=1)
        for i in range(len(o)):
            k, t, u, v, m = exact.nearest(list(tris), o[i], d[i], near, far)
            if m <= margin_tol:
                continue
            if r["tri"][i] != k:
                fails.append(f"exact seed {seed} ray {i}: oracle tri {r['tri'][i]} exact {k}")
                continue
            if k >= 0 and abs(r["t"][i] - float(t)) > _t_tol(tris[k], o[i], d[i], float(t)):
                fails.append(f"exact seed {seed} ray {i}: t {r['t'][i]} exact {float(t)}")
            if k >= 0:  # barycentric coordinates of the winner (vertex-level annotations)
                tol = _t_tol(tris[k], o[i], d[i], float(t)) / max(abs(float(t)), 1e-300)
                if abs(r["u"][i] - float(u)) > tol or abs(r["v"][i] - float(v)) > tol:
                    fails.append(f"exact seed {seed} ray {i}: (u, v) ({r['u'][i]}, {r['v'][i]}) exact "
                                 f"({float(u)}, {float(v)})")
    return fails


def pin_duplicate_tie():
    """Identical triangles tie exactly; the lower triangle id must win."""
    tri = np.array([0, 0, 1, 1, 0, 1, 0, 1, 1], np.float32)
    rng = np.random.default_rng(7)
    tgt = np.c_[rng.uniform(0.05, 0.45, (64, 2)), np.ones(64)]
    o = np.zeros((64, 3), np.float32)
    d = tgt.astype(np.float32)
    r = O.cast(_world_of([tri, tri]), np.zeros(64, np.int32), o, d, 0.1, 10.0, nthreads=1)
    bad = np.nonzero(r["tri"] != 0)[0]
    return [f"tie ray {i}: tri {r['tri'][i]}" for i in bad]


# --------------------------------------------------------------------------
# 2. closed forms
# --------------------------------------------------------------------------
def _ground_scene(sensor, pose):
    inst = [(0, 0, S.affine(np.diag([200.0, 200.0, 1.0]), (-100.0, -100.0, 0.0)), 0, (0, 0, 0))]
    return S.custom_scene([S.quad_mesh()], [(inst, [(0, pose)])], [sensor])


def pin_ray_plane():
    """Level sensors above an infinite-looking ground plane: depth / range
    follow from the pixel or beam geometry alone."""
    fails = []
    h = 1.5
    # pinhole: depth of row v = h / ((v + 1/2 - H/2) s),  s = tan(hfov/2)/(W/2)
    W, H = 64, 48
    cam = S.pinhole(W, H, 87.0, near=0.2, far=80.0)
    for yaw in (0.0, 0.7, 2.9):
        sc = _ground_scene(cam, S.sensor_pose(S.rot_zyx(yaw), (1.25, -2.5, h)))
        r = O.render(sc, nthreads=1)
        s = math.tan(float(F32(cam.hfov)) / 2) / (W / 2)
        for v in range(H):
            k = (v + 0.5 - H / 2) * s
            row = slice(v * W, (v + 1) * W)
            if k <= 0:
                if np.any(r.tri[row] != -1):
                    fails.append(f"plane: row {v} above horizon hits")
                continue
            depth = h / k
            if depth > 80.0:
                continue
            got = r.t[row]
            if np.any(np.abs(got - depth) > 1e-6 * depth):
                fails.append(f"plane: yaw {yaw} row {v} depth {got.min()}..{got.max()} want {depth}")
            # exact plane intersection of the FP32 rays: t = -o_z / d_z
            o, d = O.sensor_rays(sc, 0, np.arange(v * W, (v + 1) * W))
            tz = -o[:, 2].astype(np.float64) / d[:, 2].astype(np.float64)
            if np.any(np.abs(got - tz) > 1e-12 * tz):
                fails.append(f"plane: row {v} not on z=0")
    # LiDAR: range of channel c = h / sin(-el_c) for every azimuth
    lid = S.lidar(64, 16, 90.0, near=0.1, far=80.0)
    sc = _ground_scene(lid, S.sensor_pose(S.rot_zyx(0.3), (0.5, 0.25, h)))
    r = O.render(sc, nthreads=1)
    for c in range(16):
        el = float(F32(lid.vmax)) - c * (float(F32(lid.vmax)) - float(F32(lid.vmin))) / 15
        row = slice(c * 64, (c + 1) * 64)
        if el >= 0:
            if np.any(r.tri[row] != -1):
                fails.append(f"lidar: channel {c} above horizon hits")
            continue
        rng_ = h / math.sin(-el)
        if np.any(np.abs(r.t[row] - rng_) > 1e-6 * rng_):
            fails.append(f"lidar: channel {c} range {r.t[row].min()} want {rng_}")
    return fails


def _slab(lo, hi, o, d):
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = (lo - o) / d
        t2 = (hi - o) / d
    tmin = np.nanmax(np.minimum(t1, t2), axis=-1)
    tmax = np.nanmin(np.maximum(t1, t2), axis=-1)
    return tmin, tmax


def pin_boxes(seed=0):
    """cfg1 (ground + axis-aligned boxes): the 12-triangle box is exactly the box
    surface, so on rays away from edges the nearest hit equals the nearest slab
    entry/exit over all boxes and the ground plane, computed in FP64."""
    fails = []
    sc = S.make_cfg1(seed)
    w = O.world(sc)
    r = O.render(sc, w, nthreads=1)
    o, d = O.sensor_rays(sc, 0)
    o64, d64 = o.astype(np.float64), d.astype(np.float64)
    desc = sc.sensors[0]
    n = len(o)
    best_t = np.full(n, np.inf)
    best_seg = np.full(n, -1)
    for j in range(sc.n_inst):
        rows = np.nonzero(w.tri_inst == j)[0]
        pts = w.tris[rows].reshape(-1, 3).astype(np.float64)
        lo, hi = pts.min(0), pts.max(0)
        tmin, tmax = _slab(lo, hi, o64, d64)
        ok = tmin <= tmax
        cand = np.where(ok & (tmin >= desc.near), tmin, np.where(ok & (tmax >= desc.near), tmax, np.inf))
        cand[cand > desc.far] = np.inf
        better = cand < best_t
        best_t[better] = cand[better]
        best_seg[better] = sc.inst_seg[j]
    robust = (r.cls & O.BORDER_MASK) == 0
    hit_ref = np.isfinite(best_t)
    bad = robust & ((r.tri >= 0) != hit_ref)
    if bad.any():
        fails.append(f"boxes: hit/miss differs on {bad.sum()} robust rays")
    both = robust & hit_ref & (r.tri >= 0)
    err = np.abs(r.t[both] - best_t[both]) / best_t[both]
    if err.size and err.max() > 1e-12:
        fails.append(f"boxes: max rel depth err {err.max()}")
    if np.any(r.seg[both] != best_seg[both]):
        fails.append(f"boxes: seg differs on {(r.seg[both] != best_seg[both]).sum()} rays")
    if robust.sum() < 0.9 * n:
        fails.append("boxes: too few robust rays")
    return fails


def _sphere_t(o, d, R):
    """Entry parameter of ray o + t d into the ball |x| <= R (inf if none)."""
    a = (d * d).sum(-1)
    b = 2 * (o * d).sum(-1)
    c = (o * o).sum(-1) - R * R
    disc = b * b - 4 * a * c
    with np.errstate(invalid="ignore"):
        t = (-b - np.sqrt(disc)) / (2 * a)
    return np.where(disc >= 0, t, np.inf)


def pin_tessellated():
    """Convex tessellations bracket the smooth surface: a level-5 icosphere P
    with inradius r_in and circumradius R satisfies B(r_in) <= P <= B(R), so
    t(B(R)) <= t_mesh <= t(B(r_in)); likewise an N-gon prism of radius r lies
    between the cylinders of radius r cos(pi/N) and r."""
    fails = []
    v, t = S.icosphere_mesh(5)
    tri = v[t].reshape(-1, 9)
    a, b, c = tri[:, :3].astype(float), tri[:, 3:6].astype(float), tri[:, 6:].astype(float)
    nrm = np.cross(b - a, c - a)
    r_in = np.min(np.abs((nrm * a).sum(1)) / np.linalg.norm(nrm, axis=1))
    R = np.max(np.linalg.norm(v.astype(float), axis=1))
    rng = np.random.default_rng(3)
    n = 512
    o = rng.normal(size=(n, 3))
    o = (3.0 * o / np.linalg.norm(o, axis=1, keepdims=True)).astype(np.float32)
    tgt = rng.uniform(-0.9, 0.9, (n, 3)) * 0.6
    d = (tgt - o).astype(np.float32)
    r = O.cast(_world_of(tri), np.zeros(n, np.int32), o, d, 0.0, 100.0)
    o64, d64 = o.astype(float), d.astype(float)
    t_out, t_in = _sphere_t(o64, d64, R), _sphere_t(o64, d64, r_in)
    sel = np.isfinite(t_in)
    if np.any(r["tri"][sel] < 0):
        fails.append("sphere: ray through inner ball missed")
    lo_ok = r["t"][sel] >= t_out[sel] * (1 - 1e-12)
    hi_ok = r["t"][sel] <= t_in[sel] * (1 + 1e-12)
    if not (lo_ok.all() and hi_ok.all()):
        fails.append(f"sphere: bracket violated on {(~lo_ok).sum() + (~hi_ok).sum()} rays")
    miss_outer = ~np.isfinite(t_out)
    if np.any(r["tri"][miss_outer] >= 0):
        fails.append("sphere: ray outside the outer ball hit")
    if (1 - r_in / R) > 2e-3:
        fails.append("sphere: tessellation bound too loose")
    # 16-gon prism side: horizontal rays at mid height, 2-D bracket
    v, t = S.cylinder_mesh(16)
    tri = v[t].reshape(-1, 9)
    m = 256
    ang = rng.uniform(0, 2 * np.pi, m)
    o = np.c_[4 * np.cos(ang), 4 * np.sin(ang), np.full(m, 0.5)]
    off = rng.uniform(-0.8, 0.8, m)
    tgt = np.c_[-np.sin(ang) * off, np.cos(ang) * off, np.full(m, 0.5)]
    o, d = o.astype(np.float32), (tgt - o).astype(np.float32)
    r = O.cast(_world_of(tri), np.zeros(m, np.int32), o, d, 0.0, 100.0)
    o2, d2 = o[:, :2].astype(float), d[:, :2].astype(float)

    def circ(rad):
        a_ = (d2 * d2).sum(1)
        b_ = 2 * (o2 * d2).sum(1)
        c_ = (o2 * o2).sum(1) - rad * rad
        disc = b_ * b_ - 4 * a_ * c_
        with np.errstate(invalid="ignore"):
            return np.where(disc >= 0, (-b_ - np.sqrt(disc)) / (2 * a_), np.inf)

    t_out, t_in = circ(1.0), circ(math.cos(math.pi / 16))
    sel = np.isfinite(t_in)
    if np.any(r["tri"][sel] < 0) or np.any(r["t"][sel] < t_out[sel] * (1 - 1e-12)) or \
            np.any(r["t"][sel] > t_in[sel] * (1 + 1e-12)):
        fails.append("prism: bracket violated")
    return fails


# --------------------------------------------------------------------------
# 3. invariants
# --------------------------------------------------------------------------
def pin_invariants():
    fails = []
    sc = S.make_cfg2(n_envs=2, W=96, H=54)
    w = O.world(sc)
    r = O.render(sc, w)
    desc = sc.sensors[0]
    hit = r.tri >= 0
    if np.any((r.t[hit] < desc.near) | (r.t[hit] > desc.far)):
        fails.append("invariant: depth outside [near, far]")
    # hit point lies on the winning triangle's plane
    S_ = sc.rays_per_sensor_inst()
    env = np.repeat(O.sensor_env(sc), S_)
    g = w.env_off[env[hit]] + r.tri[hit]
    T = w.tris[g].astype(np.float64)
    a, b, c = T[:, :3], T[:, 3:6], T[:, 6:]
    nrm = np.cross(b - a, c - a)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    p = r.raw["hit"][hit]
    dist = np.abs(((p - a) * nrm).sum(1))
    if dist.max() > 1e-9 * 20:
        fails.append(f"invariant: hit off plane by {dist.max()}")
    # segmentation = label of the instance owning the triangle (CSR definition)
    counts = sc.proto_tri_counts()[sc.inst_mesh]
    owner = np.repeat(np.arange(sc.n_inst), counts)
    if np.any(r.seg[hit] != sc.inst_seg[owner[g]]):
        fails.append("invariant: seg != owner label")
    # closed room and far beyond its diagonal: no ray escapes
    far_desc = S.pinhole(96, 54, 87.0, 0.2, 20.0)
    sc2 = S.Scene(**{**sc.__dict__, "sensors": [far_desc]})
    r2 = O.render(sc2, w)
    if np.any(r2.tri < 0):
        fails.append(f"invariant: {np.sum(r2.tri < 0)} misses inside a closed room")
    # environment permutation permutes outputs; duplicates agree
    rp = O.render(S.subset(sc, [1, 0, 1]))
    n0 = desc.n_rays
    if not (np.array_equal(rp.tri[:n0], r.tri[n0:]) and np.array_equal(rp.tri[n0:2 * n0], r.tri[:n0])
            and np.array_equal(rp.tri[2 * n0:], r.tri[n0:])):
        fails.append("invariant: permutation/duplicate mismatch")
    # translating the whole scene (instances + sensors) moves nothing relative
    shift = np.array([8.0, -4.0, 2.0], np.float32)
    scs = S.Scene(**sc.__dict__)
    scs.inst_T = sc.inst_T.copy()
    scs.sensor_T = sc.sensor_T.copy()
    for k, col in enumerate((3, 7, 11)):
        scs.inst_T[:, col] += shift[k]
        scs.sensor_T[:, col] += shift[k]
    rs = O.render(scs)
    rob = ((r.cls & O.BORDER_MASK) == 0) & ((rs.cls & O.BORDER_MASK) == 0)
    if np.any(rs.tri[rob] != r.tri[rob]):
        fails.append("invariant: translation changed robust winners")
    hh = rob & hit
    # vertices move by up to an FP32 rounding (|coord| <= 20 m), which shifts
    # the hit along the ray by that amount over the grazing cosine
    tol = 8 * 2.0 ** -24 * 20.0 / r.raw["g"][hh] + 1e-6 * r.t[hh]
    if np.any(np.abs(rs.t[hh] - r.t[hh]) > tol):
        fails.append("invariant: translation changed depth")
    return fails


def pin_transform():
    """World vertices vs an FP64 evaluation of A[:, :3] v + A[:, 3]."""
    fails = []
    sc = S.make_cfg2(n_envs=2, W=16, H=9)
    w = O.world(sc)
    corners, tri_inst, _ = O.world_corners(sc)
    A = sc.inst_T.astype(np.float64).reshape(-1, 3, 4)[tri_inst]
    P = corners.astype(np.float64).reshape(-1, 3, 3)
    ref = np.einsum("nij,nkj->nki", A[:, :, :3], P) + A[:, None, :, 3]
    scale = np.einsum("nij,nkj->nki", np.abs(A[:, :, :3]), np.abs(P)) + np.abs(A[:, None, :, 3])
    err = np.abs(w.tris.reshape(-1, 3, 3) - ref)
    if np.any(err > 4 * 2.0 ** -24 * scale):
        fails.append(f"transform: error {np.max(err / scale)} x scale")
    # pure translations by representable values are exact
    Tt = sc.inst_T.copy()
    Tt[:, [0, 1, 2, 4, 5, 6, 8, 9, 10]] = [1, 0, 0, 0, 1, 0, 0, 0, 1]
    Tt[:, [3, 7, 11]] = np.round(Tt[:, [3, 7, 11]] * 4) / 4
    wt = O.world(sc, Tt)
    exp = corners.reshape(-1, 3, 3) + Tt[tri_inst][:, None, [3, 7, 11]]
    if not np.array_equal(wt.tris.reshape(-1, 3, 3), exp.astype(np.float32)):
        fails.append("transform: translation not exact")
    return fails


def pin_motion():
    """Constant-velocity motion: translation after s steps is c0 + v s dt up to
    FP32 rounding, and exactly c0 at s = 0."""
    fails = []
    sc = S.make_cfg4(n_envs=3, max_boxes=20)
    for s in (0, 1, 50, 99):
        T = O.moved_poses(sc, s)
        dyn = sc.inst_dynamic.astype(bool)
        ref = sc.inst_T[:, [3, 7, 11]].astype(float) + sc.inst_vel.astype(float) * (s * 0.01)
        err = np.abs(T[:, [3, 7, 11]] - ref)
        if np.any(err[dyn] > 1e-6 * (np.abs(ref[dyn]) + 1)):
            fails.append(f"motion: step {s} error {err.max()}")
        if not np.array_equal(T[~dyn], sc.inst_T[~dyn]):
            fails.append("motion: static instance moved")
        if not np.array_equal(T[:, [0, 1, 2, 4, 5, 6, 8, 9, 10]], sc.inst_T[:, [0, 1, 2, 4, 5, 6, 8, 9, 10]]):
            fails.append("motion: linear part changed")
    if not np.array_equal(O.moved_poses(sc, 0), sc.inst_T):
        fails.append("motion: step 0 differs")
    return fails


def pin_rays():
    """Ray generation: pinhole forward component is 1 in the sensor frame and
    the pixel grid is symmetric about the optical axis; LiDAR beams are unit
    length with the stated elevation and azimuth grid."""
    fails = []
    W, H = 32, 24
    cam = S.pinhole(W, H, 87.0)
    R = S.rot_zyx(0.4, 0.1, -0.2)
    sc = _ground_scene(cam, S.sensor_pose(R, (1.0, 2.0, 3.0)))
    o, d = O.sensor_rays(sc, 0)
    if not np.all(o == np.float32([1.0, 2.0, 3.0])):
        fails.append("rays: origin is not the pose translation")
    Rf = sc.sensor_T[0].reshape(3, 4)[:, :3].astype(float)
    local = d.astype(float) @ Rf  # R^T d (R orthonormal up to FP32 rounding)
    if np.any(np.abs(local[:, 0] - 1) > 1e-6):
        fails.append("rays: pinhole forward component != 1")
    f = (W / 2) / math.tan(float(F32(cam.hfov)) / 2)
    cols = np.arange(W * H) % W
    rows = np.arange(W * H) // W
    if np.any(np.abs(local[:, 1] + (cols + 0.5 - W / 2) / f) > 1e-6) or \
            np.any(np.abs(local[:, 2] + (rows + 0.5 - H / 2) / f) > 1e-6):
        fails.append("rays: pinhole pixel grid wrong")
    lid = S.lidar(16, 8, 90.0)
    sc = _ground_scene(lid, S.sensor_pose(np.eye(3), (0.0, 0.0, 1.0)))
    o, d = O.sensor_rays(sc, 0)
    d = d.astype(float)
    if np.any(np.abs(np.linalg.norm(d, axis=1) - 1) > 1e-6):
        fails.append("rays: lidar not unit")
    ch = np.arange(128) // 16
    az = np.arange(128) % 16
    el = np.arcsin(np.clip(d[:, 2], -1, 1))
    want_el = math.pi / 4 - ch * (math.pi / 2) / 7
    if np.any(np.abs(el - want_el) > 1e-5):
        fails.append("rays: lidar elevations wrong")
    a = np.arctan2(d[:, 1], d[:, 0])
    want_a = -math.pi + az * (2 * math.pi / 16)
    da = np.angle(np.exp(1j * (a - want_a)))
    if np.any(np.abs(da) > 1e-5):
        fails.append("rays: lidar azimuths wrong")
    return fails


def pin_table_rays(seed=0):
    """Direction-table sensors (user-defined projection models): each beam r
    travels along R table[r] from the pose's origin.  Inside an axis-aligned
    room (a scaled box whose corners are exact in FP32), the range of every
    beam is the FP64 slab exit distance along that direction; from a pose
    rotated about z only, over the ground plane, the range of a downward beam
    is h / (-table_z), because such a pose leaves the z component unchanged."""
    fails = []
    rng = np.random.default_rng(seed)
    W, H = 16, 12
    dirs = rng.normal(size=(W * H, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    dirs = dirs.astype(np.float32)
    sens = S.table_sensor(dirs, W, H, near=0.01, far=100.0)
    L = np.array([7.0, 4.0, 3.0])
    c = np.array([1.0, -2.0, 1.5])
    lo, hi = c - L / 2, c + L / 2
    room = S.affine(np.diag(L), c)
    p = np.array([1.75, -1.25, 0.875])
    for yaw, pitch, roll in ((0.3, 0.2, -0.1), (2.2, -0.4, 0.6), (0.0, 0.0, 0.0)):
        sc = S.custom_scene([S.box_mesh()], [([(0, 0, room, 0, (0, 0, 0))],
                                              [(0, S.sensor_pose(S.rot_zyx(yaw, pitch, roll), p))])], [sens])
        r = O.render(sc, nthreads=1)
        Rf = sc.sensor_T[0].reshape(3, 4)[:, :3].astype(np.float64)
        dw = dirs.astype(np.float64) @ Rf.T
        with np.errstate(divide="ignore"):
            t_axis = np.where(dw > 0, (hi - p) / dw, np.where(dw < 0, (lo - p) / dw, np.inf))
        t_exit = t_axis.min(1)
        if np.any(r.tri < 0):
            fails.append(f"table room: {np.sum(r.tri < 0)} beams escape a closed room")
            continue
        robust = (r.cls & O.BORDER_MASK) == 0
        if robust.sum() < 0.8 * len(dirs):
            fails.append("table room: too few robust beams")
        err = np.abs(r.t[robust] - t_exit[robust]) / t_exit[robust]
        if err.max() > 1e-5:
            fails.append(f"table room: yaw {yaw} max rel range err {err.max():.3g}")
    h = 1.5
    for yaw in (0.0, 1.1, -2.5):
        sc = _ground_scene(sens, S.sensor_pose(S.rot_zyx(yaw), (0.5, -0.75, h)))
        r = O.render(sc, nthreads=1)
        dz = dirs[:, 2].astype(np.float64)
        down = dz < -1e-3
        want = h / -dz[down]
        ok = want <= sens.far
        got = r.t[down][ok]
        if np.any(np.abs(got - want[ok]) > 1e-6 * want[ok]):
            fails.append(f"table ground: yaw {yaw} range differs from h / -d_z")
        if np.any(r.tri[~down & (dz > 1e-3)] != -1):
            fails.append(f"table ground: yaw {yaw} an upward beam hits the ground")
    return fails


# --------------------------------------------------------------------------
# 4. classification
# --------------------------------------------------------------------------
def pin_classifier():
    fails = []
    tri = np.array([0, 0, 2, 2, 0, 2, 0, 2, 2], np.float32)  # in z = 2
    cases = {
        "robust": ([0.5, 0.5, 0], [0, 0, 1], O.HIT),
        "edge": ([1.0, 0.0, 0], [0, 0, 1], O.HIT | O.B_BARY),
        "nearmiss": ([1.0, -1e-6, 0], [0, 0, 1], O.B_NEARMISS),
    }
    for name, (o, d, want) in cases.items():
        r = O.cast(_world_of([tri]), np.zeros(1, np.int32), np.float32([o]), np.float32([d]), 0.1, 10.0)
        if r["cls"][0] != want:
            fails.append(f"classifier {name}: {r['cls'][0]} want {want}")
    # two parallel triangles 1e-6 apart
    t2 = tri.copy()
    t2[[2, 5, 8]] += 2e-6
    r = O.cast(_world_of([tri, t2]), np.zeros(1, np.int32), np.float32([[0.5, 0.5, 0]]),
               np.float32([[0, 0, 1]]), 0.1, 10.0)
    if r["cls"][0] != O.HIT | O.B_GAP or r["tri"][0] != 0:
        fails.append(f"classifier gap: {r['cls'][0]}")
    # at the far limit and at the near limit (the triangle sits at t = 2)
    for near, far, lim in ((0.1, 2.0000001, "far"), (1.9999999, 10.0, "near")):
        r = O.cast(_world_of([tri]), np.zeros(1, np.int32), np.float32([[0.5, 0.5, 0]]),
                   np.float32([[0, 0, 1]]), near, far)
        if not r["cls"][0] & O.B_RANGE:
            fails.append(f"classifier range ({lim} limit)")
    # depth margin: the smallest of the relative gaps to the near limit, to the
    # far limit and to the next candidate, each known here in closed form
    for near, far, t2, want in ((1.8, 10.0, None, 0.1), (0.1, 2.2, None, 0.1),
                                (0.1, 10.0, 2.3, 0.15), (1.9, 2.3, 2.25, 0.05)):
        tris = [tri]
        if t2 is not None:
            second = tri.copy()
            second[[2, 5, 8]] = t2
            tris.append(second)
        r = O.cast(_world_of(tris), np.zeros(1, np.int32), np.float32([[0.5, 0.5, 0]]),
                   np.float32([[0, 0, 1]]), near, far)
        f32 = lambda x: float(np.float32(x))
        lim = [(2.0 - f32(near)) / 2.0, (f32(far) - 2.0) / 2.0]
        if t2 is not None:
            lim.append((f32(t2) - 2.0) / 2.0)
        if r["tri"][0] != 0 or abs(r["md"][0] - min(lim)) > 1e-12 or abs(min(lim) - want) > 1e-6:
            fails.append(f"classifier depth margin near {near} far {far}: {r['md'][0]} want {min(lim)}")
    # grazing incidence |cos| = 5e-4
    c = 5e-4
    d = np.float32([[math.sqrt(1 - c * c), 0, c]])
    big = np.array([-50, -50, 2, 50, -50, 2, 0, 50, 2], np.float32)
    r = O.cast(_world_of([big]), np.zeros(1, np.int32), np.float32([[0, 0, 1.99]]), d, 0.1, 100.0)
    if not r["cls"][0] & O.B_GRAZE:
        fails.append(f"classifier graze: {r['cls'][0]}")
    return fails


# --------------------------------------------------------------------------
# 6. further data types of a hit: normals, barycentrics, point clouds,
#    vertex ids
# --------------------------------------------------------------------------
def _rot(T):
    return np.asarray(T, np.float64).reshape(-1, 3, 4)


def pin_normals(seed=0):
    """cfg1 (ground + axis-aligned boxes): every robust hit's normal is the
    signed unit axis of the face it lies on, pointing back to the sensor: the
    ground seen from above gives +z exactly; a box face gives its outward axis
    (inward when the camera sits inside that box).  Also unit length,
    orthogonal to the triangle and facing the ray, on a rotated-object scene."""
    fails = []
    sc = S.make_cfg1(seed)
    w = O.world(sc)
    r = O.render(sc, w, nthreads=1)
    o, d = O.sensor_rays(sc, 0)
    rob = ((r.cls & O.BORDER_MASK) == 0) & (r.tri >= 0)
    if rob.sum() < 200:
        fails.append("normals: too few robust hits")
    owner = w.tri_inst[r.tri[rob]]
    hit = r.raw["hit"][rob]
    cam = o[0].astype(np.float64)
    want = np.zeros((rob.sum(), 3))
    for q, j in enumerate(owner):
        pts = w.tris[w.tri_inst == j].reshape(-1, 3).astype(np.float64)
        lo, hi = pts.min(0), pts.max(0)
        dist = np.r_[np.abs(hit[q] - lo), np.abs(hit[q] - hi)]
        k = int(np.argmin(dist))
        axis, sign = k % 3, (-1.0 if k < 3 else 1.0)
        if hi[axis] - lo[axis] == 0:  # flat quad (ground): facing the camera side
            sign = 1.0 if cam[axis] > lo[axis] else -1.0
        elif np.all((cam > lo) & (cam < hi)):
            sign = -sign
        want[q, axis] = sign
    if not np.array_equal(r.normal[rob].astype(np.float64), want):
        bad = np.nonzero(np.any(r.normal[rob] != want, axis=1))[0]
        fails.append(f"normals: {len(bad)} box/ground normals differ, e.g. {r.normal[rob][bad[0]]} vs {want[bad[0]]}")
    sc2 = S.make_cfg2(n_envs=1, W=64, H=36)
    w2 = O.world(sc2)
    r2 = O.render(sc2, w2)
    h = r2.tri >= 0
    n = r2.normal[h].astype(np.float64)
    T = w2.tris[r2.tri[h]].astype(np.float64)
    e1, e2 = T[:, 3:6] - T[:, :3], T[:, 6:] - T[:, :3]
    _, d2 = O.sensor_rays(sc2, 0)
    if not np.all(np.abs(np.linalg.norm(n, axis=1) - 1) <= 1e-6):  # NaN fails too
        fails.append("normals: not unit length")
    orth = np.abs(np.c_[(n * e1).sum(1) / np.linalg.norm(e1, axis=1), (n * e2).sum(1) / np.linalg.norm(e2, axis=1)])
    if not np.all(orth <= 1e-6):
        fails.append(f"normals: not orthogonal to the triangle ({np.nanmax(orth)})")
    if not np.all((n * d2[h]).sum(1) < 0):
        fails.append("normals: some face away from the sensor")
    if not (np.all(np.isnan(r2.normal[~h])) and np.all(np.isnan(r.normal[r.tri < 0]))):
        fails.append("normals: misses not NaN")
    return fails


def pin_barycentric():
    """The winner's (u, v) rebuild the hit point: (1-u-v) v0 + u v1 + v v2 =
    o + t d (FP64, rotated objects), and the reported FP32 pair is their
    rounding.  (Exact rational u, v on tiny scenes: ``pin_exact``.)"""
    fails = []
    sc = S.make_cfg2(n_envs=1, W=64, H=36)
    w = O.world(sc)
    r = O.render(sc, w)
    h = r.tri >= 0
    u, v = r.raw["u"][h], r.raw["v"][h]
    T = w.tris[r.tri[h]].astype(np.float64)
    a, b, c = T[:, :3], T[:, 3:6], T[:, 6:]
    p = (1 - u - v)[:, None] * a + u[:, None] * b + v[:, None] * c
    err = np.linalg.norm(p - r.raw["hit"][h], axis=1)
    scale = 1.0 + np.abs(r.raw["hit"][h]).max(1)
    if not np.all(err / scale <= 1e-9 / r.raw["g"][h].clip(1e-3).min()):
        fails.append(f"barycentric: rebuilt hit off by {(err / scale).max()}")
    if not np.array_equal(r.bary[h], np.c_[u, v].astype(np.float32)):
        fails.append("barycentric: reported pair is not the rounded (u, v)")
    if not np.all(np.isnan(r.bary[~h])):
        fails.append("barycentric: misses not NaN")
    return fails


def pin_point_cloud():
    """Sensor-frame points: for a pinhole the forward coordinate is the depth
    itself (local forward component 1); mapped back through the sensor pose
    (R p + o) they are the world hit points; for a LiDAR their length is the
    range."""
    fails = []
    for sc in (S.make_cfg2(n_envs=1, W=64, H=36), S.make_cfg3(n_envs=1, azimuths=64, channels=8)):
        w = O.world(sc)
        r = O.render(sc, w)
        h = r.tri >= 0
        P = _rot(sc.sensor_T)[0]
        world = r.point[h].astype(np.float64) @ P[:, :3].T + P[:, 3]
        err = np.linalg.norm(world - r.raw["hit"][h], axis=1) / np.maximum(r.t[h], 1.0)
        if not np.all(err <= 1e-6):
            fails.append(f"point cloud: R p + o off the hit by {np.nanmax(err)} (relative)")
        if sc.sensors[0].kind == 0 and not np.array_equal(r.point[h][:, 0], r.depth[h]):
            fails.append("point cloud: pinhole forward coordinate != depth")
        if sc.sensors[0].kind == 1:
            rel = np.abs(np.linalg.norm(r.point[h].astype(np.float64), axis=1) - r.t[h]) / r.t[h]
            if not np.all(rel <= 1e-6):
                fails.append(f"point cloud: lidar |p| != range ({rel.max()})")
        if not np.all(np.isnan(r.point[~h])):
            fails.append("point cloud: misses not NaN")
    return fails


def pin_vertex_ids():
    """The reported global vertex ids, looked up in the prototype vertex lists
    and moved by the owning instance's pose, are the winner's world vertices."""
    fails = []
    sc = S.make_cfg2(n_envs=1, W=64, H=36)
    w = O.world(sc)
    r = O.render(sc, w)
    h = r.tri >= 0
    allv = np.concatenate([np.asarray(v, np.float64) for v, _ in sc.protos])
    A = _rot(sc.inst_T)[w.tri_inst[r.tri[h]]]
    for k in range(3):
        pv = allv[r.vert[h][:, k]]
        moved = np.einsum("nij,nj->ni", A[:, :, :3], pv) + A[:, :, 3]
        err = np.abs(moved - w.tris[r.tri[h]][:, 3 * k:3 * k + 3])
        if not np.all(err <= 1e-5):
            fails.append(f"vertex ids: corner {k} off by {err}")
    if not np.all(r.vert[~h] == -1):
        fails.append("vertex ids: misses not -1")
    return fails


# --------------------------------------------------------------------------
# 7. stereo shadows
# --------------------------------------------------------------------------
SHADOW_S0 = 2.0 ** -13


def _pillar_scene(baseline=(0.0, -0.3, 0.0)):
    """Floor + one floating pillar, a pitched camera whose second camera sits
    `baseline` away in its own frame."""
    desc = S.pinhole(96, 54, 87.0, 0.05, 30.0)
    desc = S.SensorDesc(**{**desc.__dict__, "stereo": tuple(float(x) for x in baseline)})
    floor = (0, 0, S.affine(np.diag([40.0, 40.0, 1.0]), (-20.0, -20.0, 0.0)), 0, (0, 0, 0))
    pillar = (1, 1, S.affine(np.diag([0.3, 0.3, 1.9]), (3.15, 0.35, 1.0)), 0, (0, 0, 0))
    pose = S.sensor_pose(S.rot_zyx(0.05, 20 * S.DEG), (0.0, 0.0, 1.5))
    return S.custom_scene([S.quad_mesh(), S.box_mesh()], [([floor, pillar], [(0, pose)])], [desc])


def pin_stereo_pillar():
    """Closed form: a hit point is hidden from the second camera iff the
    segment from it to that camera crosses the pillar's surface at a
    parameter in [S0, 1]; the crossings are the FP64 slab entry and exit of
    the pillar box (the floor cannot be crossed: both ends lie above it)."""
    fails = []
    sc = _pillar_scene()
    w = O.world(sc)
    r = O.render(sc, w, nthreads=1)
    h = r.tri >= 0
    P = _rot(sc.sensor_T)[0]
    c2 = P[:, :3] @ np.array(sc.sensors[0].stereo, np.float64) + P[:, 3]
    pts = w.tris[w.tri_inst == 1].reshape(-1, 3).astype(np.float64)
    lo, hi = pts.min(0), pts.max(0)
    p = r.hit[h].astype(np.float64)
    D = c2[None, :] - p
    tmin, tmax = _slab(lo, hi, p, D)
    cross = (tmin <= tmax) & (((tmin >= SHADOW_S0) & (tmin <= 1)) | ((tmax >= SHADOW_S0) & (tmax <= 1)))
    # decisions within the classifier's margins of an edge, S0 or the camera are not compared
    rob = ((r.cls[h] & O.BORDER_MASK) == 0) & ((r.shadow_cls[h] & 2) == 0)
    bad = rob & (cross != (r.shadow[h] == 1))
    if bad.any():
        fails.append(f"stereo pillar: {bad.sum()} robust pixels disagree with the slab closed form")
    if cross[rob].sum() < 20 or (~cross[rob]).sum() < 20:
        fails.append(f"stereo pillar: degenerate case ({cross[rob].sum()} shadowed)")
    if np.any(r.shadow[~h] != 0):
        fails.append("stereo pillar: shadow set on a miss")
    return fails


def pin_stereo_zero_baseline():
    """With the second camera at the first one's centre, the segment from a
    hit back to the camera is the primary ray itself: nothing can lie on it
    (the camera is clear of every object by more than the near distance), so
    no pixel is shadowed."""
    sc = S.make_cfg2(n_envs=2, W=64, H=36)
    desc = S.SensorDesc(**{**sc.sensors[0].__dict__, "near": 0.01})
    sc = S.Scene(**{**sc.__dict__, "sensors": [desc]})
    w = O.world(sc)
    r = O.render(sc, w)
    h = np.nonzero(r.tri >= 0)[0]
    senv = np.repeat(O.sensor_env(sc), sc.rays_per_sensor_inst())
    si = np.repeat(np.arange(len(sc.sensor_ids)), sc.rays_per_sensor_inst())
    occ = np.zeros(len(h), np.uint8)
    cls = np.zeros(len(h), np.int32)
    O.lib().orc_shadow(np.ascontiguousarray(w.tris), np.ascontiguousarray(w.env_off), len(h),
                       np.ascontiguousarray(senv[h], np.int32), np.ascontiguousarray(r.tri[h], np.int32),
                       np.ascontiguousarray(r.hit[h]), np.ascontiguousarray(np.asarray(sc.sensor_T, np.float32)[si[h]]),
                       np.zeros((len(h), 3), np.float32), 1, occ, cls)
    return [f"stereo zero baseline: {int(occ.sum())} pixels shadowed"] if occ.any() else []


def pin_stereo_exact(seeds=range(40)):
    """Exact rational segment tests on the tiny scenes: the segment from the hit
    point to a second camera at o + b (identity rotation, so the centre is
    o + b rounded once; b alternates between a short baseline and two that
    bring the second camera down among the triangles), occluded iff some
    triangle meets it at an exact s in [S0, 1]."""
    fails = []
    from fractions import Fraction as Fr
    s0 = Fr(SHADOW_S0)
    n_cmp = {False: 0, True: 0}
    for seed in seeds:
        tris, o, d = tiny_scene(seed)
        wd = _world_of(tris)
        r = O.cast(wd, np.zeros(len(o), np.int32), o, d, 0.05, 50.0, nthreads=1)
        h = np.nonzero(r["tri"] >= 0)[0]
        if not len(h):
            continue
        b = np.array([(0.0, 0.3, 0.1), (1.5, -1.2, -2.0), (-2.0, 1.0, -2.2)][seed % 3], np.float32)
        pose = np.zeros((len(h), 12), np.float32)
        pose[:, [0, 5, 10]] = 1.0
        pose[:, [3, 7, 11]] = o[h]
        p = r["hit"][h].astype(np.float32)
        occ = np.zeros(len(h), np.uint8)
        cls = np.zeros(len(h), np.int32)
        O.lib().orc_shadow(np.ascontiguousarray(wd.tris), wd.env_off, len(h), np.zeros(len(h), np.int32),
                           np.ascontiguousarray(r["tri"][h], np.int32), np.ascontiguousarray(p), pose,
                           np.tile(b, (len(h), 1)), 1, occ, cls)
        for q, i in enumerate(h):
            c2 = (o[i].astype(np.float64) + b.astype(np.float64)).astype(np.float32)
            D = c2 - p[q]
            want, margin = False, math.inf
            for tri in tris:
                res = exact.intersect(tri, p[q], D)
                if res is None:
                    continue
                t, u, v = res
                margin = min(margin, float(abs(t - s0)), float(abs(t - 1)), float(abs(min(u, v, 1 - u - v))))
                if u >= 0 and v >= 0 and u + v <= 1 and s0 <= t <= 1:
                    want = True
            if margin > 1e-12:
                n_cmp[want] += 1
                if bool(occ[q]) != want:
                    fails.append(f"stereo exact seed {seed} ray {i}: oracle {occ[q]} exact {want}")
    if min(n_cmp.values()) < 20:
        fails.append(f"stereo exact: too few decided cases {n_cmp}")
    return fails


# --------------------------------------------------------------------------
# 8. FP64 world vertices (the composition a renderer intersecting in each
#    sub-mesh's own frame computes)
# --------------------------------------------------------------------------
def pin_world64(seeds=range(0, 200, 5)):
    """orc_transform64 against exact rational evaluation of A[:, :3] v + A[:, 3]
    (rounded once to FP64, so within a few FP64 ulps of the scale); orc_cast64
    on FP32-representable vertices reproduces orc_cast bit for bit; and on
    tiny scenes whose vertices are not FP32 numbers it picks the exact
    rational winner with t to FP64 accuracy."""
    from fractions import Fraction as Fr
    fails = []
    sc = S.make_cfg2(n_envs=2, W=16, H=9)
    w64 = O.world64(sc)
    corners, tri_inst, _ = O.world_corners(sc)
    rng = np.random.default_rng(3)
    for k in rng.choice(len(corners), 300, replace=False):
        A = sc.inst_T[tri_inst[k]].astype(np.float64).reshape(3, 4)
        for c in range(3):
            v = corners[k, 3 * c:3 * c + 3].astype(np.float64)
            for r in range(3):
                ex = sum((Fr(A[r, j]) * Fr(v[j]) for j in range(3)), Fr(A[r, 3]))
                scale = float(sum(abs(A[r, j] * v[j]) for j in range(3)) + abs(A[r, 3]))
                if abs(w64.tris[k, 3 * c + r] - float(ex)) > 4 * 2.0 ** -53 * scale:
                    fails.append(f"world64: triangle {k} corner {c} row {r}: {w64.tris[k, 3 * c + r]} "
                                 f"exact {float(ex)}")
    if fails:
        return fails[:5]
    # the same search on FP64 copies of FP32 vertices is the FP32 search
    sc1 = S.make_cfg1()
    w = O.world(sc1)
    w64 = O.World(w.tris.astype(np.float64), w.env_off, w.tri_inst, w.tri_seg)
    o, d = O.sensor_rays(sc1, 0)
    n = len(o)
    env = np.zeros(n, np.int32)
    a = O.cast(w, env, o, d, 0.2, 10.0, nthreads=1)
    b = O.cast(w64, env, o, d, 0.2, 10.0, nthreads=1)
    for key in ("t", "tri", "u", "v", "hit", "mb", "md", "g", "cls"):
        if not np.array_equal(a[key], b[key], equal_nan=True):
            fails.append(f"cast64: {key} differs from the FP32 search on FP32 vertices")
    # exact rationals on vertices off the FP32 grid
    near, far = 0.05, 50.0
    for seed in seeds:
        tris, o, d = tiny_scene(seed)
        g = np.random.default_rng(1000 + seed)
        t64 = tris.astype(np.float64) * (1.0 + g.uniform(-1e-6, 1e-6, tris.shape)) + g.uniform(-1e-7, 1e-7, tris.shape)
        wt = O.World(np.ascontiguousarray(t64), np.array([0, len(t64)], np.int64), np.zeros(len(t64), np.int32),
                     np.zeros(len(t64), np.int32))
        r = O.cast(wt, np.zeros(len(o), np.int32), o, d, near, far, nthreads=1)
        for i in range(len(o)):
            k, t, u, v, m = exact.nearest(list(t64), o[i], d[i], near, far)
            if m <= 1e-12:
                continue
            if r["tri"][i] != k:
                fails.append(f"cast64 exact seed {seed} ray {i}: oracle tri {r['tri'][i]} exact {k}")
            elif k >= 0 and abs(r["t"][i] - float(t)) > _t_tol(t64[k], o[i], d[i], float(t)):
                fails.append(f"cast64 exact seed {seed} ray {i}: t {r['t'][i]} exact {float(t)}")
    return fails


ALL_PINS = [pin_exact, pin_duplicate_tie, pin_ray_plane, pin_boxes, pin_tessellated,
            pin_invariants, pin_transform, pin_motion, pin_rays, pin_table_rays, pin_classifier,
            pin_normals, pin_barycentric, pin_point_cloud, pin_vertex_ids,
            pin_stereo_pillar, pin_stereo_zero_baseline, pin_stereo_exact, pin_world64]
