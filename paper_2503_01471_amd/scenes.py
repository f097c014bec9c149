"""Seeded synthetic scenes and sensors: the inputs of the ray-cast renderer.

This module only *constructs inputs*; it performs none of the renderer's
arithmetic (no vertex transform, no ray generation, no intersection).  The GPU
library and the CPU oracle both consume what it returns and nothing else is
shared between them.

Scene model (paper, Sec. III-D "Exteroceptive Sensors"): environment E_i holds a
base mesh made of n_i sub-meshes, one per object, each with its own transform
T_{j,t}.  Here a sub-mesh is an *instance*: a shared prototype mesh, a 3x4
row-major affine pose (v_world = A[:, :3] v + A[:, 3]), a segmentation label and
a dynamic flag.  Sensors are pinhole cameras and rotating LiDARs mounted per
environment with a 3x4 pose whose rotation columns are the sensor axes
(x forward, y left, z up) and whose last column is the sensor origin.

Every environment is generated from its own ``SeedSequence([seed, cfg, env])``
so any subsample of environments regenerates bit-identically.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

PINHOLE, LIDAR, TABLE = 0, 1, 2

DEG = math.pi / 180.0


# --------------------------------------------------------------------------
# data containers
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class SensorDesc:
    """Sensor model.  ``width``/``height`` are W/H for pinholes and
    azimuths/channels for LiDARs; angles in radians; ``near``/``far`` bound the
    measured quantity (depth for pinholes, range for LiDARs).  ``stereo`` is
    the centre of a stereo pair's second camera in this sensor's frame
    (metres; all zero: no second camera)."""

    kind: int
    width: int
    height: int
    hfov: float = 0.0
    vmin: float = 0.0
    vmax: float = 0.0
    hmin: float = 0.0
    hmax: float = 0.0
    near: float = 0.0
    far: float = 0.0
    dir_table: Optional[np.ndarray] = field(default=None, compare=False, hash=False)
    stereo: Tuple[float, float, float] = (0.0, 0.0, 0.0)

    @property
    def n_rays(self) -> int:
        return int(self.width) * int(self.height)


@dataclass
class Scene:
    protos: List[Tuple[np.ndarray, np.ndarray]]  # (verts float32 [nv,3], tris int32 [nt,3])
    inst_offsets: np.ndarray  # int64 [E+1]
    inst_mesh: np.ndarray  # int32 [I]
    inst_seg: np.ndarray  # int32 [I]
    inst_dynamic: np.ndarray  # uint8 [I]
    inst_T: np.ndarray  # float32 [I,12] row-major 3x4
    sensors: List[SensorDesc]
    sens_offsets: np.ndarray  # int64 [E+1]
    sensor_ids: np.ndarray  # int32 [S]
    sensor_T: np.ndarray  # float32 [S,12]
    inst_vel: np.ndarray  # float32 [I,3] (zero for static instances)
    dt: float = 0.01
    name: str = ""

    @property
    def n_envs(self) -> int:
        return len(self.inst_offsets) - 1

    @property
    def n_inst(self) -> int:
        return len(self.inst_mesh)

    def proto_tri_counts(self) -> np.ndarray:
        return np.array([len(t) for _, t in self.protos], dtype=np.int64)

    def env_tri_counts(self) -> np.ndarray:
        per_inst = self.proto_tri_counts()[self.inst_mesh]
        cs = np.concatenate([[0], np.cumsum(per_inst)])
        return cs[self.inst_offsets[1:]] - cs[self.inst_offsets[:-1]]

    def rays_per_sensor_inst(self) -> np.ndarray:
        return np.array([self.sensors[s].n_rays for s in self.sensor_ids], dtype=np.int64)

    def total_rays(self) -> int:
        return int(self.rays_per_sensor_inst().sum())


# --------------------------------------------------------------------------
# prototype meshes (outward CCW winding; triangles are two-sided anyway)
# --------------------------------------------------------------------------
def quad_mesh():
    """Unit square [0,1]^2 at z=0, normal +z (2 triangles)."""
    v = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0]], np.float32)
    t = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    return v, t


def box_mesh():
    """Unit cube [-0.5,0.5]^3, 12 triangles."""
    v = np.array([[x, y, z] for z in (-0.5, 0.5) for y in (-0.5, 0.5) for x in (-0.5, 0.5)],
                 np.float32)
    # vertex index = 4*zi + 2*yi + xi
    faces = [
        (0, 2, 3, 1),  # z-
        (4, 5, 7, 6),  # z+
        (0, 1, 5, 4),  # y-
        (2, 6, 7, 3),  # y+
        (0, 4, 6, 2),  # x-
        (1, 3, 7, 5),  # x+
    ]
    t = []
    for a, b, c, d in faces:
        t += [[a, b, c], [a, c, d]]
    return v, np.array(t, np.int32)


def cylinder_mesh(n: int):
    """Radius-1 cylinder, z in [0,1], n side segments, centre-fan caps (4n tris)."""
    ang = 2.0 * np.pi * np.arange(n) / n
    ring = np.stack([np.cos(ang), np.sin(ang)], 1)
    v = np.concatenate([
        np.c_[ring, np.zeros(n)],  # 0..n-1 bottom ring
        np.c_[ring, np.ones(n)],  # n..2n-1 top ring
        [[0, 0, 0], [0, 0, 1]],  # 2n bottom centre, 2n+1 top centre
    ]).astype(np.float32)
    t = []
    for i in range(n):
        j = (i + 1) % n
        t += [[i, j, n + j], [i, n + j, n + i]]  # side
        t += [[2 * n, j, i]]  # bottom cap (normal -z)
        t += [[2 * n + 1, n + i, n + j]]  # top cap (normal +z)
    return v, np.array(t, np.int32)


def cone_mesh(n: int):
    """Base radius 1 at z=0, apex (0,0,1), n segments, centre-fan base cap (2n tris)."""
    ang = 2.0 * np.pi * np.arange(n) / n
    v = np.concatenate([
        np.c_[np.cos(ang), np.sin(ang), np.zeros(n)],
        [[0, 0, 1], [0, 0, 0]],  # n apex, n+1 base centre
    ]).astype(np.float32)
    t = []
    for i in range(n):
        j = (i + 1) % n
        t += [[i, j, n]]
        t += [[n + 1, j, i]]
    return v, np.array(t, np.int32)


def icosphere_mesh(level: int):
    """Unit icosphere: icosahedron subdivided ``level`` times (20*4^level tris)."""
    p = (1.0 + 5.0 ** 0.5) / 2.0
    verts = [(-1, p, 0), (1, p, 0), (-1, -p, 0), (1, -p, 0), (0, -1, p), (0, 1, p),
             (0, -1, -p), (0, 1, -p), (p, 0, -1), (p, 0, 1), (-p, 0, -1), (-p, 0, 1)]
    verts = [np.array(v, float) / np.linalg.norm(v) for v in verts]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
             (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
             (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    return np.array(verts, np.float32), np.array(faces, np.int32)


# --------------------------------------------------------------------------
# pose helpers (input construction, float64 then stored as float32)
# --------------------------------------------------------------------------
def rot_zyx(yaw: float, pitch: float = 0.0, roll: float = 0.0) -> np.ndarray:
    cy, sy = math.cos(yaw), math.sin(yaw)
    cp, sp = math.cos(pitch), math.sin(pitch)
    cr, sr = math.cos(roll), math.sin(roll)
    rz = np.array([[cy, -sy, 0], [sy, cy, 0], [0, 0, 1]])
    ry = np.array([[cp, 0, sp], [0, 1, 0], [-sp, 0, cp]])
    rx = np.array([[1, 0, 0], [0, cr, -sr], [0, sr, cr]])
    return rz @ ry @ rx


def rot_uniform(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation (Shoemake's quaternion method)."""
    u1, u2, u3 = rng.random(3)
    a, b = math.sqrt(1.0 - u1), math.sqrt(u1)
    x, y = a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2)
    z, w = b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def affine(lin: np.ndarray, t: Sequence[float]) -> np.ndarray:
    """3x4 row-major affine [lin | t] flattened to 12 float32 values."""
    a = np.zeros((3, 4))
    a[:, :3] = lin
    a[:, 3] = t
    return a.astype(np.float32).reshape(12)


def sensor_pose(R: np.ndarray, origin: Sequence[float]) -> np.ndarray:
    return affine(R, origin)


# --------------------------------------------------------------------------
# sensor models used by the workloads
# --------------------------------------------------------------------------
def pinhole(W: int, H: int, hfov_deg: float = 87.0, near: float = 0.2, far: float = 10.0):
    return SensorDesc(PINHOLE, W, H, hfov=hfov_deg * DEG, near=near, far=far)


def lidar(azimuths: int, channels: int, vfov_deg: float = 90.0, near: float = 0.5,
          far: float = 30.0):
    return SensorDesc(LIDAR, azimuths, channels, vmin=-0.5 * vfov_deg * DEG,
                      vmax=0.5 * vfov_deg * DEG, hmin=-math.pi, hmax=math.pi,
                      near=near, far=far)


def table_sensor(dirs: np.ndarray, width: int, height: int, near: float, far: float):
    d = np.ascontiguousarray(dirs, np.float32).reshape(width * height, 3)
    return SensorDesc(TABLE, width, height, near=near, far=far, dir_table=d)


# --------------------------------------------------------------------------
# builders
# --------------------------------------------------------------------------
class _Builder:
    def __init__(self, protos, sensors, name):
        self.protos = protos
        self.sensors = sensors
        self.name = name
        self.inst_counts, self.mesh, self.seg, self.dyn, self.T, self.vel = [], [], [], [], [], []
        self.sens_counts, self.sid, self.sT = [], [], []

    def env(self, insts, sens):
        """insts: list of (mesh, seg, T12, dynamic, vel3); sens: list of (sensor id, T12)."""
        self.inst_counts.append(len(insts))
        for m, s, T, d, v in insts:
            self.mesh.append(m)
            self.seg.append(s)
            self.T.append(T)
            self.dyn.append(d)
            self.vel.append(v)
        self.sens_counts.append(len(sens))
        for s, T in sens:
            self.sid.append(s)
            self.sT.append(T)

    def done(self, dt=0.01) -> Scene:
        io = np.concatenate([[0], np.cumsum(self.inst_counts)]).astype(np.int64)
        so = np.concatenate([[0], np.cumsum(self.sens_counts)]).astype(np.int64)
        return Scene(
            protos=self.protos,
            inst_offsets=io,
            inst_mesh=np.array(self.mesh, np.int32),
            inst_seg=np.array(self.seg, np.int32),
            inst_dynamic=np.array(self.dyn, np.uint8),
            inst_T=np.array(self.T, np.float32).reshape(-1, 12),
            sensors=self.sensors,
            sens_offsets=so,
            sensor_ids=np.array(self.sid, np.int32),
            sensor_T=np.array(self.sT, np.float32).reshape(-1, 12),
            inst_vel=np.array(self.vel, np.float32).reshape(-1, 3),
            dt=dt,
            name=self.name,
        )


_ZERO3 = (0.0, 0.0, 0.0)


def env_rng(seed: int, cfg: int, env: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([seed, cfg, env]))


def _env_ids(n_envs, env_ids):
    return list(range(n_envs)) if env_ids is None else [int(e) for e in env_ids]


def _clear_position(rng, lo, hi, centres, radii, clearance, tries=2000):
    """Uniform position in the box [lo,hi] clear of every bounding sphere by
    ``clearance``; if none of ``tries`` samples is clear, the best one."""
    best, best_gap = None, -np.inf
    for _ in range(tries):
        p = lo + (hi - lo) * rng.random(3)
        if len(centres) == 0:
            return p
        gap = float(np.min(np.linalg.norm(centres - p, axis=1) - radii))
        if gap >= clearance:
            return p
        if gap > best_gap:
            best, best_gap = p, gap
    return best


def make_cfg1(seed: int = 0) -> Scene:
    """Small scene: ground quad [0,10]^2 + 8 axis-aligned boxes (sides U[0.2,1.5] m,
    centres U in 10x10x4 m); one 64x48 87-degree camera at (5,5,2), random yaw."""
    b = _Builder([quad_mesh(), box_mesh()], [pinhole(64, 48)], "cfg1")
    rng = env_rng(seed, 1, 0)
    insts = [(0, 0, affine(np.diag([10.0, 10.0, 1.0]), _ZERO3), 0, _ZERO3)]
    for k in range(8):
        s = rng.uniform(0.2, 1.5, 3)
        c = rng.random(3) * np.array([10.0, 10.0, 4.0])
        insts.append((1, k + 1, affine(np.diag(s), c), 0, _ZERO3))
    yaw = rng.uniform(0.0, 2 * math.pi)
    b.env(insts, [(0, sensor_pose(rot_zyx(yaw), (5.0, 5.0, 2.0)))])
    return b.done()


def make_cfg2(n_envs: int = 1024, seed: int = 0, env_ids=None, W: int = 480, H: int = 270) -> Scene:
    """Room 10x10x5 m (6 wall quads as one 12-tri instance, seg 0) with 40 random
    obstacles from {box, 16-gon cylinder, level-2 icosphere}, random 3-D rotation;
    one 480x270 87-degree camera per env in free space."""
    protos = [box_mesh(), cylinder_mesh(16), icosphere_mesh(2)]
    b = _Builder(protos, [pinhole(W, H)], "cfg2")
    room = np.array([10.0, 10.0, 5.0])
    for e in _env_ids(n_envs, env_ids):
        rng = env_rng(seed, 2, e)
        insts = [(0, 0, affine(np.diag(room), room / 2), 0, _ZERO3)]
        centres, radii = [], []
        for k in range(40):
            kind = int(rng.integers(0, 3))
            R = rot_uniform(rng)
            c = rng.random(3) * room
            if kind == 0:
                s = rng.uniform(0.2, 2.0, 3)
                insts.append((0, k + 1, affine(R @ np.diag(s), c), 0, _ZERO3))
                rad = 0.5 * float(np.linalg.norm(s))
            elif kind == 1:
                D, Hc = rng.uniform(0.2, 2.0, 2)
                lin = R @ np.diag([D / 2, D / 2, Hc])
                insts.append((1, k + 1, affine(lin, c - 0.5 * Hc * R[:, 2]), 0, _ZERO3))
                rad = math.hypot(D / 2, Hc / 2)
            else:
                D = rng.uniform(0.2, 2.0)
                insts.append((2, k + 1, affine(R * (D / 2), c), 0, _ZERO3))
                rad = D / 2
            centres.append(c)
            radii.append(rad)
        p = _clear_position(rng, np.array([0.5, 0.5, 0.5]), np.array([9.5, 9.5, 4.5]),
                            np.array(centres), np.array(radii), 0.2)
        yaw = rng.uniform(0.0, 2 * math.pi)
        pitch = rng.uniform(-15.0, 15.0) * DEG
        b.env(insts, [(0, sensor_pose(rot_zyx(yaw, pitch), p))])
    return b.done()


def make_cfg3(n_envs: int = 4096, seed: int = 0, env_ids=None, azimuths: int = 512,
              channels: int = 64) -> Scene:
    """Forest: ground [-20,20]^2 + 60 trees (8-gon capped trunk + 24-gon capped cone
    canopy sharing the tree's label); one 64x512 360x90-degree LiDAR per env."""
    protos = [quad_mesh(), cylinder_mesh(8), cone_mesh(24)]
    b = _Builder(protos, [lidar(azimuths, channels)], "cfg3")
    for e in _env_ids(n_envs, env_ids):
        rng = env_rng(seed, 3, e)
        insts = [(0, 0, affine(np.diag([40.0, 40.0, 1.0]), (-20.0, -20.0, 0.0)), 0, _ZERO3)]
        cs, rs = np.zeros((0, 2)), np.zeros(0)
        for k in range(60):
            while True:
                c = rng.uniform(-19.0, 19.0, 2)
                r = rng.uniform(0.1, 0.4)
                if len(rs) == 0 or np.all(np.linalg.norm(cs - c, axis=1) >= rs + r + 0.2):
                    break
            cs = np.vstack([cs, c])
            rs = np.append(rs, r)
            h = rng.uniform(3.0, 8.0)
            rc = rng.uniform(1.0, 2.5)
            insts.append((1, k + 1, affine(np.diag([r, r, h]), (c[0], c[1], 0.0)), 0, _ZERO3))
            ch = h + 1.5 - 0.5 * h
            insts.append((2, k + 1, affine(np.diag([rc, rc, ch]), (c[0], c[1], 0.5 * h)), 0,
                          _ZERO3))
        while True:
            p = rng.uniform(-15.0, 15.0, 2)
            if np.all(np.linalg.norm(cs - p, axis=1) >= rs + 0.3):
                break
        z = rng.uniform(0.5, 2.0)
        yaw = rng.uniform(0.0, 2 * math.pi)
        b.env(insts, [(0, sensor_pose(rot_zyx(yaw), (p[0], p[1], z)))])
    return b.done()


CFG4_SENSORS = [pinhole(480, 270), pinhole(240, 135), lidar(512, 32)]


def make_cfg4(n_envs: int = 2048, seed: int = 0, env_ids=None, max_boxes: int = 200) -> Scene:
    """Uneven batch: per env U{5..max_boxes} axis-aligned boxes (sides U[0.2,1.5] m,
    centres U in 10x10x4 m), 30% moving with v ~ U[-1,1]^3 m/s, plus the ground
    quad; one sensor per env drawn from {480x270 camera, 240x135 camera,
    32x512 LiDAR}, placed in free space with yaw/pitch as in the room scenes."""
    b = _Builder([quad_mesh(), box_mesh()], list(CFG4_SENSORS), "cfg4")
    room = np.array([10.0, 10.0, 4.0])
    for e in _env_ids(n_envs, env_ids):
        rng = env_rng(seed, 4, e)
        k = int(rng.integers(5, max_boxes + 1))
        insts = [(0, 0, affine(np.diag([10.0, 10.0, 1.0]), _ZERO3), 0, _ZERO3)]
        centres, radii = [], []
        for j in range(k):
            s = rng.uniform(0.2, 1.5, 3)
            c = rng.random(3) * room
            moving = bool(rng.random() < 0.3)
            v = tuple(rng.uniform(-1.0, 1.0, 3)) if moving else _ZERO3
            insts.append((1, j + 1, affine(np.diag(s), c), int(moving), v))
            centres.append(c)
            radii.append(0.5 * float(np.linalg.norm(s)))
        sid = int(rng.integers(0, 3))
        p = _clear_position(rng, np.array([0.5, 0.5, 0.5]), np.array([9.5, 9.5, 3.5]),
                            np.array(centres), np.array(radii), 0.2)
        yaw = rng.uniform(0.0, 2 * math.pi)
        pitch = rng.uniform(-15.0, 15.0) * DEG
        b.env(insts, [(sid, sensor_pose(rot_zyx(yaw, pitch), p))])
    return b.done()


def subset(scene: Scene, env_ids: Sequence[int]) -> Scene:
    """Environments ``env_ids`` of ``scene`` (in the given order) as a new scene."""
    io, so = scene.inst_offsets, scene.sens_offsets
    ii = np.concatenate([np.arange(io[e], io[e + 1]) for e in env_ids]).astype(np.int64)
    si = np.concatenate([np.arange(so[e], so[e + 1]) for e in env_ids]).astype(np.int64)
    ic = np.array([io[e + 1] - io[e] for e in env_ids], np.int64)
    sc = np.array([so[e + 1] - so[e] for e in env_ids], np.int64)
    return Scene(
        protos=scene.protos,
        inst_offsets=np.concatenate([[0], np.cumsum(ic)]).astype(np.int64),
        inst_mesh=scene.inst_mesh[ii], inst_seg=scene.inst_seg[ii],
        inst_dynamic=scene.inst_dynamic[ii], inst_T=scene.inst_T[ii],
        sensors=scene.sensors,
        sens_offsets=np.concatenate([[0], np.cumsum(sc)]).astype(np.int64),
        sensor_ids=scene.sensor_ids[si], sensor_T=scene.sensor_T[si],
        inst_vel=scene.inst_vel[ii], dt=scene.dt, name=scene.name + "-subset")


def make(cfg: int, n_envs: Optional[int] = None, seed: int = 0, env_ids=None) -> Scene:
    if cfg == 1:
        return make_cfg1(seed)
    fn = {2: make_cfg2, 3: make_cfg3, 4: make_cfg4}[cfg]
    kw = {} if n_envs is None else {"n_envs": n_envs}
    return fn(seed=seed, env_ids=env_ids, **kw)


def custom_scene(protos, envs, sensors, dt: float = 0.01, name: str = "custom") -> Scene:
    """Scene from explicit parts.  ``envs`` is a list of (insts, sens) with
    insts = [(mesh, seg, T12, dynamic, vel3)] and sens = [(sensor id, T12)]."""
    b = _Builder(list(protos), list(sensors), name)
    for insts, sens in envs:
        b.env(insts, sens)
    return b.done(dt)
