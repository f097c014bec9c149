"""Python binding of the renderer's C ABI (``include/rc.h``).

Argument marshalling only: every function forwards to the ``rc_*`` entry point
of the same name in ``librc.so``; every step of the rendering path runs in the
library's HIP kernels.  Device buffers are torch tensors on a HIP device
(their ``data_ptr()`` is passed), host arrays are numpy arrays.  Loading fails
loudly if the library has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librc.so")

RC_PINHOLE, RC_LIDAR, RC_TABLE = 0, 1, 2
RC_BUILD_SAH = 0
RC_BUILD_LBVH = 1
RC_BUILD_TWO_LEVEL = 2
RC_SCENE_TWO_LEVEL_ONLY = 1
RC_RENDER_PLAIN, RC_RENDER_FLAT, RC_RENDER_BATCHED, RC_RENDER_BRUTE = 0, 1, 2, 3

# Every function declared in include/rc.h.
ABI = [
    "rc_status_string", "rc_last_error", "rc_create", "rc_destroy", "rc_memory_used", "rc_mesh_add",
    "rc_scene_load", "rc_scene_options", "rc_sensor_add", "rc_sensors_attach", "rc_ray_layout", "rc_env_tri_offsets",
    "rc_set_instance_poses", "rc_set_sensor_poses", "rc_move_instances", "rc_build", "rc_refit", "rc_render",
    "rc_render_noalloc", "rc_render_stats", "rc_debug_world", "rc_debug_rays", "rc_debug_bvh", "rc_autotune", "rc_tuning_set", "rc_step_graph_create",
    "rc_graph_set_step", "rc_graph_launch", "rc_graph_destroy", "rc_server_create", "rc_server_submit",
    "rc_server_poll", "rc_server_wait", "rc_server_outputs", "rc_server_release", "rc_server_destroy",
]
RC_SERVE_PLAIN, RC_SERVE_BATCHED = 0, 1
RC_OUT_DEPTH, RC_OUT_SEG, RC_OUT_TRI, RC_OUT_HIT = 1, 2, 4, 8


class RCError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


class rc_sensor_desc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("width", C.c_int32), ("height", C.c_int32), ("hfov", C.c_float),
                ("vmin", C.c_float), ("vmax", C.c_float), ("hmin", C.c_float), ("hmax", C.c_float),
                ("near_", C.c_float), ("far_", C.c_float), ("dir_table", C.c_void_p), ("stereo", C.c_float * 3)]


class rc_outputs(C.Structure):
    _fields_ = [("depth", C.c_void_p), ("seg", C.c_void_p), ("tri", C.c_void_p), ("hit_xyz", C.c_void_p),
                ("normal", C.c_void_p), ("bary", C.c_void_p), ("point", C.c_void_p), ("vert", C.c_void_p),
                ("shadow", C.c_void_p)]


def _outputs(total_rays, depth=None, seg=None, tri=None, hit_xyz=None, normal=None, bary=None, point=None,
             vert=None, shadow=None) -> rc_outputs:
    def opt(t, dt, k, what):
        return None if t is None else _dev(t, dt, k * total_rays, what)
    return rc_outputs(opt(depth, "float32", 1, "depth"), opt(seg, "int32", 1, "seg"), opt(tri, "int32", 1, "tri"),
                      opt(hit_xyz, "float32", 3, "hit_xyz"), opt(normal, "float32", 3, "normal"),
                      opt(bary, "float32", 2, "bary"), opt(point, "float32", 3, "point"),
                      opt(vert, "int32", 3, "vert"), opt(shadow, "uint8", 1, "shadow"))


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)


class rc_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


def torch_allocator(device: int = 0) -> rc_allocator:
    """An ``rc_allocator`` that takes the library's device memory from torch's
    caching allocator (so it shows in ``torch.cuda.memory_allocated``)."""
    import torch

    def _alloc(user, nbytes, stream):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device, int(stream or 0))
        except Exception:  # reported by the library as RC_E_OOM
            return None

    def _free(user, ptr, nbytes, stream):
        torch.cuda.caching_allocator_delete(int(ptr))

    return rc_allocator(ALLOC_FN(_alloc), FREE_FN(_free), None)


class rc_request(C.Structure):
    _fields_ = [("n_envs", C.c_int32), ("env_ids", C.c_void_p), ("sensor_id", C.c_int32),
                ("sensor_T", C.c_void_p), ("out", rc_outputs), ("lib_outputs", C.c_int32)]


_lib = None


def lib():
    """The loaded ``librc.so`` (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2503_01471_amd.build`")
        L = C.CDLL(LIB_PATH)
        P, I32, I64, SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        sig = {
            "rc_status_string": (C.c_char_p, [I32]),
            "rc_last_error": (C.c_char_p, []),
            "rc_create": (I32, [I32, P, C.POINTER(rc_allocator), SZ, C.POINTER(P)]),
            "rc_destroy": (I32, [P]),
            "rc_memory_used": (I32, [P, C.POINTER(SZ)]),
            "rc_mesh_add": (I32, [P, P, I32, P, I32, C.POINTER(I32)]),
            "rc_scene_load": (I32, [P, I32, P, P, P, P]),
            "rc_scene_options": (I32, [P, I32]),
            "rc_sensor_add": (I32, [P, C.POINTER(rc_sensor_desc), C.POINTER(I32)]),
            "rc_sensors_attach": (I32, [P, P, P]),
            "rc_ray_layout": (I32, [P, P, C.POINTER(I64)]),
            "rc_env_tri_offsets": (I32, [P, P]),
            "rc_set_instance_poses": (I32, [P, P, P]),
            "rc_set_sensor_poses": (I32, [P, P, P]),
            "rc_move_instances": (I32, [P, P, I32, C.c_float, P]),
            "rc_build": (I32, [P, P, I32, P]),
            "rc_refit": (I32, [P, P, P]),
            "rc_render": (I32, [P, C.POINTER(rc_outputs), I32, P]),
            "rc_render_noalloc": (I32, [P, C.POINTER(rc_outputs), P]),
            "rc_render_stats": (I32, [P, P, P]),
            "rc_debug_world": (I32, [P, P]),
            "rc_debug_rays": (I32, [P, I32, I64, P, P, P]),
            "rc_debug_bvh": (I32, [P, I32, C.POINTER(I32), P, P, P, P, C.POINTER(I32)]),
            "rc_autotune": (I32, [P, C.c_char_p, P]),
            "rc_tuning_set": (I32, [P, P]),
            "rc_step_graph_create": (I32, [P, C.POINTER(rc_outputs), P, C.c_float, C.POINTER(P)]),
            "rc_graph_set_step": (I32, [P, I32, P]),
            "rc_graph_launch": (I32, [P, P]),
            "rc_graph_destroy": (I32, [P]),
            "rc_server_create": (I32, [P, I32, I32, SZ, C.POINTER(P)]),
            "rc_server_submit": (I32, [P, C.POINTER(rc_request), C.POINTER(C.c_uint64)]),
            "rc_server_poll": (I32, [P, C.c_uint64, C.POINTER(I32), C.POINTER(C.c_double)]),
            "rc_server_wait": (I32, [P, C.c_uint64, C.POINTER(C.c_double)]),
            "rc_server_outputs": (I32, [P, C.c_uint64, C.POINTER(rc_outputs)]),
            "rc_server_release": (I32, [P, C.c_uint64]),
            "rc_server_destroy": (I32, [P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int) -> None:
    if status != 0:
        L = lib()
        raise RCError(status, f"{L.rc_status_string(status).decode()}: {L.rc_last_error().decode()}")


def _host(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a) -> Optional[int]:
    """Address of a numpy array or torch tensor (None passes NULL)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _dev(t, dtype_name: str, numel: int, what: str):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{what} must be a torch tensor on a HIP device")
    if str(t.dtype) != "torch." + dtype_name or not t.is_contiguous() or t.numel() < numel:
        raise TypeError(f"{what} must be a contiguous torch.{dtype_name} tensor with >= {numel} elements")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream or None
    return getattr(stream, "cuda_stream", stream) or None


# --------------------------------------------------------------------------
# one wrapper per entry point
# --------------------------------------------------------------------------
_allocators = {}  # context -> its rc_allocator (the callbacks must outlive the context)


def rc_create(device: int = 0, stream=None, hbm_budget: int = 0, allocator: Optional[rc_allocator] = None):
    out = C.c_void_p()
    _check(lib().rc_create(device, _stream(stream) if stream is not None else None,
                           None if allocator is None else C.byref(allocator), hbm_budget, C.byref(out)))
    if allocator is not None:
        _allocators[out.value] = allocator
    return out.value


def rc_destroy(ctx) -> None:
    _check(lib().rc_destroy(ctx))
    _allocators.pop(ctx, None)


def rc_memory_used(ctx) -> int:
    n = C.c_size_t()
    _check(lib().rc_memory_used(ctx, C.byref(n)))
    return n.value


def rc_mesh_add(ctx, xyz, tris) -> int:
    xyz = _host(xyz, np.float32).reshape(-1, 3)
    tris = _host(tris, np.int32).reshape(-1, 3)
    mid = C.c_int32()
    _check(lib().rc_mesh_add(ctx, _ptr(xyz), len(xyz), _ptr(tris), len(tris), C.byref(mid)))
    return mid.value


def rc_scene_load(ctx, inst_offsets, inst_mesh, inst_seg, inst_dynamic=None) -> None:
    io = _host(inst_offsets, np.int64)
    im = _host(inst_mesh, np.int32)
    iseg = _host(inst_seg, np.int32)
    idyn = None if inst_dynamic is None else _host(inst_dynamic, np.uint8)
    _check(lib().rc_scene_load(ctx, len(io) - 1, _ptr(io), _ptr(im), _ptr(iseg), _ptr(idyn)))


def rc_scene_options(ctx, flags) -> None:
    _check(lib().rc_scene_options(ctx, int(flags)))


def rc_sensor_add(ctx, kind, width, height, hfov=0.0, vmin=0.0, vmax=0.0, hmin=0.0, hmax=0.0, near=0.0,
                  far=0.0, dir_table=None, stereo=(0.0, 0.0, 0.0)) -> int:
    tab = None if dir_table is None else _host(dir_table, np.float32)
    d = rc_sensor_desc(kind, width, height, hfov, vmin, vmax, hmin, hmax, near, far,
                       None if tab is None else tab.ctypes.data, (C.c_float * 3)(*[float(x) for x in stereo]))
    sid = C.c_int32()
    _check(lib().rc_sensor_add(ctx, C.byref(d), C.byref(sid)))
    return sid.value


def rc_sensors_attach(ctx, sens_offsets, sensor_ids) -> None:
    so = _host(sens_offsets, np.int64)
    ids = _host(sensor_ids, np.int32)
    _check(lib().rc_sensors_attach(ctx, _ptr(so), _ptr(ids)))


def rc_ray_layout(ctx, n_sensor_inst: int):
    off = np.zeros(n_sensor_inst + 1, np.int64)
    tot = C.c_int64()
    _check(lib().rc_ray_layout(ctx, _ptr(off), C.byref(tot)))
    return off, tot.value


def rc_env_tri_offsets(ctx, n_envs: int) -> np.ndarray:
    off = np.zeros(n_envs + 1, np.int64)
    _check(lib().rc_env_tri_offsets(ctx, _ptr(off)))
    return off


def rc_set_instance_poses(ctx, d_inst_T, stream=None) -> None:
    _check(lib().rc_set_instance_poses(ctx, _dev(d_inst_T, "float32", 0, "d_inst_T"), _stream(stream)))


def rc_set_sensor_poses(ctx, d_sensor_T, stream=None) -> None:
    _check(lib().rc_set_sensor_poses(ctx, _dev(d_sensor_T, "float32", 0, "d_sensor_T"), _stream(stream)))


def rc_move_instances(ctx, d_vel, step: int, dt: float, stream=None) -> None:
    _check(lib().rc_move_instances(ctx, _dev(d_vel, "float32", 0, "d_vel"), step, dt, _stream(stream)))


def _mask(env_mask):
    return None if env_mask is None else _dev(env_mask, "uint8", 0, "env_mask")


def rc_build(ctx, builder: int = RC_BUILD_SAH, stream=None, env_mask=None) -> None:
    """env_mask: None (every environment) or a uint8 device tensor [n_envs]."""
    _check(lib().rc_build(ctx, _mask(env_mask), builder, _stream(stream)))


def rc_refit(ctx, stream=None, env_mask=None) -> None:
    """env_mask: None (every environment) or a uint8 device tensor [n_envs]."""
    _check(lib().rc_refit(ctx, _mask(env_mask), _stream(stream)))


def rc_render(ctx, depth=None, seg=None, tri=None, hit_xyz=None, mode: int = RC_RENDER_FLAT, stream=None,
              total_rays: int = 0, normal=None, bary=None, point=None, vert=None, shadow=None) -> None:
    out = _outputs(total_rays, depth, seg, tri, hit_xyz, normal, bary, point, vert, shadow)
    _check(lib().rc_render(ctx, C.byref(out), mode, _stream(stream)))


def rc_render_noalloc(ctx, depth=None, seg=None, tri=None, hit_xyz=None, stream=None, total_rays: int = 0,
                      normal=None, bary=None, point=None, vert=None, shadow=None) -> None:
    out = _outputs(total_rays, depth, seg, tri, hit_xyz, normal, bary, point, vert, shadow)
    _check(lib().rc_render_noalloc(ctx, C.byref(out), _stream(stream)))


def rc_render_stats(ctx, stream=None) -> np.ndarray:
    c = np.zeros(4, np.int64)
    _check(lib().rc_render_stats(ctx, _stream(stream), _ptr(c)))
    return c


def rc_debug_world(ctx, n_tris: int) -> np.ndarray:
    w = np.zeros((n_tris, 9), np.float32)
    _check(lib().rc_debug_world(ctx, _ptr(w)))
    return w


def rc_debug_rays(ctx, s: int, ray_idx):
    idx = _host(ray_idx, np.int64)
    o = np.zeros((len(idx), 3), np.float32)
    d = np.zeros((len(idx), 3), np.float32)
    _check(lib().rc_debug_rays(ctx, s, len(idx), _ptr(idx), _ptr(o), _ptr(d)))
    return o, d


def rc_debug_bvh(ctx, e: int, n_tris: int) -> dict:
    cap = n_tris + n_tris // 4 + 2
    boxes = np.zeros((cap, 2, 6), np.float32)
    ch = np.zeros((cap, 2), np.int32)
    par = np.zeros(cap, np.int32)
    ids = np.zeros(max(n_tris, 1), np.int32)
    nn = C.c_int32()
    root = C.c_int32()
    _check(lib().rc_debug_bvh(ctx, e, C.byref(nn), _ptr(boxes), _ptr(ch), _ptr(par), _ptr(ids), C.byref(root)))
    n = nn.value
    return dict(n_nodes=n, boxes=boxes[:n], children=ch[:n], parent=par[:n], leaf_ids=ids[:n_tris],
                root=root.value)


def rc_autotune(ctx, cache_path: Optional[str] = None):
    """Returns (tile columns, tiles per queue pop, cost order flag, node width)."""
    ch = np.zeros(4, np.int32)
    _check(lib().rc_autotune(ctx, None if cache_path is None else cache_path.encode(), _ptr(ch)))
    return tuple(int(x) for x in ch)


def rc_tuning_set(ctx, tile_cols: int = 8, chunk: int = 4, cost_order: int = 1, width: int = 2) -> None:
    ch = np.array([tile_cols, chunk, cost_order, width], np.int32)
    _check(lib().rc_tuning_set(ctx, _ptr(ch)))


def rc_step_graph_create(ctx, d_vel, dt: float, depth=None, seg=None, tri=None, hit_xyz=None, total_rays: int = 0,
                         normal=None, bary=None, point=None, vert=None, shadow=None):
    out = _outputs(total_rays, depth, seg, tri, hit_xyz, normal, bary, point, vert, shadow)
    g = C.c_void_p()
    _check(lib().rc_step_graph_create(ctx, C.byref(out), _dev(d_vel, "float32", 0, "d_vel"), dt, C.byref(g)))
    return g.value


def rc_graph_set_step(graph, step: int, stream=None) -> None:
    _check(lib().rc_graph_set_step(graph, step, _stream(stream)))


def rc_graph_launch(graph, stream=None) -> None:
    _check(lib().rc_graph_launch(graph, _stream(stream)))


def rc_graph_destroy(graph) -> None:
    _check(lib().rc_graph_destroy(graph))


def rc_server_create(ctx, mode: int = RC_SERVE_BATCHED, n_streams: int = 4, hbm_budget: int = 4 << 30):
    """hbm_budget 0: half of the device memory free at creation."""
    srv = C.c_void_p()
    _check(lib().rc_server_create(ctx, mode, n_streams, hbm_budget, C.byref(srv)))
    return srv.value


def rc_server_submit(server, env_ids, sensor_id: int, depth=None, seg=None, sensor_T=None, tri=None,
                     hit_xyz=None, lib_outputs: int = 0) -> int:
    """Caller device buffers (depth / seg / tri / hit_xyz, each optional), or
    with ``lib_outputs`` (RC_OUT_* bits) and no buffers, library outputs read
    through :func:`rc_server_outputs` and freed by :func:`rc_server_release`."""
    ids = _host(env_ids, np.int32)
    T = None if sensor_T is None else _host(sensor_T, np.float32)
    n = len(ids)
    out = rc_outputs(None if depth is None else _dev(depth, "float32", 0, "depth"),
                     None if seg is None else _dev(seg, "int32", 0, "seg"),
                     None if tri is None else _dev(tri, "int32", 0, "tri"),
                     None if hit_xyz is None else _dev(hit_xyz, "float32", 0, "hit_xyz"))
    req = rc_request(n, ids.ctypes.data, sensor_id, None if T is None else T.ctypes.data, out, lib_outputs)
    t = C.c_uint64()
    _check(lib().rc_server_submit(server, C.byref(req), C.byref(t)))
    return t.value


def rc_server_outputs(server, ticket: int, n_rays: int, device: int = 0) -> dict:
    """Views (torch tensors, no copy) of a completed ticket's library outputs;
    valid until :func:`rc_server_release`.  n_rays: rays of the request."""
    import torch
    o = rc_outputs()
    _check(lib().rc_server_outputs(server, ticket, C.byref(o)))

    def view(ptr, typestr, k):
        if not ptr:
            return None
        return torch.as_tensor(_DeviceArray(ptr, n_rays * k, typestr), device=torch.device("cuda", device))
    return {"depth": view(o.depth, "<f4", 1), "seg": view(o.seg, "<i4", 1), "tri": view(o.tri, "<i4", 1),
            "hit_xyz": view(o.hit_xyz, "<f4", 3)}


class _DeviceArray:
    """A device buffer the library owns, described by the array interface
    torch reads for device memory (the tensor views it without a copy)."""

    def __init__(self, ptr: int, n: int, typestr: str):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": typestr, "data": (int(ptr), False),
                                         "strides": None, "version": 2}


def rc_server_release(server, ticket: int) -> None:
    _check(lib().rc_server_release(server, ticket))


def rc_server_poll(server, ticket: int):
    """(done, latency_s); a reported completion releases a caller-buffer
    ticket (library-output tickets stay until rc_server_release)."""
    done = C.c_int32()
    lat = C.c_double()
    _check(lib().rc_server_poll(server, ticket, C.byref(done), C.byref(lat)))
    return bool(done.value), lat.value


def rc_server_wait(server, ticket: int) -> float:
    lat = C.c_double()
    _check(lib().rc_server_wait(server, ticket, C.byref(lat)))
    return lat.value


def rc_server_destroy(server) -> None:
    _check(lib().rc_server_destroy(server))
