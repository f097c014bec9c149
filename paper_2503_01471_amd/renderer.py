"""Load a generated scene into the HIP renderer (marshalling only).

``Renderer(scene)`` registers the scene's prototype meshes, instances and
sensors through the C ABI, keeps the pose tensors on the device and exposes
build / refit / render with torch output tensors.  No rendering arithmetic
happens here.
"""
from __future__ import annotations

import numpy as np
import torch

from . import rc


class Renderer:
    def __init__(self, scene, device: int = 0, hbm_budget: int = 0, build: bool = True, allocator: str = "torch",
                 scene_flags: int = 0):
        """allocator: "torch" (library memory from torch's caching allocator) or
        "hip" (the library's own hipMalloc); scene_flags: rc_scene_options
        (RC_SCENE_TWO_LEVEL_ONLY: build with RC_BUILD_TWO_LEVEL)."""
        self.scene = scene
        self.device = torch.device("cuda", device)
        hook = {"torch": lambda: rc.torch_allocator(device), "hip": lambda: None}[allocator]()
        self.ctx = rc.rc_create(device, None, hbm_budget, allocator=hook)
        for v, t in scene.protos:
            rc.rc_mesh_add(self.ctx, v, t)
        if scene_flags:
            rc.rc_scene_options(self.ctx, scene_flags)
        rc.rc_scene_load(self.ctx, scene.inst_offsets, scene.inst_mesh, scene.inst_seg, scene.inst_dynamic)
        for desc in scene.sensors:
            rc.rc_sensor_add(self.ctx, desc.kind, desc.width, desc.height, desc.hfov, desc.vmin, desc.vmax,
                             desc.hmin, desc.hmax, desc.near, desc.far, desc.dir_table, getattr(desc, "stereo", (0, 0, 0)))
        rc.rc_sensors_attach(self.ctx, scene.sens_offsets, scene.sensor_ids)
        self.n_si = len(scene.sensor_ids)
        self.ray_offsets, self.total_rays = rc.rc_ray_layout(self.ctx, self.n_si)
        self.env_tri_off = rc.rc_env_tri_offsets(self.ctx, scene.n_envs)
        self.n_tris = int(self.env_tri_off[-1])
        self.inst_T = torch.from_numpy(np.ascontiguousarray(scene.inst_T, np.float32)).to(self.device)
        self.sensor_T = torch.from_numpy(np.ascontiguousarray(scene.sensor_T, np.float32)).to(self.device)
        self.inst_vel = torch.from_numpy(np.ascontiguousarray(scene.inst_vel, np.float32)).to(self.device)
        if scene.n_inst:
            rc.rc_set_instance_poses(self.ctx, self.inst_T)
        else:
            rc.rc_set_instance_poses(self.ctx, torch.zeros(12, device=self.device))
        if self.n_si:
            rc.rc_set_sensor_poses(self.ctx, self.sensor_T)
        else:
            rc.rc_set_sensor_poses(self.ctx, torch.zeros(12, device=self.device))
        if build:
            self.build(builder=rc.RC_BUILD_TWO_LEVEL if scene_flags & rc.RC_SCENE_TWO_LEVEL_ONLY else rc.RC_BUILD_SAH)

    # -- acceleration structure --------------------------------------------
    def _mask(self, envs):
        """uint8 device mask over environments from a list of env ids (None: all)."""
        if envs is None:
            return None
        m = torch.zeros(self.scene.n_envs, dtype=torch.uint8, device=self.device)
        ids = torch.as_tensor(np.asarray(envs, np.int64), device=self.device)
        if ids.numel():
            m[ids] = 1
        return m

    def build(self, stream=None, envs=None, builder=rc.RC_BUILD_SAH):
        rc.rc_build(self.ctx, builder, stream, env_mask=self._mask(envs))

    def refit(self, stream=None, envs=None):
        rc.rc_refit(self.ctx, stream, env_mask=self._mask(envs))

    def move(self, step: int, stream=None):
        rc.rc_move_instances(self.ctx, self.inst_vel, step, float(self.scene.dt), stream)

    def set_sensor_poses(self, T: torch.Tensor, stream=None):
        rc.rc_set_sensor_poses(self.ctx, T, stream)

    # -- outputs -------------------------------------------------------------
    def alloc(self, depth=True, seg=True, tri=False, hit=False, normal=False, bary=False, point=False, vert=False,
              shadow=False):
        n = self.total_rays
        d = self.device

        def mk(flag, shape, dt):
            return torch.empty(shape, dtype=dt, device=d) if flag else None
        return dict(depth=mk(depth, n, torch.float32), seg=mk(seg, n, torch.int32), tri=mk(tri, n, torch.int32),
                    hit_xyz=mk(hit, (n, 3), torch.float32), normal=mk(normal, (n, 3), torch.float32),
                    bary=mk(bary, (n, 2), torch.float32), point=mk(point, (n, 3), torch.float32),
                    vert=mk(vert, (n, 3), torch.int32), shadow=mk(shadow, n, torch.uint8))

    def render(self, out=None, mode: int = rc.RC_RENDER_FLAT, stream=None, **which):
        if out is None:
            out = self.alloc(**which) if which else self.alloc(depth=True, seg=True, tri=True, hit=True)
        rc.rc_render(self.ctx, out.get("depth"), out.get("seg"), out.get("tri"), out.get("hit_xyz"), mode, stream,
                     self.total_rays, normal=out.get("normal"), bary=out.get("bary"), point=out.get("point"),
                     vert=out.get("vert"), shadow=out.get("shadow"))
        return out

    def stats(self):
        return rc.rc_render_stats(self.ctx)

    def close(self):
        if self.ctx:
            rc.rc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
