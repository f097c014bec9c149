"""GPU parity of the two-level form (RC_BUILD_TWO_LEVEL): per-mesh BVHs in
each mesh's own frame under a per-environment BVH of instance boxes.

Its result is the exact nearest hit on the moved meshes with the moved
vertices unrounded, so the reference is the oracle on FP64 world vertices
(``O.world64``), under the same parity contract as the single-level form.
Every launch form of the two-level scene is bit-identical; against the
single-level form (FP32 world vertices) the triangle ids are compared and the
disagreements counted."""
import numpy as np
import pytest

import parity
from oracle import oracle as O
from paper_2503_01471_amd import rc, scenes as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(f"\n[gpu] {msg}", flush=True)


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def _R(scene, **kw):
    from paper_2503_01471_amd.renderer import Renderer
    return Renderer(scene, **kw)


def _host(out):
    return {k: (None if v is None else v.cpu().numpy()) for k, v in out.items()}


def _render(R, mode):
    o = _host(R.render(mode=mode))
    torch.cuda.synchronize()
    return o


def _forms_equal(R, ref):
    for mode in (rc.RC_RENDER_PLAIN, rc.RC_RENDER_BATCHED):
        o = _render(R, mode)
        for k in ("depth", "seg", "tri"):
            assert np.array_equal(o[k], ref[k]), (mode, k)
        assert np.array_equal(np.nan_to_num(o["hit_xyz"]), np.nan_to_num(ref["hit_xyz"])), mode


def _check(scene, poses=None, R=None, sample=None):
    """Two-level render of `scene` (already built two-level in R, else built
    here) against the FP64-vertex oracle; returns the outputs."""
    _need_gpu()
    own = R is None
    if own:
        R = _R(scene, build=False)
        rc.rc_build(R.ctx, rc.RC_BUILD_TWO_LEVEL)
    out = _render(R, rc.RC_RENDER_FLAT)
    _forms_equal(R, out)
    w64 = O.world64(scene, poses)
    if sample is None:
        ora = O.render(scene, w64)
        got = out
    else:
        rng = np.random.default_rng(0)
        g = np.sort(rng.choice(R.total_rays, sample, replace=False))
        s = np.searchsorted(R.ray_offsets, g, side="right") - 1
        ora = O.render(scene, w64, sensor_inst=s, ray_idx=g - R.ray_offsets[s])
        got = {k: (None if v is None else v[g]) for k, v in out.items()}
    rep = parity.compare(got, ora)
    print(scene.name, rep, flush=True)
    parity.assert_contract(rep)
    if own:
        R.close()
    return out, rep


def test_two_level_cfg1_every_ray():
    scene = S.make_cfg1()
    _say("two-level cfg1")
    out, rep = _check(scene)
    assert rep["robust"] > 0.9 * rep["n"]
    # against the single-level form: the same triangles but where the FP32
    # rounding of the moved vertices decides (axis-aligned boxes: never)
    R = _R(scene)
    flat = _render(R, rc.RC_RENDER_FLAT)
    R.close()
    assert np.array_equal(flat["tri"], out["tri"])


def test_two_level_rotated_and_scaled():
    """Rotated, non-uniformly scaled cylinders, spheres and boxes in a room
    (inverse poses with every entry nonzero)."""
    scene = S.make_cfg2(n_envs=3, W=96, H=54)
    _say("two-level cfg2 slice")
    out, rep = _check(scene)
    R = _R(scene)
    flat = _render(R, rc.RC_RENDER_FLAT)
    R.close()
    ora32 = O.render(scene)
    robust = (ora32.cls & O.BORDER_MASK) == 0
    diff = int(np.sum(robust & (flat["tri"] != out["tri"])))
    print(f"robust rays where the single- and two-level forms differ: {diff} of {int(robust.sum())}", flush=True)
    assert diff <= 1e-4 * robust.sum()


def test_two_level_forest_full_resolution():
    scene = S.make_cfg3(n_envs=4)
    _say("two-level cfg3 slice")
    _check(scene)


def test_two_level_motion_refit_and_graph():
    """Moving boxes: eager moves with a refit of the instance boxes only, and
    the captured step graph, against the oracle at the moved poses."""
    _need_gpu()
    scene = S.make_cfg4(n_envs=6)
    R = _R(scene, build=False)
    rc.rc_build(R.ctx, rc.RC_BUILD_TWO_LEVEL)
    for step in (1, 37):
        _say(f"two-level cfg4 step {step}")
        R.move(step)
        R.refit()
        _check(scene, O.moved_poses(scene, step), R=R)
    n = R.total_rays
    gout = dict(depth=torch.empty(n, device="cuda"), seg=torch.empty(n, dtype=torch.int32, device="cuda"),
                tri=torch.empty(n, dtype=torch.int32, device="cuda"))
    g = rc.rc_step_graph_create(R.ctx, R.inst_vel, float(scene.dt), depth=gout["depth"], seg=gout["seg"],
                                tri=gout["tri"], total_rays=n)
    rc.rc_graph_set_step(g, 5)
    for step in (5, 6, 7):
        _say(f"two-level graph replay step {step}")
        rc.rc_graph_launch(g)
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in gout.items()}
        R.move(step)
        R.refit()
        ref = _render(R, rc.RC_RENDER_BATCHED)
        for k in ("depth", "seg", "tri"):
            assert np.array_equal(got[k], ref[k]), (step, k)
    rep = parity.compare(got, O.render(scene, O.world64(scene, O.moved_poses(scene, 7))))
    parity.assert_contract(rep)
    rc.rc_graph_destroy(g)
    R.close()


def test_two_level_mode_switches_and_errors():
    _need_gpu()
    scene = S.make_cfg4(n_envs=4)
    R = _R(scene)
    flat = _render(R, rc.RC_RENDER_FLAT)
    rc.rc_build(R.ctx, rc.RC_BUILD_TWO_LEVEL)
    two = _render(R, rc.RC_RENDER_FLAT)
    # a masked build must keep the form of the last full build
    mask = torch.ones(scene.n_envs, dtype=torch.uint8, device="cuda")
    with pytest.raises(rc.RCError) as ei:
        rc.rc_build(R.ctx, rc.RC_BUILD_SAH, env_mask=mask)
    assert ei.value.status == -4
    rc.rc_build(R.ctx, rc.RC_BUILD_TWO_LEVEL, env_mask=mask)
    assert np.array_equal(_render(R, rc.RC_RENDER_FLAT)["tri"], two["tri"])
    # stereo shadows need the single-level BVH
    o = R.alloc(depth=True, seg=True, tri=True, shadow=True)
    with pytest.raises(rc.RCError) as ei:
        R.render(out=o, mode=rc.RC_RENDER_FLAT)
    assert ei.value.status == -4
    # the further outputs read the world copy and work in both forms
    x2 = _host(R.render(mode=rc.RC_RENDER_BATCHED, depth=True, seg=True, tri=True, normal=True, point=True))
    rc.rc_build(R.ctx, rc.RC_BUILD_SAH)
    back = _render(R, rc.RC_RENDER_FLAT)
    for k in ("depth", "seg", "tri"):
        assert np.array_equal(back[k], flat[k]), k
    x1 = _host(R.render(mode=rc.RC_RENDER_BATCHED, depth=True, seg=True, tri=True, normal=True, point=True))
    same = x1["tri"] == x2["tri"]
    assert np.array_equal(x1["normal"][same], x2["normal"][same], equal_nan=True)
    R.close()
    # a mesh above the two-level limit
    big = S.icosphere_mesh(5)  # 20480 triangles
    ctx = rc.rc_create(0)
    try:
        mid = rc.rc_mesh_add(ctx, *big)
        rc.rc_scene_load(ctx, [0, 1], [mid], [1])
        rc.rc_set_instance_poses(ctx, torch.tensor(S.affine(np.eye(3), (0, 0, 0)), dtype=torch.float32,
                                                   device="cuda").reshape(-1))
        with pytest.raises(rc.RCError) as ei:
            rc.rc_build(ctx, rc.RC_BUILD_TWO_LEVEL)
        assert ei.value.status == -1
    finally:
        rc.rc_destroy(ctx)


@pytest.mark.parametrize("cfg", [3, 4])
def test_two_level_full_size_sampled(cfg):
    """The full-size workload built two-level, batched at the autotuner's
    choice, on a seeded sample of rays."""
    _need_gpu()
    scene = S.make(cfg)
    _say(f"two-level full {scene.name}: envs={scene.n_envs} rays={scene.total_rays()}")
    R = _R(scene, build=False)
    rc.rc_build(R.ctx, rc.RC_BUILD_TWO_LEVEL)
    rc.rc_autotune(R.ctx, None)
    _check(scene, R=R, sample=12000)
    R.close()


def test_two_level_only_scene():
    """RC_SCENE_TWO_LEVEL_ONLY: the renders of a two-level build of the same
    scene loaded normally (every form, refits of moving boxes, a step graph)
    and the oracle's, a fraction of the library memory, and RC_E_STATE for
    what needs the single-level arrays."""
    _need_gpu()
    scene = S.make_cfg4(n_envs=6)
    A = _R(scene, build=False)
    rc.rc_build(A.ctx, rc.RC_BUILD_TWO_LEVEL)
    B = _R(scene, scene_flags=rc.RC_SCENE_TWO_LEVEL_ONLY)
    ma, mb = rc.rc_memory_used(A.ctx), rc.rc_memory_used(B.ctx)
    print(f"library bytes: normal load {ma}, two-level only {mb}", flush=True)
    assert mb < ma
    ref = _render(A, rc.RC_RENDER_FLAT)
    for mode in (rc.RC_RENDER_PLAIN, rc.RC_RENDER_FLAT, rc.RC_RENDER_BATCHED):
        got = _render(B, mode)
        for k in ("depth", "seg", "tri"):
            assert np.array_equal(got[k], ref[k]), (mode, k)
        assert np.array_equal(np.nan_to_num(got["hit_xyz"]), np.nan_to_num(ref["hit_xyz"])), mode
    parity.assert_contract(parity.compare(ref, O.render(scene, O.world64(scene))))
    for step in (3, 40):
        _say(f"two-level only, step {step}")
        for R in (A, B):
            R.move(step)
            R.refit()
        a, b = _render(A, rc.RC_RENDER_BATCHED), _render(B, rc.RC_RENDER_BATCHED)
        for k in ("depth", "seg", "tri"):
            assert np.array_equal(a[k], b[k]), (step, k)
    n = B.total_rays
    gout = dict(depth=torch.empty(n, device="cuda"), seg=torch.empty(n, dtype=torch.int32, device="cuda"),
                tri=torch.empty(n, dtype=torch.int32, device="cuda"))
    g = rc.rc_step_graph_create(B.ctx, B.inst_vel, float(scene.dt), depth=gout["depth"], seg=gout["seg"],
                                tri=gout["tri"], total_rays=n)
    rc.rc_graph_set_step(g, 5)
    rc.rc_graph_launch(g)
    torch.cuda.synchronize()
    A.move(5)
    A.refit()
    a = _render(A, rc.RC_RENDER_BATCHED)
    for k in ("depth", "seg", "tri"):
        assert np.array_equal(gout[k].cpu().numpy(), a[k]), ("graph", k)
    rc.rc_graph_destroy(g)
    # what needs the single-level arrays
    for call in (lambda: rc.rc_build(B.ctx, rc.RC_BUILD_SAH), lambda: rc.rc_build(B.ctx, rc.RC_BUILD_LBVH),
                 lambda: B.render(mode=rc.RC_RENDER_BRUTE),
                 lambda: B.render(mode=rc.RC_RENDER_BATCHED, depth=True, seg=True, tri=True, normal=True),
                 lambda: B.render(out=B.alloc(depth=True, seg=True, tri=True, shadow=True), mode=rc.RC_RENDER_FLAT),
                 lambda: rc.rc_debug_world(B.ctx, B.n_tris)):
        with pytest.raises(rc.RCError) as ei:
            call()
        assert ei.value.status == -4
    with pytest.raises(rc.RCError) as ei:
        rc.rc_scene_options(B.ctx, 2)
    assert ei.value.status == -1
    # still usable after the refusals
    b = _render(B, rc.RC_RENDER_BATCHED)
    for k in ("depth", "seg", "tri"):
        assert np.array_equal(b[k], a[k]), ("after errors", k)
    A.close()
    B.close()
