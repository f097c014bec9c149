"""rc_render_noalloc, the batched render whose queue heads live in the
library's static device array, against rc_render's batched form (and the
oracle) through the C ABI: two calls in a row, the second on a smaller
scene of another context, so the array holds the first call's heads when the
second one starts."""
import numpy as np
import pytest

import parity
from oracle import oracle as O
from paper_2503_01471_amd import rc, scenes as S

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(f"\n[gpu] {msg}", flush=True)


def _filled(R):
    """Every output of rc_render's first four kinds, pre-filled with values no
    render writes, so an unwritten ray shows."""
    o = R.alloc(depth=True, seg=True, tri=True, hit=True)
    o["depth"].fill_(-7.0)
    o["seg"].fill_(-7)
    o["tri"].fill_(-7)
    o["hit_xyz"].fill_(-7.0)
    return o


def _host(o):
    return {k: v.cpu().numpy() for k, v in o.items() if v is not None}


def _render_both(R, chunk):
    ref = _filled(R)
    got = _filled(R)
    rc.rc_tuning_set(R.ctx, 8, chunk, 1)
    R.render(out=ref, mode=rc.RC_RENDER_BATCHED)
    used = rc.rc_memory_used(R.ctx)
    rc.rc_render_noalloc(R.ctx, got["depth"], got["seg"], got["tri"], got["hit_xyz"], None, R.total_rays)
    torch.cuda.synchronize()
    assert rc.rc_memory_used(R.ctx) == used  # no library allocation
    ref, got = _host(ref), _host(got)
    for k in ("depth", "seg", "tri"):
        assert np.array_equal(got[k], ref[k]), k
        assert not np.any(got[k] == -7), k
    assert np.array_equal(np.isnan(got["hit_xyz"]), np.isnan(ref["hit_xyz"]))
    assert np.array_equal(np.nan_to_num(got["hit_xyz"]), np.nan_to_num(ref["hit_xyz"]))
    return got


def _oracle_check(scene, got):
    rep = parity.compare({**got, "hit_xyz": got["hit_xyz"].reshape(-1, 3)}, O.render(scene))
    print(rep, flush=True)
    parity.assert_contract(rep)


def test_noalloc_matches_batched_then_smaller():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2503_01471_amd.renderer import Renderer
    big = S.make_cfg4(n_envs=8, env_ids=list(range(8)))
    small = S.make_cfg4(n_envs=3, env_ids=[40, 41, 42])
    _say(f"noalloc: {big.name} {big.n_envs} envs, {big.total_rays()} rays")
    RB = Renderer(big)
    gb = _render_both(RB, 1)
    _oracle_check(big, gb)
    _say(f"noalloc: smaller scene, other context: {small.n_envs} envs, {small.total_rays()} rays")
    RS = Renderer(small)
    assert RS.total_rays < RB.total_rays
    gs = _render_both(RS, 4)
    _oracle_check(small, gs)
    # and back on the first context with another pop size, then without a queue
    _say("noalloc: first context again, 16 tiles per pop")
    _render_both(RB, 16)
    _say("noalloc: first context, one-launch tuning")
    _render_both(RB, 0)
    with pytest.raises(rc.RCError) as ei:
        rc.rc_render_noalloc(RB.ctx, None, None, None, None, None, 0, normal=torch.empty(3, device="cuda"))
    assert ei.value.status == -1
    RS.close()
    RB.close()
