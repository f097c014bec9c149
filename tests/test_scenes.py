"""Seeded input generators: reproducibility, sizes and mesh sanity."""
import numpy as np
import pytest

from paper_2503_01471_amd import scenes as S


def _edges_closed(v, t):
    from collections import Counter
    c = Counter()
    for a, b, d in t:
        for x, y in ((a, b), (b, d), (d, a)):
            c[(min(x, y), max(x, y))] += 1
    return all(n == 2 for n in c.values())


@pytest.mark.parametrize("mesh,ntri", [(S.box_mesh(), 12), (S.cylinder_mesh(16), 64), (S.cylinder_mesh(8), 32),
                                       (S.cone_mesh(24), 48), (S.icosphere_mesh(2), 320)])
def test_prototypes_closed(mesh, ntri):
    v, t = mesh
    assert len(t) == ntri
    assert _edges_closed(v, t)
    # outward winding: signed volume positive
    a, b, c = (v[t[:, i]].astype(float) for i in range(3))
    assert np.einsum("ij,ij->i", a, np.cross(b, c)).sum() > 0


def test_sizes():
    assert S.make_cfg1().env_tri_counts().tolist() == [98]
    assert S.make_cfg1().total_rays() == 3072
    sc3 = S.make_cfg3(n_envs=3)
    assert sc3.env_tri_counts().tolist() == [4802] * 3
    assert sc3.total_rays() == 3 * 32768
    sc2 = S.make_cfg2(n_envs=4)
    assert np.all(sc2.env_tri_counts() >= 12 + 40 * 12)
    assert np.all(sc2.env_tri_counts() <= 12 + 40 * 320)
    sc4 = S.make_cfg4(n_envs=8)
    assert np.all((sc4.env_tri_counts() >= 2 + 5 * 12) & (sc4.env_tri_counts() <= 2 + 200 * 12))


@pytest.mark.parametrize("cfg", [2, 3, 4])
def test_subsample_regenerates(cfg):
    full = S.make(cfg, n_envs=6)
    part = S.make(cfg, env_ids=[4, 1])
    ref = S.subset(full, [4, 1])
    for k in ("inst_offsets", "inst_mesh", "inst_seg", "inst_dynamic", "inst_T", "sens_offsets",
              "sensor_ids", "sensor_T", "inst_vel"):
        assert np.array_equal(getattr(part, k), getattr(ref, k)), k


def test_seed_changes_scene():
    a, b = S.make_cfg2(n_envs=1, seed=0), S.make_cfg2(n_envs=1, seed=1)
    assert not np.array_equal(a.inst_T, b.inst_T)
