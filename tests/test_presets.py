"""Sensor presets and user-defined projection models (host side)."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2503_01471_amd import presets as P
from paper_2503_01471_amd import scenes as S


@pytest.mark.parametrize("name", sorted(P.PRESETS))
def test_preset_is_valid(name):
    d = P.PRESETS[name]()
    assert d.width > 0 and d.height > 0 and 0 < d.near < d.far
    if d.kind == S.TABLE:
        t = np.asarray(d.dir_table, np.float64)
        assert t.shape == (d.width * d.height, 3)
        assert np.abs(np.linalg.norm(t, axis=1) - 1).max() < 1e-6
    if d.kind == S.LIDAR:
        assert d.vmax > d.vmin and d.hmax - d.hmin == pytest.approx(2 * math.pi)


def test_tof_grid_geometry():
    d = P.tof_grid(8, 4, 45.0, 30.0, 0.02, 4.0)
    t = np.asarray(d.dir_table, np.float64).reshape(4, 8, 3)
    az = np.degrees(np.arctan2(t[..., 1], t[..., 0]))
    el = np.degrees(np.arcsin(t[..., 2]))
    # zone centres evenly spaced, symmetric about +x, row 0 on top, column 0 on the left (+y)
    assert np.allclose(az[0], 22.5 - (np.arange(8) + 0.5) * 45.0 / 8, atol=1e-4)
    assert np.allclose(el[:, 0], 15.0 - (np.arange(4) + 0.5) * 30.0 / 4, atol=1e-4)


def test_dome_geometry():
    d = P.dome_lidar(5, 12, 0.3, 20.0)
    t = np.asarray(d.dir_table, np.float64).reshape(5, 12, 3)
    assert np.allclose(t[0], [0, 0, 1], atol=1e-7)  # pole ring
    assert np.abs(t[-1, :, 2]).max() < 1e-6  # last ring on the horizon
    polar = np.degrees(np.arccos(np.clip(t[..., 2], -1, 1)))
    assert np.allclose(polar.mean(1), [0, 22.5, 45, 67.5, 90], atol=1e-4)
    od = P.ouster_dome(16, 64)
    assert od.vmin == 0.0 and od.vmax == pytest.approx(math.pi / 2)


def test_presets_in_a_closed_room_see_walls():
    """Oracle: every ray of every preset, from inside a closed room, hits a
    surface within range (dome and ToF ranges are positive and finite)."""
    sc = S.make_cfg2(n_envs=1, W=8, H=8)
    for d in (P.vl53l5cx(far=30.0), P.dome_lidar(6, 16, 0.05, 30.0), P.ouster_dome(8, 32, far=30.0),
              P.realsense_d455(32, 18)):
        s2 = S.Scene(**{**sc.__dict__, "sensors": [d]})
        r = O.render(s2)
        assert np.all(r.tri >= 0) and np.all(r.t[r.tri >= 0] >= d.near)
