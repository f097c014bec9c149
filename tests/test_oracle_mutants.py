"""Planted mistakes in the oracle are caught by its pins.

Each mutant is the oracle's C source with one plausible slip (a dropped term,
a wrong sign, a transposed operand, a wrong index or comparison), compiled on
the CPU into a temporary library.  The pins are then run against that library;
every mutant must fail at least one of them.  This shows that the pins, which
do not come from the oracle, constrain every part of it."""
import os
import subprocess

import pytest

import pins
from oracle import oracle as O

MUTANTS = {
    "det_drop_term": ("const double det = e1x * px + e1y * py + e1z * pz;",
                      "const double det = e1x * px + e1y * py;"),
    "q_sign": ("const double qx = sy * e1z - sz * e1y;", "const double qx = sz * e1y - sy * e1z;"),
    "t_uses_e1": ("const double t = (e2x * qx + e2y * qy + e2z * qz) * inv;",
                  "const double t = (e1x * qx + e1y * qy + e1z * qz) * inv;"),
    "bary_no_sum": ("if (u >= 0.0 && v >= 0.0 && u + v <= 1.0 && t >= tn && t <= tf)",
                    "if (u >= 0.0 && v >= 0.0 && u <= 1.0 && t >= tn && t <= tf)"),
    "near_ignored": ("if (u >= 0.0 && v >= 0.0 && u + v <= 1.0 && t >= tn && t <= tf)",
                     "if (u >= 0.0 && v >= 0.0 && u + v <= 1.0 && t <= tf)"),
    "tie_reversed": ("return ta < tb || (ta == tb && ia < ib);", "return ta < tb || (ta == tb && ia > ib);"),
    "transform_transposed": ("fmaf(row[0], x, fmaf(row[1], y, fmaf(row[2], z, row[3])))",
                             "fmaf(A[r], x, fmaf(A[4 + r], y, fmaf(A[8 + r], z, row[3])))"),
    "pinhole_axis_swap": ("dl[1] = -((((float)col + 0.5f) - hw) * s);",
                          "dl[1] = -((((float)row + 0.5f) - hw) * s);"),
    "pinhole_up_down": ("dl[2] = -((((float)row + 0.5f) - hh) * s);", "dl[2] = ((((float)row + 0.5f) - hh) * s);"),
    "lidar_channel_order": ("(double)vmax - (double)ch * ((double)vmax - (double)vmin) / (double)(H - 1)",
                            "(double)vmin + (double)ch * ((double)vmax - (double)vmin) / (double)(H - 1)"),
    "lidar_az_range": ("(double)hmin + (double)az * ((double)hmax - (double)hmin) / (double)W",
                       "(double)hmin + (double)az * ((double)hmax - (double)hmin) / (double)(W - 1)"),
    "ray_dir_transposed": ("fmaf(row[0], dl[0], fmaf(row[1], dl[1], row[2] * dl[2]))",
                           "fmaf(row[0], dl[0], fmaf(row[2], dl[1], row[1] * dl[2]))"),
    "hit_point_index": ("hit_out[3 * r + 1] = oy + bt * dy;", "hit_out[3 * r + 1] = oy + bt * dx;"),
    "graze_flag_inverted": ("if (g < GRAZE)", "if (g > GRAZE)"),
    "candidates_strict": ("if (m >= -MARGIN && t >= lo && t <= hi)", "if (m >= 0.0 && t >= lo && t <= hi)"),
    "motion_no_step": ("fmaf(vel[3 * i + r], sdt, T0[12 * i + 4 * r + 3])",
                       "fmaf(vel[3 * i + r], dt, T0[12 * i + 4 * r + 3])"),
    "normal_not_flipped": ("const double sgn = along > 0.0 ? -1.0 : 1.0;", "const double sgn = 1.0;"),
    "normal_cross_index": ("nv[1] = e1[2] * e2[0] - e1[0] * e2[2];", "nv[1] = e1[2] * e2[1] - e1[0] * e2[2];"),
    "point_world_dir": ("point[3 * r + k] = (float)(t[r] * (double)dl[3 * r + k]);",
                        "point[3 * r + k] = (float)(t[r] * (double)d[3 * r + k]);"),
    "local_dir_rotated": ("dl_out[3 * i + k] = dl[k];", "dl_out[3 * i + k] = dl[(k + 1) % 3];"),
    "bary_swapped": ("u_out[r] = bu;", "u_out[r] = bv;"),
    "shadow_backward": ("u + v <= 1.0 && t >= SHADOW_S0 && t <= 1.0)", "u + v <= 1.0 && t >= -1.0 && t <= 1.0)"),
    "shadow_beyond_camera": ("u + v <= 1.0 && t >= SHADOW_S0 && t <= 1.0)",
                             "u + v <= 1.0 && t >= SHADOW_S0 && t <= 4.0)"),
    "shadow_no_sum": ("u + v <= 1.0 && t >= SHADOW_S0 && t <= 1.0)", "t >= SHADOW_S0 && t <= 1.0)"),
    "shadow_centre_transposed": ("fmaf(P[4 * k + 0], B[0], fmaf(P[4 * k + 1], B[1], fmaf(P[4 * k + 2], B[2], P[4 * k + 3])))",
                                 "fmaf(P[k], B[0], fmaf(P[4 + k], B[1], fmaf(P[8 + k], B[2], P[4 * k + 3])))"),
    "shadow_dir_reversed": ("D32[k] = c2 - p[3 * r + k];", "D32[k] = p[3 * r + k] - c2;"),
    "table_xy_swapped": ("dl[0] = table[3 * r + 0];\n            dl[1] = table[3 * r + 1];",
                         "dl[0] = table[3 * r + 1];\n            dl[1] = table[3 * r + 0];"),
    "table_z_from_y": ("dl[2] = table[3 * r + 2];", "dl[2] = table[3 * r + 1];"),
    "table_wrong_beam": ("dl[0] = table[3 * r + 0];", "dl[0] = table[3 * (r / 2) + 0];"),
    "range_flag_near_dropped": ("if ((bt - tn) / bt <= MARGIN || (tf - bt) / bt <= MARGIN)",
                                "if ((tf - bt) / bt <= MARGIN)"),
    "depth_margin_near_dropped": ("double md = fmin((bt - tn) / bt, (tf - bt) / bt);",
                                  "double md = (tf - bt) / bt;"),
    "depth_margin_far_dropped": ("double md = fmin((bt - tn) / bt, (tf - bt) / bt);",
                                 "double md = (bt - tn) / bt;"),
    "transform64_transposed": ("(((double)row[0] * x + (double)row[1] * y) + (double)row[2] * z)",
                               "(((double)A[r] * x + (double)A[4 + r] * y) + (double)A[8 + r] * z)"),
    "transform64_z_from_y": ("(double)row[1] * y) + (double)row[2] * z)", "(double)row[1] * y) + (double)row[2] * y)"),
    "transform64_rounded": ("out[9 * i + 3 * c + r] = (((double)row[0]", "out[9 * i + 3 * c + r] = (float)(((double)row[0]"),
    "cast64_vertex_shift": ("v[j] = t32 ? (double)t32[9 * k + j] : t64[9 * k + j];",
                            "v[j] = t32 ? (double)t32[9 * k + j] : t64[9 * k + (j + 3) % 9];"),
    "cast64_vertices_rounded": ("v[j] = t32 ? (double)t32[9 * k + j] : t64[9 * k + j];",
                                "v[j] = t32 ? (double)t32[9 * k + j] : (double)(float)t64[9 * k + j];"),
}

FAST_ARGS = {pins.pin_exact: dict(seeds=range(60))}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    src = open(O.SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mpath = tmp_path / "m.c"
    mpath.write_text(src.replace(old, new))
    so = str(tmp_path / "libm.so")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                           "-o", so, str(mpath), "-lm"])
    saved = O.lib()
    O._lib = O.load(so)
    try:
        caught = []
        for pin in pins.ALL_PINS:
            try:
                fails = pin(**FAST_ARGS.get(pin, {}))
            except Exception as e:  # a crash on bad output also counts as caught
                fails = [f"{type(e).__name__}: {e}"]
            if fails:
                caught.append(pin.__name__)
                break
        assert caught, f"mutant {name} passed every pin"
    finally:
        O._lib = saved


def test_vertex_id_mutant_is_caught(monkeypatch):
    """The vertex-id mapping lives in Python: dropping each prototype's vertex
    offset must be caught by the vertex-id pin."""
    import numpy as np

    def no_offset(scene):
        per = [np.asarray(t, np.int64) for _, t in scene.protos]
        return np.concatenate([per[m] for m in scene.inst_mesh])

    monkeypatch.setattr(O, "tri_vertex_ids", no_offset)
    assert pins.pin_vertex_ids()
