"""Parity contract between GPU outputs and the oracle.

On every *robust* ray (the oracle's margins: barycentric > 1e-4, depth gap
> 1e-4 relative, range limits > 1e-4 relative, grazing cosine >= 1e-3; misses
with no near-miss candidate): hit/miss status, triangle id and segmentation
label are bit-exact and depth is within 1e-5 relative.  Borderline rays are
counted by class and reported with their agreement, not asserted.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O

DEPTH_RTOL = 1e-5


def compare(gpu: dict, ora: "O.Render") -> dict:
    depth = np.asarray(gpu["depth"], np.float32)
    tri = np.asarray(gpu["tri"]) if gpu.get("tri") is not None else None
    seg = np.asarray(gpu["seg"])
    cls = ora.cls
    robust = (cls & O.BORDER_MASK) == 0
    hit_o = ora.tri >= 0
    hit_g = depth >= 0
    rep = dict(n=len(depth), robust=int(robust.sum()))
    rep["hitmiss_mismatch"] = int(np.sum(robust & (hit_o != hit_g)))
    if tri is not None:
        rep["tri_mismatch"] = int(np.sum(robust & (tri != ora.tri)))
    rep["seg_mismatch"] = int(np.sum(robust & (seg != ora.seg)))
    both = robust & hit_o & hit_g
    rel = np.abs(depth[both].astype(np.float64) - ora.t[both]) / ora.t[both]
    rep["max_rel_depth"] = float(rel.max()) if rel.size else 0.0
    miss = robust & ~hit_o
    rep["miss_sentinel_bad"] = int(np.sum(miss & ((depth != -1.0) | (seg != -1))))
    # borderline rays, by class
    border = ~robust
    rep["borderline"] = int(border.sum())
    for name, bit in (("bary", O.B_BARY), ("gap", O.B_GAP), ("range", O.B_RANGE), ("graze", O.B_GRAZE),
                      ("nearmiss", O.B_NEARMISS)):
        rep[f"border_{name}"] = int(np.sum((cls & bit) != 0))
    if tri is not None:
        rep["border_tri_agree"] = int(np.sum(border & (tri == ora.tri)))
        rep["all_tri_agree"] = int(np.sum(tri == ora.tri))
    bh = border & hit_o & hit_g & ((tri == ora.tri) if tri is not None else True)
    rel_b = np.abs(depth[bh].astype(np.float64) - ora.t[bh]) / ora.t[bh]
    rep["border_max_rel_depth"] = float(rel_b.max()) if rel_b.size else 0.0
    if gpu.get("hit_xyz") is not None:
        h = np.asarray(gpu["hit_xyz"], np.float64).reshape(-1, 3)
        ok = both & ((tri == ora.tri) if tri is not None else True)
        err = np.abs(h[ok] - ora.hit[ok].astype(np.float64))
        scale = np.maximum(np.abs(ora.raw["hit"][ok]), 1.0)
        rep["max_hit_err_ulps"] = float((err / (scale * 2.0 ** -24)).max()) if err.size else 0.0
        rep["miss_hit_not_nan"] = int(np.sum(miss & ~np.all(np.isnan(h), axis=1)))
    return rep


def assert_contract(rep: dict) -> None:
    assert rep["hitmiss_mismatch"] == 0, rep
    assert rep.get("tri_mismatch", 0) == 0, rep
    assert rep["seg_mismatch"] == 0, rep
    assert rep["max_rel_depth"] <= DEPTH_RTOL, rep
    assert rep["miss_sentinel_bad"] == 0, rep
    if "max_hit_err_ulps" in rep:
        assert rep["max_hit_err_ulps"] <= 4.0, rep
        assert rep["miss_hit_not_nan"] == 0, rep


# Further data types of a hit: both sides evaluate the same FP64 expressions on
# identical FP32 vertices and rays and differ only in operation order (a few
# FP64 ulps), so after the single rounding to FP32 they agree to within one
# FP32 ulp: 2^-22 absolute for unit-range quantities (normal components, u, v),
# 2^-21 relative for sensor-frame points.
TOL_UNIT = 2.0 ** -22
TOL_POINT_REL = 2.0 ** -21


def compare_extras(gpu: dict, ora: "O.Render") -> dict:
    """Normals, barycentrics, sensor-frame points and vertex ids on every ray
    where GPU and oracle picked the same triangle (all robust hits), plus the
    miss sentinels on every ray both call a miss."""
    tri = np.asarray(gpu["tri"])
    same = (tri == ora.tri) & (tri >= 0)
    miss = (tri < 0) & (ora.tri < 0)
    rep = dict(compared=int(same.sum()))
    robust = (ora.cls & O.BORDER_MASK) == 0
    rep["robust_hits_not_compared"] = int(np.sum(robust & (ora.tri >= 0) & ~same))
    if gpu.get("normal") is not None:
        e = np.abs(gpu["normal"][same].astype(np.float64) - ora.normal[same])
        rep["normal_max_abs"] = float(e.max()) if e.size else 0.0
        rep["normal_bad"] = int(np.sum(~(e <= TOL_UNIT).all(1)))
        rep["normal_miss_bad"] = int(np.sum(~np.isnan(gpu["normal"][miss]).all(1)))
    if gpu.get("bary") is not None:
        e = np.abs(gpu["bary"][same].astype(np.float64) - ora.bary[same])
        rep["bary_max_abs"] = float(e.max()) if e.size else 0.0
        rep["bary_bad"] = int(np.sum(~(e <= TOL_UNIT).all(1)))
        rep["bary_miss_bad"] = int(np.sum(~np.isnan(gpu["bary"][miss]).all(1)))
    if gpu.get("point") is not None:
        g, o = gpu["point"][same].astype(np.float64), ora.point[same].astype(np.float64)
        scale = np.maximum(np.abs(o).max(1, initial=0.0), 1e-30)
        e = np.abs(g - o).max(1, initial=0.0) / scale
        rep["point_max_rel"] = float(e.max()) if e.size else 0.0
        rep["point_bad"] = int(np.sum(~(e <= TOL_POINT_REL)))
        rep["point_miss_bad"] = int(np.sum(~np.isnan(gpu["point"][miss]).all(1)))
    if gpu.get("vert") is not None:
        rep["vert_bad"] = int(np.sum(np.any(gpu["vert"][same] != ora.vert[same], 1)))
        rep["vert_miss_bad"] = int(np.sum(np.any(gpu["vert"][miss] != -1, 1)))
    return rep


def assert_extras(rep: dict) -> None:
    assert rep["robust_hits_not_compared"] == 0, rep
    for k, v in rep.items():
        if k.endswith("_bad"):
            assert v == 0, (k, rep)
