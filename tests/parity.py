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
