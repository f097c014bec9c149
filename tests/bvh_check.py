"""CPU validator for a downloaded per-environment BVH (``rc_debug_bvh``)."""
from __future__ import annotations

import numpy as np

MAX_NODE_DEPTH = 18


def _expand_lo(x):
    x = np.float32(x)
    if abs(x) < np.float32(2.0 ** -100):
        return np.float32(-(2.0 ** -100))
    return np.nextafter(x, np.float32(-np.inf))


def _expand_hi(x):
    x = np.float32(x)
    if abs(x) < np.float32(2.0 ** -100):
        return np.float32(2.0 ** -100)
    return np.nextafter(x, np.float32(np.inf))


def leaf_decode(ref):
    code = ~int(ref)
    return code >> 3, (code & 7) + 1


def validate(bvh: dict, tris: np.ndarray) -> list:
    """Every triangle in exactly one leaf; each stored child box is the
    one-step outward expansion of the exact bounds of the child's triangles;
    parent links consistent; internal-node depth bounded."""
    errs = []
    n = len(tris)
    ids = bvh["leaf_ids"]
    if sorted(ids.tolist()) != list(range(n)):
        errs.append("leaf ids are not a permutation")
        return errs
    verts = tris.reshape(-1, 3, 3)
    seen = np.zeros(n, np.int32)
    root = bvh["root"]
    if n == 0:
        return errs
    if root < 0:
        first, cnt = leaf_decode(root)
        if first != 0 or cnt != n:
            errs.append("root leaf does not cover all triangles")
        return errs

    def bounds(ref, depth):
        if ref < 0:
            first, cnt = leaf_decode(ref)
            seen[first:first + cnt] += 1
            v = verts[ids[first:first + cnt]].reshape(-1, 3)
            return v.min(0), v.max(0)
        if depth > MAX_NODE_DEPTH:
            errs.append(f"node {ref} deeper than {MAX_NODE_DEPTH}")
        los, his = [], []
        for side in (0, 1):
            c = int(bvh["children"][ref, side])
            if c >= 0 and bvh["parent"][c] != ref:
                errs.append(f"parent of {c} is {bvh['parent'][c]} not {ref}")
            lo, hi = bounds(c, depth + 1)
            box = bvh["boxes"][ref, side]
            want = np.array([_expand_lo(x) for x in lo] + [_expand_hi(x) for x in hi], np.float32)
            if not np.array_equal(box, want):
                errs.append(f"node {ref} side {side}: box {box} != expanded bounds {want}")
            los.append(lo)
            his.append(hi)
        return np.minimum(*los), np.maximum(*his)

    if bvh["parent"][root] != -1:
        errs.append("root has a parent")
    bounds(root, 0)
    if not np.all(seen == 1):
        errs.append(f"leaf coverage wrong: {np.bincount(seen)}")
    return errs
