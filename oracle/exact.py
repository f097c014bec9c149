"""Exact rational nearest hit for tiny scenes (test infrastructure only).

Every FP32 input (vertex, origin, direction, near, far) is converted to the
rational number it represents, and the ray/triangle intersection is evaluated
with ``fractions.Fraction``: no rounding anywhere.  This pins the FP64 oracle:
on rays whose exact decision margins exceed a tiny threshold the oracle must
pick the same triangle, and its t must agree to FP64 accuracy.

Intersection definition used here (barycentric form, written independently of
the oracle's Moller-Trumbore code): the ray o + t d meets the plane of triangle
(a, b, c) where  o + t d = a + u (b - a) + v (c - a); solving the 3x3 system by
Cramer's rule gives t, u, v; the ray hits if the system is non-singular,
u >= 0, v >= 0, u + v <= 1 and near <= t <= far.  Nearest hit = smallest t,
then smallest triangle index.
"""
from __future__ import annotations

from fractions import Fraction as F
from typing import List, Optional, Sequence, Tuple


def _det3(c0, c1, c2):
    """Determinant of the 3x3 matrix with columns c0, c1, c2."""
    return (c0[0] * (c1[1] * c2[2] - c1[2] * c2[1])
            - c1[0] * (c0[1] * c2[2] - c0[2] * c2[1])
            + c2[0] * (c0[1] * c1[2] - c0[2] * c1[1]))


def intersect(tri: Sequence[float], o: Sequence[float], d: Sequence[float]):
    """Exact (t, u, v) of the ray against the triangle's plane, or None if the
    ray is parallel to the plane (singular system)."""
    a = [F(float(x)) for x in tri[0:3]]
    b = [F(float(x)) for x in tri[3:6]]
    c = [F(float(x)) for x in tri[6:9]]
    O = [F(float(x)) for x in o]
    D = [F(float(x)) for x in d]
    e1 = [b[i] - a[i] for i in range(3)]
    e2 = [c[i] - a[i] for i in range(3)]
    rhs = [O[i] - a[i] for i in range(3)]
    # columns: e1 * u + e2 * v - D * t = rhs
    negD = [-x for x in D]
    den = _det3(e1, e2, negD)
    if den == 0:
        return None
    u = _det3(rhs, e2, negD) / den
    v = _det3(e1, rhs, negD) / den
    t = _det3(e1, e2, rhs) / den
    return t, u, v


def nearest(tris: List[Sequence[float]], o, d, near: float, far: float):
    """Exact nearest hit: (index, t, u, v, margin) with index -1 on a miss.

    ``margin`` is the smallest exact distance of any triangle's acceptance
    decision from its boundary (u, v, 1-u-v, (t-near)/|t|, (far-t)/|t|) and of
    the winner's t from any other accepted triangle's t (relative); a ray whose
    margin is tiny can legitimately be decided either way by rounded
    arithmetic."""
    N, Fr = F(float(near)), F(float(far))
    best = None
    margin = None
    accepted = []
    for k, tri in enumerate(tris):
        r = intersect(tri, o, d)
        if r is None:
            continue
        t, u, v = r
        w = 1 - u - v
        tt = abs(t) if t != 0 else F(1)
        dec = min(abs(u), abs(v), abs(w), abs(t - N) / tt, abs(Fr - t) / tt)
        margin = dec if margin is None else min(margin, dec)
        if u >= 0 and v >= 0 and w >= 0 and N <= t <= Fr:
            accepted.append((t, k, u, v))
    if accepted:
        accepted.sort(key=lambda x: (x[0], x[1]))
        t, k, u, v = accepted[0]
        for t2, k2, _, _ in accepted[1:]:
            gap = (t2 - t) / t
            margin = gap if margin is None else min(margin, gap)
        best = (k, t, u, v)
    if margin is None:
        margin = F(1)
    if best is None:
        return -1, None, None, None, margin
    return best[0], best[1], best[2], best[3], margin
