"""Exact rational geometry used to pin the oracle (pure Python ``fractions``).

These routines decide the same questions as the oracle by *different*
constructions, in exact arithmetic on the FP32/FP64 inputs:

* face vs closed box: clip the face polygon against the box's half-spaces
  (Sutherland-Hodgman), non-empty result = they meet;
* segment vs triangle / segment: solve the linear system by Cramer's rule;
* bin ranges: floor of the exact rational (x - lo) * B / (hi - lo).
"""
from __future__ import annotations

from fractions import Fraction as Fr
from typing import List, Optional, Sequence, Tuple


def fr(x) -> Fr:
    return Fr(float(x))


def clip_halfspace(poly: List[tuple], axis: int, bound: Fr, keep_ge: bool) -> List[tuple]:
    out: List[tuple] = []
    n = len(poly)
    for i in range(n):
        P, Qp = poly[i], poly[(i + 1) % n]
        inP = P[axis] >= bound if keep_ge else P[axis] <= bound
        inQ = Qp[axis] >= bound if keep_ge else Qp[axis] <= bound
        if inP:
            out.append(P)
        if inP != inQ:
            t = (bound - P[axis]) / (Qp[axis] - P[axis])
            out.append(tuple(P[k] + t * (Qp[k] - P[k]) for k in range(len(P))))
    return out


def face_meets_box(face: Sequence[Sequence[float]], m: Sequence[float], h: float) -> bool:
    """Does the closed face (segment or triangle) meet the closed cube [m-h, m+h]^D?"""
    dim = len(m)
    poly = [tuple(fr(v[a]) for a in range(dim)) for v in face]
    H = fr(h)
    for a in range(dim):
        M = fr(m[a])
        poly = clip_halfspace(poly, a, M - H, True)
        if not poly:
            return False
        poly = clip_halfspace(poly, a, M + H, False)
        if not poly:
            return False
    return True


def plane_meets_box(tri, m, h) -> bool:
    """Does the supporting plane of the triangle meet the closed cube?"""
    a, b, c = [[fr(x) for x in v] for v in tri]
    e1 = [b[i] - a[i] for i in range(3)]
    e2 = [c[i] - a[i] for i in range(3)]
    n = [e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]]
    H = fr(h)
    vals = []
    for sx in (-1, 1):
        for sy in (-1, 1):
            for sz in (-1, 1):
                p = [fr(m[0]) + sx * H, fr(m[1]) + sy * H, fr(m[2]) + sz * H]
                vals.append(sum(n[i] * (p[i] - a[i]) for i in range(3)))
    return min(vals) <= 0 <= max(vals)


def aabb_meets_box(face, m, h) -> bool:
    dim = len(m)
    H = fr(h)
    for a in range(dim):
        lo = min(fr(v[a]) for v in face)
        hi = max(fr(v[a]) for v in face)
        if lo > fr(m[a]) + H or hi < fr(m[a]) - H:
            return False
    return True


def _det3(c0, c1, c2) -> Fr:
    return (c0[0] * (c1[1] * c2[2] - c1[2] * c2[1])
            - c1[0] * (c0[1] * c2[2] - c0[2] * c2[1])
            + c2[0] * (c0[1] * c1[2] - c0[2] * c1[1]))


def segment_triangle(o, D, tri) -> Optional[Tuple[Fr, Fr, Fr]]:
    """Exact (t, u, v) with o + t D = a + u (b-a) + v (c-a), all in the closed ranges; else None."""
    o = [fr(x) for x in o]
    D = [fr(x) for x in D]
    a, b, c = [[fr(x) for x in v] for v in tri]
    e1 = [b[i] - a[i] for i in range(3)]
    e2 = [c[i] - a[i] for i in range(3)]
    nd = [-x for x in D]
    rhs = [o[i] - a[i] for i in range(3)]
    det = _det3(e1, e2, nd)
    if det == 0:
        return None
    u = _det3(rhs, e2, nd) / det
    v = _det3(e1, rhs, nd) / det
    t = _det3(e1, e2, rhs) / det
    if u < 0 or v < 0 or u + v > 1 or t < 0 or t > 1:
        return None
    return t, u, v


def segment_segment(o, D, seg) -> Optional[Tuple[Fr, Fr]]:
    """Exact (t, s) with o + t D = a + s (b - a), both in [0, 1]; else None."""
    o = [fr(x) for x in o]
    D = [fr(x) for x in D]
    a, b = [[fr(x) for x in v] for v in seg]
    e = [b[0] - a[0], b[1] - a[1]]
    # t D - s e = a - o
    det = D[0] * (-e[1]) - (-e[0]) * D[1]
    if det == 0:
        return None
    r = [a[0] - o[0], a[1] - o[1]]
    t = (r[0] * (-e[1]) - (-e[0]) * r[1]) / det
    s = (D[0] * r[1] - D[1] * r[0]) / det
    if t < 0 or t > 1 or s < 0 or s > 1:
        return None
    return t, s


def exact_bin(x, lo, hi, B) -> int:
    """floor((x - lo) * B / (hi - lo)) in exact arithmetic, clamped to [0, B-1]."""
    v = (fr(x) - fr(lo)) * B / (fr(hi) - fr(lo))
    i = v.numerator // v.denominator
    return max(0, min(B - 1, i))


def near_integer(x, lo, hi, B, tol=Fr(1, 10 ** 5)) -> bool:
    v = (fr(x) - fr(lo)) * B / (fr(hi) - fr(lo))
    r = v - (v.numerator // v.denominator)
    if r == 0:
        return False     # exactly on a boundary: no rounding can move it
    return r < tol or (1 - r) < tol
