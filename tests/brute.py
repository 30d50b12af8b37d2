"""Brute-force grid construction for tiny scenes, independent of the oracle.

Every cell of the grid is tested against every triangle's bounding box with
exact rational arithmetic: cell x on an axis covers the half-open interval
[lo + x*w, lo + (x+1)*w) with w = (hi - lo) / res, except that cell 0 extends to
-inf and cell res-1 to +inf (points outside the grid are clamped onto it); a
triangle's closed interval [min p, max p] meets that cell iff
min p < upper and max p >= lower.  On dyadic inputs, where the FP32 map
floor((p - lo) * inv) is exact, this is the same cell set the paper's CountCells
and GlobalCoords enumerate.
"""
from fractions import Fraction

import numpy as np


def _axis_cells(pmin: Fraction, pmax: Fraction, lo: Fraction, w: Fraction, res: int):
    out = []
    for x in range(res):
        lower = None if x == 0 else lo + x * w
        upper = None if x == res - 1 else lo + (x + 1) * w
        below_upper = True if upper is None else pmin < upper
        above_lower = True if lower is None else pmax >= lower
        if below_upper and above_lower:
            out.append(x)
    return out


def brute_pairs(verts, tris, lo, hi, res):
    """Sorted list of (cell, obj) pairs, by testing every cell for every triangle."""
    res = [int(r) for r in res]
    lof = [Fraction(float(v)) for v in lo]
    w = [(Fraction(float(hi[a])) - lof[a]) / res[a] for a in range(3)]
    pairs = []
    for t, tri in enumerate(np.asarray(tris)):
        per_axis = []
        for a in range(3):
            ps = [Fraction(float(verts[a][int(i)])) for i in tri]
            per_axis.append(_axis_cells(min(ps), max(ps), lof[a], w[a], res[a]))
        for z in range(res[2]):
            for y in range(res[1]):
                for x in range(res[0]):
                    if x in per_axis[0] and y in per_axis[1] and z in per_axis[2]:
                        pairs.append((x + res[0] * (y + res[1] * z), t))
    pairs.sort()
    return pairs


def dyadic_scene(rng: np.random.Generator, ntris: int, lo: float, hi: float, spread: float,
                 step: float = 1.0 / 16):
    """Random triangles with coordinates on a 1/16 lattice, some outside [lo, hi]."""
    c = rng.uniform(lo - 1.0, hi + 1.0, size=(ntris, 1, 3))
    off = rng.uniform(-spread, spread, size=(ntris, 3, 3))
    v = np.round((c + off) / step) * step
    verts = np.ascontiguousarray(v.reshape(ntris * 3, 3).T.astype(np.float32))
    tris = np.arange(3 * ntris, dtype=np.uint32).reshape(ntris, 3)
    return verts, tris


def _clip(poly, axis, bound, keep_above):
    """Sutherland-Hodgman: the part of polygon poly (list of rational 3-points) on
    one closed side of the plane coordinate[axis] = bound."""
    def inside(p):
        return p[axis] >= bound if keep_above else p[axis] <= bound
    out = []
    n = len(poly)
    for i in range(n):
        p, q = poly[i], poly[(i + 1) % n]
        ip, iq = inside(p), inside(q)
        if ip:
            out.append(p)
        if ip != iq and p[axis] != q[axis]:
            t = (bound - p[axis]) / (q[axis] - p[axis])
            r = tuple(p[a] + t * (q[a] - p[a]) for a in range(3))
            if inside(r):
                out.append(r)
    return out


def triangle_touches_box(tri, lower, upper) -> bool:
    """Exact test: does the closed triangle (3 rational 3-points) meet the closed
    box [lower, upper]?  The triangle is clipped by the box's six half-spaces;
    they meet iff something is left."""
    poly = [tuple(Fraction(c) for c in p) for p in tri]
    for a in range(3):
        poly = _clip(poly, a, Fraction(lower[a]), True)
        if not poly:
            return False
        poly = _clip(poly, a, Fraction(upper[a]), False)
        if not poly:
            return False
    return True
