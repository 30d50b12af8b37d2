"""Pins of the oracle's removal of false intersections (Test Results, Hairball;
Conclusions and Future Work): its FP32 triangle/cell test against an exact
rational clip of the triangle by the cell, on non-dyadic grids.

The FP32 test must never drop a cell the triangle touches (no false
negatives), and may keep only cells within the stated margin of the triangle.
"""
from fractions import Fraction

import numpy as np
import pytest

import fp32_model
import oracle
from brute import triangle_touches_box
from paper_2403_10647_amd import scenes

MARGIN = Fraction(1, 64)   # cells, on every side of a cell


def _soup(tri_coords):
    v = np.asarray(tri_coords, np.float64).reshape(-1, 3, 3)
    return scenes.soup_from_vertices(v)


def _exact_u(verts, tri, lo, hi, res):
    """Rational values of the FP32 grid coordinates, from the exact rounding model."""
    u = []
    for j in range(3):
        row = []
        for a in range(3):
            inv = fp32_model.inv_cell(lo[a], hi[a], int(res[a]))
            s = fp32_model.rn32(fp32_model.exact(verts[a][int(tri[j])]) - fp32_model.exact(lo[a]))
            row.append(fp32_model.rn32(s * inv))
        u.append(tuple(row))
    return u


def _check_scene(verts, tris, lo, hi, res):
    box_lo, box_m, count = oracle.count_cells(verts, tris, lo, hi, res)
    cells, objs, kept = oracle.make_pairs_culled(verts, tris, lo, hi, res, box_lo, box_m, count)
    rx, ry = int(res[0]), int(res[1])
    by_obj = {}
    for c, o in zip(cells.tolist(), objs.tolist()):
        by_obj.setdefault(o, []).append(c)
    tested = dropped = 0
    for t in range(tris.shape[0]):
        u_or, inside = oracle.grid_coords(verts, tris[t], lo, hi, res)
        u = _exact_u(verts, tris[t], lo, hi, res)
        assert all(Fraction(float(u_or[j][a])) == u[j][a] for j in range(3) for a in range(3))
        box = [(int(box_lo[t, 0]) + x, int(box_lo[t, 1]) + y, int(box_lo[t, 2]) + z)
               for z in range(int(box_m[t, 2])) for y in range(int(box_m[t, 1])) for x in range(int(box_m[t, 0]))]
        got = by_obj.get(t, [])
        assert got == sorted(got) and int(kept[t]) == len(got)
        ids = [x + rx * (y + ry * z) for x, y, z in box]
        if not inside or int(count[t]) <= 2:
            assert got == ids          # the whole box is kept
            continue
        tested += 1
        for (x, y, z), cid in zip(box, ids):
            touch = triangle_touches_box(u, (x, y, z), (x + 1, y + 1, z + 1))
            near = triangle_touches_box(u, (x - 2 * MARGIN, y - 2 * MARGIN, z - 2 * MARGIN),
                                        (x + 1 + 2 * MARGIN, y + 1 + 2 * MARGIN, z + 1 + 2 * MARGIN))
            k = cid in got
            assert not touch or k, ("dropped a touched cell", t, (x, y, z))
            assert not k or near, ("kept a cell beyond the margin", t, (x, y, z))
            dropped += not k
    return tested, dropped


def _random_scene(rng, n, lo, hi, spread):
    c = rng.uniform(lo, hi, size=(n, 1, 3))
    off = rng.uniform(-spread, spread, size=(n, 3, 3))
    v = np.clip(c + off, lo, hi)
    return scenes.soup_from_vertices(v)


@pytest.mark.parametrize("seed", range(4))
def test_culling_against_exact_clipping(seed):
    rng = np.random.default_rng(100 + seed)
    lo = rng.uniform(-5, 5, size=3).astype(np.float32)
    hi = (lo + rng.uniform(3.3, 9.7, size=3)).astype(np.float32)
    res = rng.integers(5, 14, size=3).astype(np.uint32)
    verts, tris = _random_scene(rng, 60, lo.astype(np.float64), hi.astype(np.float64), 2.5)
    tested, dropped = _check_scene(verts, tris, lo, hi, res)
    assert tested > 20 and dropped > 50


def test_long_thin_diagonal_triangles():
    # Hairball-like slivers across the grid: most of their boxes are empty of them
    rng = np.random.default_rng(7)
    lo, hi, res = np.zeros(3, np.float32), np.full(3, 7.3, np.float32), np.array([9, 11, 10], np.uint32)
    tri = []
    for _ in range(25):
        a = rng.uniform(0.2, 7.0, size=3)
        b = rng.uniform(0.2, 7.0, size=3)
        w = rng.normal(size=3) * 0.05
        tri.append([a, b, b + w])
    verts, tris = _soup(tri)
    tested, dropped = _check_scene(verts, tris, lo, hi, res)
    assert tested == 25 and dropped > 1000


def test_triangle_through_cell_corners_keeps_touched_cells():
    # in a 4 x 4 x 1 grid of unit cells, the triangle (0.5, 0.5), (3.5, 0.5),
    # (0.5, 3.5) has its long edge on x + y = 4, which passes exactly through
    # the corners (1, 3), (2, 2), (3, 1): it touches the 13 cells with x + y <= 4
    # of its 16-cell box and misses (2, 3), (3, 2), (3, 3)
    lo, hi, res = np.zeros(3, np.float32), np.array([4, 4, 1], np.float32), np.array([4, 4, 1], np.uint32)
    verts, tris = _soup([[[0.5, 0.5, 0.5], [3.5, 0.5, 0.5], [0.5, 3.5, 0.5]]])
    box_lo, box_m, count = oracle.count_cells(verts, tris, lo, hi, res)
    assert count.tolist() == [16]
    cells, objs, kept = oracle.make_pairs_culled(verts, tris, lo, hi, res, box_lo, box_m, count)
    got = sorted((c % 4, c // 4) for c in cells.tolist())
    assert got == sorted((x, y) for x in range(4) for y in range(4) if x + y <= 4)
    assert kept.tolist() == [13]
    _check_scene(verts, tris, lo, hi, res)


def test_vertex_cells_are_always_kept_and_boxes_shrink():
    s = scenes.make_scene("mixed", seed=2, ntris=3000)
    box_lo, box_m, count = oracle.count_cells(s.verts, s.tris, s.lo, s.hi, s.res)
    cells, objs, kept = oracle.make_pairs_culled(s.verts, s.tris, s.lo, s.hi, s.res, box_lo, box_m, count)
    assert (kept >= 1).all() and (kept <= count).all() and kept.sum() < count.sum()
    rx, ry = int(s.res[0]), int(s.res[1])
    inv = oracle.inv_cell(s.lo, s.hi, s.res)
    kept_set = set(zip(cells.tolist(), objs.tolist()))
    for t in range(0, 3000, 7):
        for j in range(3):
            v = s.tris[t, j]
            xyz = [min(max(int(np.floor(np.float32(np.float32(s.verts[a][v] - s.lo[a]) * inv[a]))), 0), int(s.res[a]) - 1)
                   for a in range(3)]
            assert (xyz[0] + rx * (xyz[1] + ry * xyz[2]), t) in kept_set


def test_outside_and_small_triangles_keep_their_box():
    lo, hi, res = np.zeros(3, np.float32), np.full(3, 8, np.float32), np.full(3, 8, np.uint32)
    verts, tris = _soup([
        [[-1.0, 0.5, 0.5], [6.5, 0.5, 0.5], [0.5, 6.5, 0.5]],   # reaches below lo: whole box
        [[1.5, 1.5, 1.5], [2.5, 1.5, 1.5], [1.5, 1.7, 1.5]],    # two cells: whole box
        [[0.5, 0.5, 0.5], [7.5, 7.5, 7.5], [0.5, 0.6, 0.5]],    # a long sliver: culled
    ])
    box_lo, box_m, count = oracle.count_cells(verts, tris, lo, hi, res)
    cells, objs, kept = oracle.make_pairs_culled(verts, tris, lo, hi, res, box_lo, box_m, count)
    assert kept[0] == count[0] and kept[1] == count[1] == 2
    assert kept[2] < count[2] // 10
    _check_scene(verts, tris, lo, hi, res)


def test_culled_build_is_the_sorted_kept_set():
    s = scenes.make_scene("arch", seed=1, ntris=20_000)
    c, o, r, nbox = oracle.build_scene_culled(s)
    g = oracle.build_scene(s, stages=True)
    assert nbox == g.npairs and len(c) < nbox
    box_lo, box_m, count = g.box_lo, g.box_m, g.count
    c0, o0, kept = oracle.make_pairs_culled(s.verts, s.tris, s.lo, s.hi, s.res, box_lo, box_m, count)
    order = np.lexsort((o0, c0))
    assert np.array_equal(c, c0[order]) and np.array_equal(o, o0[order])
    # the kept pairs are a subset of the box pairs
    full = set(zip(g.cells.tolist(), g.objs.tolist()))
    assert all(p in full for p in zip(c.tolist(), o.tolist()))
    rr = r.reshape(-1, 2).astype(np.int64)
    assert rr[0, 0] == 0 and rr[-1, 1] == len(c) and np.array_equal(rr[1:, 0], rr[:-1, 1])
    assert np.array_equal(rr[:, 1] - rr[:, 0], np.bincount(c, minlength=rr.shape[0]))


def test_exact_clipper_hand_cases():
    # the brute force itself: touching at a corner, an edge crossing a face,
    # a gap, a triangle inside, a box inside a large triangle
    box = ((0, 0, 0), (1, 1, 1))
    assert triangle_touches_box([(1, 1, 1), (2, 1, 1), (2, 2, 2)], *box)                  # shares a corner
    assert not triangle_touches_box([(Fraction(11, 10), 0, 0), (2, 1, 1), (2, 0, 1)], *box)  # beyond x = 1
    assert triangle_touches_box([(Fraction(1, 2), Fraction(1, 2), -1), (Fraction(1, 2), Fraction(1, 2), 2),
                                 (3, 3, 3)], *box)                                         # pierces the box
    assert triangle_touches_box([(Fraction(1, 4),) * 3, (Fraction(1, 2),) * 3, (Fraction(1, 3), 0, 0)], *box)
    assert triangle_touches_box([(-5, -5, Fraction(1, 2)), (9, -5, Fraction(1, 2)), (-5, 9, Fraction(1, 2))], *box)
    # the plane x + y + z = 3.5 passes near the corner (1, 1, 1) but misses the box
    assert not triangle_touches_box([(Fraction(7, 2), 0, 0), (0, Fraction(7, 2), 0), (0, 0, Fraction(7, 2))], *box)
    assert triangle_touches_box([(3, 0, 0), (0, 3, 0), (0, 0, 3)], *box)                  # through (1, 1, 1)
