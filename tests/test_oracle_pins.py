"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these checks re-types the oracle's formulas: they compare it against a
brute-force cell-by-cell construction in exact arithmetic, the cell counts of
the paper's Figure 1, closed-form properties of GlobalCoords, textbook library
routines for the scan, sort and range steps, and structural invariants.
"""
import math
import os

import numpy as np
import pytest

import oracle
import fp32_model
from brute import brute_pairs, dyadic_scene
from paper_2403_10647_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _soup(tri_coords):
    v = np.asarray(tri_coords, np.float64).reshape(-1, 3, 3)
    return scenes.soup_from_vertices(v)


# --- brute force on tiny dyadic scenes -------------------------------------------------

@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("grid", [((0, 0, 0), (8, 8, 8), (8, 8, 8)),
                                  ((-4, 0, 2), (4, 8, 6), (16, 4, 8)),
                                  ((0, 0, 0), (8, 8, 8), (1, 8, 2))])
def test_oracle_equals_brute_force(seed, grid):
    lo, hi, res = (np.asarray(x, np.float32) for x in grid)
    res = res.astype(np.uint32)
    rng = np.random.default_rng(seed)
    verts, tris = dyadic_scene(rng, 40, float(lo.min()), float(hi.max()), spread=1.5)
    g = oracle.build_stages(verts, tris, lo, hi, res)
    want = brute_pairs(verts, tris, lo, hi, res)
    got = list(zip(g.cells.tolist(), g.objs.tolist()))
    assert got == want
    # ranges against a textbook binary search on the brute-force cell list
    bc = np.asarray([c for c, _ in want], np.int64)
    ncell = int(np.prod(res.astype(np.int64)))
    cells = np.arange(ncell)
    begin = np.searchsorted(bc, cells, side="left")
    end = np.searchsorted(bc, cells, side="right")
    assert np.array_equal(g.ranges[0::2], begin) and np.array_equal(g.ranges[1::2], end)


def test_on_face_and_out_of_bounds_points():
    # 8 cells of side 1 on [0, 8]: a point on a face belongs to the upper cell,
    # points outside the bounds are clamped onto the boundary cells.
    lo, hi, res = np.zeros(3, np.float32), np.full(3, 8, np.float32), np.full(3, 8, np.uint32)
    verts, tris = _soup([
        [[3, 3, 3], [3, 3, 3], [3, 3, 3]],            # exactly on a corner -> cell (3,3,3)
        [[8, 8, 8], [8, 8, 8], [8, 8, 8]],            # on hi -> last cell
        [[-5, -5, -5], [-1, -2, -3], [-4, -4, -4]],   # entirely below lo -> cell 0
        [[2.5, 0, 0], [4, 0, 0], [3.5, 0, 0]],        # x in [2.5, 4] -> cells 2,3,4
        [[20, 1, 1], [30, 1, 1], [40, 1, 1]],         # beyond hi -> clamped onto x = 7
    ])
    box_lo, box_m, count = oracle.count_cells(verts, tris, lo, hi, res)
    assert count.tolist() == [1, 1, 1, 3, 1]
    assert box_lo[0].tolist() == [3, 3, 3] and box_lo[1].tolist() == [7, 7, 7]
    assert box_lo[2].tolist() == [0, 0, 0] and box_lo[3].tolist() == [2, 0, 0]
    assert box_lo[4].tolist() == [7, 1, 1]


def test_nan_and_inf_coordinates():
    lo, hi, res = np.zeros(3, np.float32), np.full(3, 8, np.float32), np.full(3, 8, np.uint32)
    nan, inf = float("nan"), float("inf")
    verts, tris = _soup([
        [[nan, 1.5, 1.5], [2.5, 1.5, 1.5], [5.5, 1.5, 1.5]],   # NaN ignored: x cells 2..5
        [[nan, 1, 1], [nan, 1, 1], [nan, 1, 1]],               # all NaN -> cell 0
        [[-inf, 1, 1], [0.5, 1, 1], [0.5, 1, 1]],              # -inf -> cell 0
        [[inf, 1, 1], [0.5, 1, 1], [0.5, 1, 1]],               # +inf -> cell 7: x 0..7
    ])
    box_lo, box_m, count = oracle.count_cells(verts, tris, lo, hi, res)
    assert count.tolist() == [4, 1, 1, 8]
    assert box_lo[:, 0].tolist() == [2, 0, 0, 0]


# --- the FP32 map on non-dyadic grids, against an exact rational model ----------------------

def _face_points(rng, lo, hi, res, nface=24):
    """Points at, and one or two ulps beside, the cell faces of one axis (plus random
    points and the bounds themselves), as float32."""
    pts = [lo, hi, np.nextafter(lo, np.float32(-np.inf)), np.nextafter(hi, np.float32(np.inf))]
    for k in rng.integers(0, res + 1, size=nface):
        p = np.float32(float(lo) + int(k) * (float(hi) - float(lo)) / int(res))
        for step in range(-2, 3):
            q = p
            for _ in range(abs(step)):
                q = np.nextafter(q, np.float32(np.inf if step > 0 else -np.inf))
            pts.append(q)
    pts += list(rng.uniform(float(lo), float(hi), size=8).astype(np.float32))
    return np.asarray(pts, np.float32)


def _non_dyadic_grid(rng):
    lo = rng.uniform(-60, 60, size=3).astype(np.float32)
    ext = rng.uniform(0.3, 150, size=3)
    hi = (lo.astype(np.float64) + ext).astype(np.float32)
    res = rng.integers(3, 1025, size=3)
    res = np.where((res & (res - 1)) == 0, res + 1, res).astype(np.uint32)   # no powers of two
    return lo, hi, res


def test_fp32_map_matches_rational_model_at_cell_faces():
    # the map is a fixed FP32 sequence (Section 3 leaves it open; the reading is
    # floor((p - lo) * inv) with inv = res / (hi - lo), each step rounded once):
    # every box corner the oracle reports must equal that sequence evaluated in
    # exact rationals with an explicit round-to-nearest-even, on grids whose inv
    # is not a power of two and on points at and beside the cell faces.
    rng = np.random.default_rng(11)
    differs = 0
    checked = 0
    for _ in range(12):
        lo, hi, res = _non_dyadic_grid(rng)
        axes = [_face_points(rng, lo[a], hi[a], int(res[a])) for a in range(3)]
        n = max(len(x) for x in axes)
        picks = [rng.choice(axes[a], size=(n, 3)) for a in range(3)]
        # vertex j of triangle t on axis a is picks[a][t, j]
        verts = np.stack([picks[a].reshape(-1) for a in range(3)]).astype(np.float32)
        tris = np.arange(3 * n, dtype=np.uint32).reshape(n, 3)
        box_lo, box_m, _ = oracle.count_cells(verts, tris, lo, hi, res)
        for a in range(3):
            memo = {}

            def model(p, a=a):
                key = float(p)
                if key not in memo:
                    memo[key] = (fp32_model.cell_fp32(p, lo[a], hi[a], int(res[a])),
                                 fp32_model.cell_exact(p, lo[a], hi[a], int(res[a])))
                return memo[key]
            for t in range(n):
                pmin, pmax = picks[a][t].min(), picks[a][t].max()
                want_lo, ex_lo = model(pmin)
                want_hi, ex_hi = model(pmax)
                assert int(box_lo[t, a]) == want_lo, (a, float(pmin), lo[a], hi[a], res[a])
                assert int(box_lo[t, a]) + int(box_m[t, a]) - 1 == want_hi, (a, float(pmax), lo[a], hi[a], res[a])
                checked += 2
            differs += sum(1 for f, e in memo.values() if f != e)
    # the inputs do reach the cases where rounding decides the cell
    assert checked > 9000 and differs >= 100, (checked, differs)


def test_fp32_map_face_case_rounds_up():
    # (p - lo) * inv is just below 4 in exact arithmetic but rounds to 4.0 in
    # FP32: the contract's sequence puts the point in cell 4, exact arithmetic in 3
    lo, hi, res = np.zeros(3, np.float32), np.full(3, np.float32(17.219383)), np.full(3, 112, np.uint32)
    p = np.float32(0.61497796)
    assert fp32_model.cell_fp32(p, lo[0], hi[0], 112) == 4
    assert fp32_model.cell_exact(p, lo[0], hi[0], 112) == 3
    verts, tris = _soup([[[p, p, p], [p, p, p], [p, p, p]]])
    box_lo, box_m, count = oracle.count_cells(verts, tris, lo, hi, res)
    assert box_lo[0].tolist() == [4, 4, 4] and count.tolist() == [1]
    assert np.float32(oracle.inv_cell(lo, hi, res)[0]) == np.float32(fp32_model.inv_cell(lo[0], hi[0], 112))


def test_rational_rounding_model_matches_ieee_binary32():
    # the model itself, against the host's binary32 arithmetic (normal,
    # subnormal and overflowing results)
    rng = np.random.default_rng(5)
    a = (rng.standard_normal(3000) * 10.0 ** rng.integers(-30, 30, 3000)).astype(np.float32)
    b = (rng.standard_normal(3000) * 10.0 ** rng.integers(-30, 30, 3000)).astype(np.float32)
    with np.errstate(all="ignore"):
        for hw, ex in ((a * b, lambda x, y: x * y), (a / b, lambda x, y: x / y), (a - b, lambda x, y: x - y)):
            for x, y, h in zip(a, b, hw):
                m = fp32_model.rn32(ex(fp32_model.exact(x), fp32_model.exact(y)))
                if np.isinf(h):
                    assert m == (math.inf if h > 0 else -math.inf)
                else:
                    assert m == fp32_model.exact(h)


def test_invalid_grid_and_bad_index():
    verts, tris = _soup([[[0, 0, 0], [1, 1, 1], [2, 2, 2]]])
    ok = (np.zeros(3, np.float32), np.ones(3, np.float32), np.full(3, 4, np.uint32))
    with pytest.raises(oracle.OracleError) as e:
        oracle.count_cells(verts, tris, ok[0], ok[0], ok[2])       # lo == hi
    assert e.value.status == -1
    with pytest.raises(oracle.OracleError):
        oracle.count_cells(verts, tris, ok[0], ok[1], np.array([4, 0, 4], np.uint32))
    with pytest.raises(oracle.OracleError):
        oracle.count_cells(verts, tris, ok[0], ok[1], np.array([4, 1025, 4], np.uint32))
    bad = tris.copy()
    bad[0, 2] = 3
    with pytest.raises(oracle.OracleError) as e:
        oracle.count_cells(verts, bad, *ok)
    assert e.value.status == -5


def test_overflow_is_reported():
    # 5 triangles spanning a 1024^3 grid give NO = 5 * 2^30 > 2^32 - 1.
    verts, tris = _soup([[[0, 0, 0], [1, 1, 1], [0, 1, 0]]] * 5)
    lo, hi, res = np.zeros(3, np.float32), np.ones(3, np.float32), np.full(3, 1024, np.uint32)
    _, _, count = oracle.count_cells(verts, tris, lo, hi, res)
    assert count.tolist() == [1 << 30] * 5
    _, no = oracle.exclusive_sum(count)
    assert no == 5 << 30
    with pytest.raises(oracle.OracleError) as e:
        oracle.build(verts, tris, lo, hi, res)
    assert e.value.status == -3


# --- the paper's Figure 1 ---------------------------------------------------------------

def _figure1():
    grid, tris, want = None, [], []
    for line in open(os.path.join(GOLDEN, "figure1.txt")):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "grid":
            grid = [float(x) for x in f[1:]]
        elif f[0] == "tri":
            tris.append([float(x) for x in f[1:10]])
            want.append(int(f[10]))
    lo = np.asarray(grid[0:3], np.float32)
    hi = np.asarray(grid[3:6], np.float32)
    res = np.asarray(grid[6:9], np.uint32)
    return lo, hi, res, tris, want


def test_figure1_cell_counts():
    lo, hi, res, coords, want = _figure1()
    assert want == [1, 12]   # the caption's counts
    verts, tris = _soup(coords)
    g = oracle.build_stages(verts, tris, lo, hi, res)
    assert g.count.tolist() == want
    assert g.npairs == 13
    assert list(zip(g.cells.tolist(), g.objs.tolist())) == brute_pairs(verts, tris, lo, hi, res)
    # the 12 pairs of the large triangle, in object order, visit x fastest
    c = g.cells_objorder[1:].astype(np.int64)
    xyz = np.stack([c % 8, (c // 8) % 8, c // 64], axis=1)
    assert xyz[:3, 0].tolist() == [1, 2, 3] and set(xyz[:, 1]) == {2, 3} and set(xyz[:, 2]) == {3, 4}


# --- GlobalCoords ------------------------------------------------------------------------

def test_global_coords_enumerates_box_x_fastest():
    lo = np.array([5, 7, 11], np.uint32)
    for mx in range(1, 7):
        for my in range(1, 7):
            for mz in range(1, 7):
                m = np.array([mx, my, mz], np.uint32)
                got = [tuple(oracle.global_coords(lo, m, r)) for r in range(mx * my * mz)]
                want = [(5 + x, 7 + y, 11 + z) for z in range(mz) for y in range(my) for x in range(mx)]
                assert got == want


def test_global_coords_large_boxes():
    rng = np.random.default_rng(3)
    for _ in range(200):
        m = rng.integers(1, 1025, size=3).astype(np.uint32)
        while int(np.prod(m.astype(np.int64))) > (1 << 30):
            m = (m // 2 + 1).astype(np.uint32)
        lo = np.zeros(3, np.uint32)
        n = int(np.prod(m.astype(np.int64)))
        for rid in [0, n - 1, int(rng.integers(0, n))]:
            x, y, z = (int(v) for v in oracle.global_coords(lo, m, rid))
            assert 0 <= x < m[0] and 0 <= y < m[1] and 0 <= z < m[2]
            # the enumeration is the mixed-radix expansion of rid
            q, rx = divmod(rid, int(m[0]))
            rz, ry = divmod(q, int(m[1]))
            assert (x, y, z) == (rx, ry, rz)


# --- scan, sort and range steps against textbook routines ---------------------------------

def test_exclusive_sum_matches_cumsum():
    rng = np.random.default_rng(0)
    for n in [0, 1, 7, 1000, 65537]:
        cnt = rng.integers(0, 1 << 30, size=n).astype(np.uint32)
        start, no = oracle.exclusive_sum(cnt)
        cs = np.cumsum(cnt.astype(np.uint64))
        assert no == (int(cs[-1]) if n else 0)
        assert np.array_equal(start, np.concatenate([[0], cs[:-1]]).astype(np.uint64) if n else start)


def test_sort_matches_lexsort():
    rng = np.random.default_rng(1)
    cells = rng.integers(0, 50, size=5000).astype(np.uint32)
    objs = np.sort(rng.integers(0, 1 << 31, size=5000)).astype(np.uint32)  # object order
    sc, so = oracle.sort_pairs(cells, objs)
    order = np.lexsort((objs, cells))
    assert np.array_equal(sc, cells[order]) and np.array_equal(so, objs[order])


def test_ranges_match_bincount():
    rng = np.random.default_rng(2)
    cells = np.sort(rng.integers(0, 300, size=4000)).astype(np.uint32)
    r = oracle.ranges(cells, 400).reshape(-1, 2).astype(np.int64)
    cnt = np.bincount(cells, minlength=400)
    assert np.array_equal(r[:, 1] - r[:, 0], cnt)
    assert r[0, 0] == 0 and r[-1, 1] == 4000 and np.array_equal(r[1:, 0], r[:-1, 1])


# --- invariants on the synthetic workloads -------------------------------------------------

def _check_invariants(s, g):
    res = s.res.astype(np.int64)
    assert g.npairs == int(g.count.astype(np.int64).sum())
    assert np.array_equal(g.count.astype(np.int64), np.prod(g.box_m.astype(np.int64), axis=1))
    assert (g.count >= 1).all()
    c = g.cells.astype(np.int64)
    o = g.objs.astype(np.int64)
    assert (np.diff(c) >= 0).all()
    same = np.diff(c) == 0
    assert (np.diff(o)[same] > 0).all()              # ascending and duplicate-free per cell
    # each pair's cell lies inside its object's cell box
    x, y, z = c % res[0], (c // res[0]) % res[1], c // (res[0] * res[1])
    bl = g.box_lo[o].astype(np.int64)
    bh = bl + g.box_m[o].astype(np.int64) - 1
    for a, v in enumerate((x, y, z)):
        assert ((v >= bl[:, a]) & (v <= bh[:, a])).all()
    # every object appears exactly count times
    assert np.array_equal(np.bincount(o, minlength=s.ntris), g.count.astype(np.int64))
    # the sorted list is a permutation of the object-order list
    a = np.sort(g.cells_objorder.astype(np.int64) * s.ntris + g.objs_objorder)
    b = c * s.ntris + o
    assert np.array_equal(a, b)
    # ranges tile [0, NO) and agree with a textbook search
    r = g.ranges.reshape(-1, 2).astype(np.int64)
    assert r[0, 0] == 0 and r[-1, 1] == g.npairs and np.array_equal(r[1:, 0], r[:-1, 1])
    probe = np.random.default_rng(0).integers(0, r.shape[0], size=2000)
    assert np.array_equal(r[probe, 0], np.searchsorted(c, probe, "left"))
    assert np.array_equal(r[probe, 1], np.searchsorted(c, probe, "right"))


def test_invariants_small_scene():
    s = scenes.make_scene("small")
    g = oracle.build_scene(s, stages=True)
    _check_invariants(s, g)
    assert 17000 < g.npairs < 18000


@pytest.mark.parametrize("name,n", [("mixed", 60_000), ("arch", 60_000)])
def test_invariants_scaled_scenes(name, n):
    s = scenes.make_scene(name, ntris=n)
    g = oracle.build_scene(s, stages=True)
    _check_invariants(s, g)


def test_batch_grid_invariants():
    for s in scenes.make_batch(0, ngrids=3, sizes=np.array([1000, 2500, 4000])):
        _check_invariants(s, oracle.build_scene(s, stages=True))


# --- Table 1 identities (statistics reporter) ----------------------------------------------

def _num(tok):
    mult = {"K": 1e3, "M": 1e6}.get(tok[-1], 1.0)
    body = tok[:-1] if tok[-1] in "KM" else tok
    dec = len(body.split(".")[1]) if "." in body else 0
    half = 0.5 * 10.0 ** (-dec) * mult
    return float(body) * mult, half


def test_table1_identities():
    from paper_2403_10647_amd import stats
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table1.txt")) if l.strip() and not l.startswith("#")]
    assert len(rows) == 7
    for name, tri, dims, cells, pe, ain, mxc, acell, mem in rows:
        T, dT = _num(tri)
        res = [int(d) for d in dims.split("x")]
        cl, dcl = _num(cells)
        pct, dpct = _num(pe)
        avg_items, davg_items = _num(ain)
        avg_cells, davg = _num(acell)
        mem_mb, dmem = _num(mem)
        ncell = math.prod(res)
        assert abs(ncell - cl) <= dcl, name
        no_lo, no_hi = (T - dT) * (acell_lo := avg_cells - davg), (T + dT) * (avg_cells + davg)
        # memory column = 4 (cells + NO) bytes in MiB
        lo_row = stats.table1(res, T, no_lo, 1, int(mxc))
        hi_row = stats.table1(res, T, no_hi, 1, int(mxc))
        assert lo_row["memory_MiB"] - dmem <= mem_mb <= hi_row["memory_MiB"] + dmem, name
        # NO = nonEmpty * avg items per non-empty cell
        ne_lo = ncell * (1 - (pct + dpct) / 100)
        ne_hi = ncell * (1 - (pct - dpct) / 100)
        assert ne_lo * (avg_items - davg_items) <= no_hi and no_lo <= ne_hi * (avg_items + davg_items), name
        # the reporter's other columns are consistent with the printed row
        row = stats.table1(res, T, (no_lo + no_hi) / 2, int(round((ne_lo + ne_hi) / 2)), int(mxc))
        assert abs(row["pct_empty"] - pct) < 0.05, name
        assert abs(row["avg_cells_per_item"] - avg_cells) <= davg + 1e-9, name
        assert abs(row["avg_items_per_nonempty"] - avg_items) / avg_items < 0.01, name
    assert acell_lo > 0


def test_stats_from_ranges():
    from paper_2403_10647_amd import stats
    s = scenes.make_scene("small")
    g = oracle.build_scene(s, stages=True)
    row = stats.table1_from_ranges(s.res, s.ntris, g.ranges, g.count)
    assert row["cells"] == 32768
    assert math.isclose(row["avg_cells_per_item"], g.npairs / 4096)
    assert row["max_cells_per_item"] == int(g.count.max())
    assert math.isclose(row["memory_MiB"], 4 * (32768 + g.npairs) / 2 ** 20)


def test_probe_writes_nothing_and_empty_scene():
    # the sizing probe only reports NO; an empty scene builds to all-empty ranges
    verts, tris = np.zeros((3, 0), np.float32), np.zeros((0, 3), np.uint32)
    lo, hi, res = np.zeros(3, np.float32), np.ones(3, np.float32), np.array([2, 2, 7], np.uint32)
    assert oracle.probe_npairs(verts, tris, lo, hi, res) == 0
    c, o, r = oracle.build(verts, tris, lo, hi, res)
    assert len(c) == 0 and len(o) == 0 and r.shape == (56,) and not r.any()
    v2, t2 = _soup([[[0.1, 0.1, 0.1], [0.9, 0.9, 0.9], [0.5, 0.5, 0.5]]])
    assert oracle.probe_npairs(v2, t2, lo, hi, res) == 2 * 2 * 7
