"""GPU parity of the build with false intersections removed (grid_build_culled)
against the oracle's culled build (Test Results, Hairball; Conclusions and
Future Work), bit for bit: the overlap test is a fixed sequence of FP32
operations on both sides, so the kept pair set is unique and the tolerance is
zero.  Scenes span several expansion tiles (4096 box pairs) with ragged tails;
the digit-width cases run zero to four radix passes over the kept pairs."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_2403_10647_amd import scenes

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_10647_amd import _lib
    _lib.lib()
    return _lib


def _say(*a):
    print(*a, flush=True)


def _scene(verts, tris, lo, hi, res, name="adhoc"):
    return scenes.Scene(name, np.ascontiguousarray(verts, np.float32), np.ascontiguousarray(tris, np.uint32),
                        np.asarray(lo, np.float32), np.asarray(hi, np.float32), np.asarray(res, np.uint32))


def _check(G, s):
    _say("culled build", s.name, s.ntris, list(map(int, s.res)))
    g = G.GridInput.from_scene(s)
    r, nbox = G.build_culled(g)
    c, o, rg = r.numpy()
    oc, oo, orr, obox = oracle.build_scene_culled(s)
    assert nbox == obox
    assert r.npairs == len(oc)
    assert np.array_equal(c, oc)
    assert np.array_equal(o, oo)
    assert np.array_equal(rg, orr)
    return r, nbox


@pytest.mark.parametrize("name,n", [("small", None), ("mixed", 100_003), ("arch", 200_001), ("hairball", 60_007)])
def test_culled_equals_oracle(G, name, n):
    r, nbox = _check(G, scenes.make_scene(name, seed=1, ntris=n))
    assert r.npairs <= nbox


def test_culled_hairball_drops_most_box_pairs(G):
    r, nbox = _check(G, scenes.make_scene("hairball", seed=2, ntris=200_000))
    assert r.npairs < 0.5 * nbox


@pytest.mark.parametrize("digit", [4, 8, 9, 11])
def test_culled_under_digit_widths(G, digit):
    G.tune_set("max_digit_bits", digit)
    try:
        s = scenes.make_scene("mixed", seed=3, ntris=40_000)
        s.name = f"mixed-digit{digit}"
        _check(G, s)
    finally:
        G.tune_set("max_digit_bits", 9)


@pytest.mark.parametrize("res", [(1, 1, 1), (2, 1, 1), (64, 1, 1), (300, 200, 1)])
def test_culled_few_key_bits(G, res):
    # zero, one and two radix passes; one cell takes no sort at all
    s = scenes.make_scene("mixed", seed=4, ntris=20_000)
    s = _scene(s.verts, s.tris, s.lo, s.hi, res, name=f"mixed-res{res}")
    _check(G, s)


def test_culled_ignores_the_fused_first_pass_and_sort_shapes(G):
    s = scenes.make_scene("hairball", seed=5, ntris=30_000)
    want = oracle.build_scene_culled(s)
    for knob, val in (("fused_expand", 1), ("sort_shape", 0), ("sort_shape", 2)):
        G.tune_set(knob, val)
        try:
            r, nbox = G.build_culled(G.GridInput.from_scene(s))
            c, o, rg = r.numpy()
            assert np.array_equal(c, want[0]) and np.array_equal(o, want[1]) and np.array_equal(rg, want[2]), knob
        finally:
            G.tune_set("fused_expand", 0)
            G.tune_set("sort_shape", 3)


def test_culled_outside_and_nan_vertices_keep_their_boxes(G):
    # a triangle with a vertex beyond the bounds, one with a NaN vertex, and a
    # sliver inside: the first two keep their whole (clamped) boxes
    tri = [[[-3.0, 0.5, 0.5], [2.5, 3.5, 0.5], [0.5, 0.2, 3.1]],
           [[0.5, 0.5, 0.5], [np.nan, 1.0, 1.0], [3.5, 3.5, 3.5]],
           [[0.2, 0.2, 0.2], [3.8, 3.7, 3.9], [3.81, 3.72, 3.88]]]
    verts, tris = scenes.soup_from_vertices(np.asarray(tri, np.float64))
    s = _scene(verts, tris, [0, 0, 0], [4, 4, 4], [4, 4, 4], name="outside-nan")
    r, nbox = _check(G, s)
    _, _, count = oracle.count_cells(s.verts, s.tris, s.lo, s.hi, s.res)
    objs = r.numpy()[1]
    assert int((objs == 0).sum()) == int(count[0]) and int((objs == 1).sum()) == int(count[1])
    assert int((objs == 2).sum()) < int(count[2])


def test_culled_empty_scene(G):
    s = _scene(np.zeros((3, 0), np.float32), np.zeros((0, 3), np.uint32), [0, 0, 0], [1, 1, 1], [3, 2, 5], "empty")
    r, nbox = _check(G, s)
    assert r.npairs == 0 and nbox == 0


def test_culled_capacity_errors(G):
    s = scenes.make_scene("hairball", seed=6, ntris=10_000)
    g = G.GridInput.from_scene(s)
    nbox, _ = G.count(g)
    oc = oracle.build_scene_culled(s)[0]
    kept = len(oc)
    # outputs one pair short of the kept pairs: the kept count is reported
    out = G.GridResult(torch.zeros(kept - 1, dtype=torch.int32, device="cuda"),
                       torch.zeros(kept - 1, dtype=torch.int32, device="cuda"),
                       torch.zeros(2 * g.ncells, dtype=torch.int32, device="cuda"), 0)
    with pytest.raises(G.GridError) as e:
        G.build_culled(g, box_cap=nbox, out=out)
    assert e.value.status == G.GRID_E_CAPACITY and out.npairs == kept
    # a box capacity below the box pairs: nothing is kept, the box count is reported
    L = G.lib()
    ws = G.Workspace()
    wp, wn = ws.ptr_size(G.workspace_size_culled(g.ntris, nbox - 1, g.res))
    big = torch.zeros(nbox, dtype=torch.int32, device="cuda")
    o = G.grid_out(big.data_ptr(), big.data_ptr(), out.ranges.data_ptr(), nbox, 0)
    nb = C.c_uint64(0)
    st = L.grid_build_culled(*G._input_args(g), wp, wn, C.c_uint64(nbox - 1), C.byref(o), C.byref(nb), G._stream())
    assert st == G.GRID_E_CAPACITY and nb.value == nbox and o.npairs == 0
    # and then the build with room for everything is exact
    _check(G, s)
