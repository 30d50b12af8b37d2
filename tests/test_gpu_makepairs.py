"""GPU parity of the per-object pair generation (one thread per object writes
all of its object's pairs, as sorted-grid builders do): the same grid as the
oracle and as the per-pair expansion, bit for bit, across radix plans with
zero to three passes, empty scenes and objects of very uneven size."""
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


@pytest.fixture
def per_object(G):
    G.tune_set("per_object_pairs", 1)
    try:
        yield
    finally:
        G.tune_set("per_object_pairs", 0)


def _say(*a):
    print(*a, flush=True)


def _check(G, s):
    _say("per-object build", s.name, s.ntris, list(s.res))
    r = G.build(G.GridInput.from_scene(s))
    c, o, rg = r.numpy()
    oc, oo, orr = oracle.build_scene(s)
    assert r.npairs == len(oc), s.name
    assert np.array_equal(c, oc), s.name
    assert np.array_equal(o, oo), s.name
    assert np.array_equal(rg, orr), s.name


def _scene(verts, tris, lo, hi, res, name):
    return scenes.Scene(name, np.ascontiguousarray(verts, np.float32), np.ascontiguousarray(tris, np.uint32),
                        np.asarray(lo, np.float32), np.asarray(hi, np.float32), np.asarray(res, np.uint32))


def test_per_object_matches_oracle(G, per_object):
    assert G.tune_get("per_object_pairs") == 1
    _check(G, scenes.make_scene("small", seed=4))                   # 15 key bits: 2 passes
    _check(G, scenes.make_scene("mixed", seed=5, ntris=40_000))     # huge and tiny triangles
    _check(G, scenes.make_scene("arch", seed=6, ntris=150_000))     # 3 passes


def test_per_object_degenerate_grids(G, per_object):
    s = scenes.make_scene("small", seed=7, ntris=3000)
    s.res = np.asarray([1, 1, 1], np.uint32)                         # one cell: no radix pass
    _check(G, s)
    s = scenes.make_scene("small", seed=8, ntris=3000)
    s.res = np.asarray([300, 1, 1], np.uint32)                       # 9 key bits: one pass
    _check(G, s)
    empty = _scene(np.zeros((3, 0), np.float32), np.zeros((0, 3), np.uint32), [0, 0, 0], [1, 1, 1], [4, 5, 6], "empty")
    r = G.build(G.GridInput.from_scene(empty), cap_pairs=0)
    assert r.npairs == 0 and not r.ranges.any().item()


def test_per_object_equals_per_pair_at_1m(G):
    g = G.GridInput.from_scene(scenes.make_scene("mixed", seed=9, ntris=1_000_000))
    ref = G.build(g)
    G.tune_set("per_object_pairs", 1)
    try:
        r = G.build(g, cap_pairs=ref.npairs)
    finally:
        G.tune_set("per_object_pairs", 0)
    _say("1M mixed", ref.npairs)
    assert r.npairs == ref.npairs
    n = ref.npairs
    assert torch.equal(r.cells[:n], ref.cells[:n])
    assert torch.equal(r.objs[:n], ref.objs[:n])
    assert torch.equal(r.ranges, ref.ranges)


def test_per_object_capacity_error(G, per_object):
    # too small a capacity: the required count is reported and nothing is written
    g = G.GridInput.from_scene(scenes.make_scene("small", seed=10))
    n, _ = G.count(g)
    out = G.GridResult(torch.full((n - 1,), -7, dtype=torch.int32, device="cuda"),
                       torch.full((n - 1,), -7, dtype=torch.int32, device="cuda"),
                       torch.full((2 * g.ncells,), -7, dtype=torch.int32, device="cuda"), 0)
    with pytest.raises(G.GridError) as e:
        G.build(g, out=out)
    assert e.value.status == G.GRID_E_CAPACITY and out.npairs == n
    assert bool((out.cells == -7).all()) and bool((out.objs == -7).all()) and bool((out.ranges == -7).all())


def test_per_object_four_radix_passes(G, per_object):
    # 19 key bits at digits of at most 6 bits: four passes, every histogram run counter in use
    s = scenes.make_scene("small", seed=11, ntris=20_000)
    s.res = np.asarray([128, 64, 64], np.uint32)
    G.tune_set("max_digit_bits", 6)
    try:
        passes = G.sort_plan(19)[0]
        assert passes == 4
        _check(G, s)
    finally:
        G.tune_set("max_digit_bits", 9)


def test_per_object_knob_left_alone_elsewhere(G, per_object):
    # batched builds always expand per pair, and a fused first pass regenerates
    # its keys itself: both still give the oracle's grids with the knob set
    batch = scenes.make_batch(12, ngrids=6, sizes=np.array([3000, 0, 12_000, 5, 9000, 700]))
    for s in batch:
        if s.ntris == 0:
            s.lo, s.hi = np.zeros(3, np.float32), np.ones(3, np.float32)
            s.res = np.asarray([3, 2, 5], np.uint32)
    res = G.build_batched([G.GridInput.from_scene(s) for s in batch])
    for r, s in zip(res, batch):
        c, o, rg = r.numpy()
        oc, oo, orr = oracle.build_scene(s)
        assert np.array_equal(c, oc) and np.array_equal(o, oo) and np.array_equal(rg, orr), s.name
    G.tune_set("fused_expand", 1)
    try:
        _check(G, scenes.make_scene("mixed", seed=13, ntris=30_000))
    finally:
        G.tune_set("fused_expand", 0)
