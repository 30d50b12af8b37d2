"""GPU parity of batched builds: every grid of a batch equals its plain build and
the oracle, bit for bit."""
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


def _cmp_oracle(r, s):
    c, o, rg = r.numpy()
    oc, oo, orr = oracle.build_scene(s)
    assert r.npairs == len(oc), s.name
    assert np.array_equal(c, oc), s.name
    assert np.array_equal(o, oo), s.name
    assert np.array_equal(rg, orr), s.name


def _uneven_batch():
    rng = np.random.default_rng(11)
    sizes = [1, 0, 5000, 17, 120_000, 3, 2048, 2049, 40_000, 999, 0, 60_000]
    out = scenes.make_batch(1, ngrids=len(sizes), sizes=np.asarray(sizes))
    out[5].res = np.asarray([1, 1, 1], np.uint32)           # a one-cell grid
    out[7].res = np.asarray([1024, 1, 3], np.uint32)
    out[9].res = np.asarray([512, 512, 512], np.uint32)      # 27 cell bits
    for s in out:
        if s.ntris == 0:
            s.lo = np.zeros(3, np.float32)
            s.hi = np.ones(3, np.float32)
            s.res = np.asarray(rng.integers(1, 9, size=3), np.uint32)
    return out


def test_count_batched_matches_oracle(G):
    batch = _uneven_batch()
    _say("count_batched", [s.ntris for s in batch])
    caps = G.count_batched([G.GridInput.from_scene(s) for s in batch])
    for s, n in zip(batch, caps):
        _, _, cnt = oracle.count_cells(s.verts, s.tris, s.lo, s.hi, s.res)
        assert n == int(cnt.astype(np.int64).sum()), s.name


def test_batched_uneven_matches_oracle(G):
    batch = _uneven_batch()
    _say("build_batched uneven", [s.ntris for s in batch])
    res = G.build_batched([G.GridInput.from_scene(s) for s in batch])
    for r, s in zip(res, batch):
        _cmp_oracle(r, s)


def test_batched_tiles_over_two_grids(G):
    # count tiles (8192 triangles) that hold triangles of exactly two grids,
    # with and without empty grids between them, and tiles over three
    sizes = [6000, 0, 0, 6000, 3000, 9000, 0, 100, 8000, 200, 0]
    batch = scenes.make_batch(6, ngrids=len(sizes), sizes=np.asarray(sizes))
    for s in batch:
        if s.ntris == 0:
            s.lo = np.zeros(3, np.float32)
            s.hi = np.ones(3, np.float32)
            s.res = np.asarray([2, 3, 4], np.uint32)
    _say("build_batched two-grid tiles", sizes)
    inputs = [G.GridInput.from_scene(s) for s in batch]
    caps = G.count_batched(inputs)
    res = G.build_batched(inputs)
    for s, n, r in zip(batch, caps, res):
        assert n == r.npairs, s.name
        _cmp_oracle(r, s)


def test_batched_equals_plain_on_512_grids(G):
    batch = scenes.make_batch(0, ngrids=512)
    _say("build_batched 512", sum(s.ntris for s in batch))
    inputs = [G.GridInput.from_scene(s) for s in batch]
    res = G.build_batched(inputs)
    ws = G.Workspace()
    for i, (g, r) in enumerate(zip(inputs, res)):
        p = G.build(g, cap_pairs=r.npairs, ws=ws)
        assert p.npairs == r.npairs
        assert torch.equal(p.cells[:p.npairs], r.cells[:r.npairs]), i
        assert torch.equal(p.objs[:p.npairs], r.objs[:r.npairs]), i
        assert torch.equal(p.ranges, r.ranges), i
    for i in (0, 1, 255, 511):
        _cmp_oracle(res[i], batch[i])


def test_batched_repeat_identical(G):
    batch = scenes.make_batch(2, ngrids=64)
    inputs = [G.GridInput.from_scene(s) for s in batch]
    outs = G.alloc_results(inputs, G.count_batched(inputs))
    G.build_batched(inputs, outs)
    first = [o.numpy() for o in outs]
    for rep in range(5):
        G.build_batched(inputs, outs)
        for a, o in zip(first, outs):
            for x, y in zip(a, o.numpy()):
                assert np.array_equal(x, y), rep


def test_batched_capacity_error(G):
    batch = scenes.make_batch(3, ngrids=4, sizes=np.array([100, 200, 300, 400]))
    inputs = [G.GridInput.from_scene(s) for s in batch]
    caps = G.count_batched(inputs)
    caps[2] -= 1
    outs = G.alloc_results(inputs, caps)
    with pytest.raises(G.GridError) as e:
        G.build_batched(inputs, outs)
    assert e.value.status == G.GRID_E_CAPACITY
    assert outs[2].npairs == caps[2] + 1


def test_batched_chunks_when_keys_exceed_32_bits(G):
    # 40 grids of 2^27 cells need 27 + 6 bits: the batch is split into runs whose
    # packed keys fit in 32 bits; results must still equal the plain builds.
    rng = np.random.default_rng(5)
    batch = scenes.make_batch(4, ngrids=40, sizes=rng.integers(1, 300, size=40))
    for s in batch:
        s.res = np.asarray([512, 512, 512], np.uint32)
    _say("build_batched chunked", len(batch))
    inputs = [G.GridInput.from_scene(s) for s in batch]
    res = G.build_batched(inputs)
    ws = G.Workspace()
    for i in (0, 31, 32, 39):
        p = G.build(inputs[i], cap_pairs=res[i].npairs, ws=ws)
        assert torch.equal(p.cells[:p.npairs], res[i].cells[:res[i].npairs]), i
        assert torch.equal(p.objs[:p.npairs], res[i].objs[:res[i].npairs]), i
        assert torch.equal(p.ranges, res[i].ranges), i
    del res
    torch.cuda.empty_cache()


@pytest.mark.parametrize("fused,digit,shape", [(0, 8, 3), (1, 8, 3), (1, 10, 3), (0, 11, 3), (0, 9, 0), (0, 9, 1),
                                                (0, 9, 2), (0, 10, 4)])
def test_batched_under_tuning(G, fused, digit, shape):
    G.tune_set("fused_expand", fused)
    G.tune_set("max_digit_bits", digit)
    G.tune_set("sort_shape", shape)
    G.tune_set("small_tiles", 0)  # this batch would otherwise run the small-build shape
    try:
        batch = _uneven_batch()[:9]
        res = G.build_batched([G.GridInput.from_scene(s) for s in batch])
        for r, s in zip(res, batch):
            _cmp_oracle(r, s)
    finally:
        G.tune_set("fused_expand", 0)
        G.tune_set("max_digit_bits", 9)
        G.tune_set("sort_shape", 3)
        G.tune_set("small_tiles", 1)


def test_batched_build_object_repeats(G):
    # marshalled once, called again and again: the same grids as build_batched and the oracle
    batch = _uneven_batch()[:8]
    inputs = [G.GridInput.from_scene(s) for s in batch]
    ref = G.build_batched(inputs)
    outs = G.alloc_results(inputs, [r.npairs for r in ref])
    b = G.BatchedBuild(inputs, outs)
    for _ in range(3):
        for o in outs:
            o.cells.fill_(0)
        b()
        for o, r in zip(outs, ref):
            assert o.npairs == r.npairs
            assert torch.equal(o.cells[:o.npairs], r.cells[:r.npairs])
            assert torch.equal(o.objs[:o.npairs], r.objs[:r.npairs])
            assert torch.equal(o.ranges, r.ranges)
    for o, s in zip(outs, batch):
        _cmp_oracle(o, s)
