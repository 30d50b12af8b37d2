"""GPU parity: the HIP library against the CPU oracle, bit for bit.

Every output is integer indexing plus one fixed FP32 sequence, so the
tolerance is zero.  Sizes span several tiles (8192 triangles per count tile,
4096 pairs per expansion tile, 8192 to 16384 pairs per radix tile, 4096 merge
items per range tile) with ragged tails.
"""
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


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def _soup(tri_coords):
    v = np.asarray(tri_coords, np.float64).reshape(-1, 3, 3)
    return scenes.soup_from_vertices(v)


def _scene(verts, tris, lo, hi, res, name="adhoc"):
    return scenes.Scene(name, np.ascontiguousarray(verts, np.float32), np.ascontiguousarray(tris, np.uint32),
                        np.asarray(lo, np.float32), np.asarray(hi, np.float32), np.asarray(res, np.uint32))


def _check_build(G, s):
    _say("build", s.name, s.ntris, list(s.res))
    g = G.GridInput.from_scene(s)
    r = G.build(g)
    c, o, rg = r.numpy()
    oc, oo, orr = oracle.build_scene(s)
    assert r.npairs == len(oc)
    assert np.array_equal(c, oc)
    assert np.array_equal(o, oo)
    assert np.array_equal(rg, orr)
    return r


# ---- scans -------------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2047, 2048, 2049, 65539, 1_000_003])
def test_scan_exclusive_sum(G, n):
    _say("scan exsum", n)
    x = np.random.default_rng(n).integers(0, 1 << 20, size=n).astype(np.uint32)
    out, tot = G.scan_u32(_dev(x), G.SCAN_EXCLUSIVE_SUM)
    cs = np.cumsum(x.astype(np.uint64))
    assert tot == int(cs[-1])
    assert np.array_equal(_u32(out), (cs - x).astype(np.uint32))


@pytest.mark.parametrize("n", [1, 2049, 1_000_003])
def test_scan_inclusive_max(G, n):
    _say("scan max", n)
    x = np.random.default_rng(n).integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    out, tot = G.scan_u32(_dev(x), G.SCAN_INCLUSIVE_MAX)
    want = np.maximum.accumulate(x)
    assert tot == int(want[-1]) and np.array_equal(_u32(out), want)


@pytest.mark.parametrize("n,density", [(1, 0.5), (4099, 0.01), (100_003, 0.3), (100_003, 0.0), (100_003, 1.0)])
def test_scan_segmented(G, n, density):
    _say("scan seg", n, density)
    rng = np.random.default_rng(n)
    x = rng.integers(0, 1000, size=n).astype(np.uint32)
    f = (rng.random(n) < density).astype(np.uint32)
    out, tot = G.scan_u32(_dev(x), G.SCAN_SEGMENTED_EXCLUSIVE_SUM, flags=_dev(f))
    want = np.zeros(n, np.uint64)
    acc = 0
    for i in range(n):  # plain definition
        if f[i]:
            acc = 0
        want[i] = acc
        acc += int(x[i])
    assert np.array_equal(_u32(out), want.astype(np.uint32))
    assert tot == acc


# ---- radix sort ----------------------------------------------------------------------------

@pytest.mark.parametrize("n,bits,kind", [
    (1, 8, "rand"), (8191, 15, "rand"), (8192, 15, "rand"), (8193, 22, "rand"),
    (300_001, 25, "rand"), (300_001, 32, "rand"), (200_000, 9, "equal"),
    (200_000, 20, "sorted"), (200_000, 20, "reverse"), (1_000_000, 29, "rand"), (50_000, 1, "rand"),
])
def test_sort_pairs_stable(G, n, bits, kind):
    _say("sort", n, bits, kind)
    rng = np.random.default_rng(bits)
    hi = 1 << bits
    if kind == "rand":
        k = rng.integers(0, hi, size=n, dtype=np.uint64).astype(np.uint32)
    elif kind == "equal":
        k = np.full(n, hi - 1, np.uint32)
    elif kind == "sorted":
        k = np.sort(rng.integers(0, hi, size=n)).astype(np.uint32)
    else:
        k = np.sort(rng.integers(0, hi, size=n))[::-1].astype(np.uint32)
    v = np.arange(n, dtype=np.uint32)
    kd, vd = _dev(k), _dev(v)
    G.sort_pairs(kd, vd, bits)
    order = np.argsort(k, kind="stable")
    assert np.array_equal(_u32(kd), k[order])
    assert np.array_equal(_u32(vd), v[order])


# ---- stages ---------------------------------------------------------------------------------

@pytest.mark.parametrize("name,n", [("small", None), ("mixed", 150_000), ("arch", 150_000)])
def test_count_stage(G, name, n):
    s = scenes.make_scene(name, ntris=n)
    _say("count", name, s.ntris)
    no, start = G.count(G.GridInput.from_scene(s), with_start=True)
    _, _, cnt = oracle.count_cells(s.verts, s.tris, s.lo, s.hi, s.res)
    ostart, ono = oracle.exclusive_sum(cnt)
    assert no == ono
    assert np.array_equal(_u32(start).astype(np.uint64), ostart)


@pytest.mark.parametrize("name,n", [("small", None), ("mixed", 150_000), ("arch", 150_000)])
def test_expand_stage(G, name, n):
    s = scenes.make_scene(name, ntris=n)
    _say("expand", name, s.ntris)
    c, o = G.expand(G.GridInput.from_scene(s))
    og = oracle.build_stages(s.verts, s.tris, s.lo, s.hi, s.res)
    assert np.array_equal(_u32(c), og.cells_objorder)
    assert np.array_equal(_u32(o), og.objs_objorder)


# ---- whole builds -----------------------------------------------------------------------------

def test_build_small_scene(G):
    _check_build(G, scenes.make_scene("small"))


@pytest.mark.parametrize("name,n", [("mixed", 20_011), ("mixed", 200_003), ("arch", 20_011), ("arch", 200_003)])
def test_build_scaled_scenes(G, name, n):
    _check_build(G, scenes.make_scene(name, ntris=n))


@pytest.mark.parametrize("res", [(1, 1, 1), (1, 1, 2), (7, 1, 3), (1024, 1, 1), (33, 17, 5), (256, 256, 16)])
def test_build_resolutions(G, res):
    s = scenes.make_scene("mixed", ntris=5000)
    s.res = np.asarray(res, np.uint32)
    s.name = f"mixed-res{res}"
    _check_build(G, s)


def test_build_edge_geometry(G):
    nan, inf = float("nan"), float("inf")
    verts, tris = _soup([
        [[3, 3, 3], [3, 3, 3], [3, 3, 3]],
        [[8, 8, 8], [8, 8, 8], [8, 8, 8]],
        [[-5, -5, -5], [-1, -2, -3], [-4, -4, -4]],
        [[2.5, 0, 0], [4, 0, 0], [3.5, 0, 0]],
        [[20, 1, 1], [30, 1, 1], [40, 1, 1]],
        [[nan, 1.5, 1.5], [2.5, 1.5, 1.5], [5.5, 1.5, 1.5]],
        [[nan, 1, 1], [nan, 1, 1], [nan, 1, 1]],
        [[-inf, 1, 1], [0.5, 1, 1], [0.5, 1, 1]],
        [[inf, 1, 1], [0.5, 1, 1], [0.5, 1, 1]],
        [[0, 0, 0], [8, 8, 8], [0, 8, 0]],          # the whole grid
        [[1e-7, 1, 1], [7.9999995, 1, 1], [4, 1, 1]],
    ] * 300)
    _check_build(G, _scene(verts, tris, [0, 0, 0], [8, 8, 8], [8, 8, 8], "edges"))


def test_build_dyadic_random(G):
    from brute import dyadic_scene
    for seed in range(3):
        verts, tris = dyadic_scene(np.random.default_rng(seed), 20_000, -4.0, 4.0, 1.5)
        _check_build(G, _scene(verts, tris, [-4, -4, -4], [4, 4, 4], [16, 32, 8], f"dyadic{seed}"))


def test_build_one_triangle_and_empty(G):
    verts, tris = _soup([[[0.1, 0.2, 0.3], [0.5, 0.9, 0.3], [0.2, 0.2, 0.8]]])
    _check_build(G, _scene(verts, tris, [0, 0, 0], [1, 1, 1], [10, 10, 10], "one"))
    s = _scene(np.zeros((3, 0), np.float32), np.zeros((0, 3), np.uint32), [0, 0, 0], [1, 1, 1], [4, 5, 6], "empty")
    g = G.GridInput.from_scene(s)
    r = G.build(g, cap_pairs=0)
    assert r.npairs == 0
    assert not _u32(r.ranges).any()


def test_build_huge_triangles(G):
    # few triangles covering most of a large grid: long per-object segments
    verts, tris = _soup([[[0, 0, 0], [100, 100, 100], [0, 100, 0]],
                         [[10, 10, 10], [90, 20, 70], [50, 50, 50]],
                         [[1, 1, 1], [1.5, 1.5, 1.5], [1, 1.5, 1]]])
    _check_build(G, _scene(verts, tris, [0, 0, 0], [100, 100, 100], [200, 100, 50], "huge"))


def test_build_indexed_mesh(G):
    # shared vertices and an arbitrary index order
    rng = np.random.default_rng(7)
    nv = 5000
    verts = rng.uniform(0, 10, size=(3, nv)).astype(np.float32)
    tris = rng.integers(0, nv, size=(30_000, 3)).astype(np.uint32)
    _check_build(G, _scene(verts, tris, [0, 0, 0], [10, 10, 10], [20, 20, 20], "indexed"))


def test_build_soup_and_indexed_triangles_interleaved(G):
    # triangles listing three consecutive vertices (one wide load per
    # coordinate in the count) side by side with ones that list their own three
    # vertices in another order or repeat one (three loads), within the same waves
    rng = np.random.default_rng(17)
    n = 20_000
    centres = rng.uniform(0.5, 9.5, size=(n, 3))
    verts = np.ascontiguousarray((centres.repeat(3, axis=0) + rng.uniform(-0.2, 0.2, size=(3 * n, 3))).T, np.float32)
    base = 3 * np.arange(n, dtype=np.uint32)[:, None]
    orders = np.array([[0, 1, 2], [1, 0, 2], [2, 1, 0], [0, 2, 1], [0, 0, 1], [2, 2, 2]], np.uint32)
    pick = np.where(rng.random(n) < 0.5, 0, rng.integers(1, len(orders), size=n))
    tris = np.ascontiguousarray(base + orders[pick], np.uint32)
    _check_build(G, _scene(verts, tris, [0, 0, 0], [10, 10, 10], [40, 40, 40], "soup+reordered"))


def test_repeat_builds_identical(G):
    s = scenes.make_scene("arch", ntris=100_000)
    g = G.GridInput.from_scene(s)
    first = [x.copy() for x in G.build(g).numpy()]
    for i in range(10):
        again = G.build(g).numpy()
        for a, b in zip(first, again):
            assert np.array_equal(a, b), f"repeat {i} differs"


# ---- errors ----------------------------------------------------------------------------------

def test_error_paths(G):
    s = scenes.make_scene("small")
    g = G.GridInput.from_scene(s)
    for lo, hi, res in [([0, 0, 0], [0, 1, 1], [4, 4, 4]), ([0, 0, 0], [1, 1, 1], [4, 0, 4]),
                        ([0, 0, 0], [1, 1, 1], [4, 1025, 4]), ([float("nan"), 0, 0], [1, 1, 1], [4, 4, 4])]:
        bad = G.GridInput(g.verts, g.tris, lo, hi, res)
        with pytest.raises(G.GridError) as e:
            G.build(bad, cap_pairs=10)
        assert e.value.status == G.GRID_E_INVAL
    # capacity too small reports the required count and writes no output
    no, _ = G.count(g)

    def sentinel_out(cap, ncells):
        r = G.GridResult(torch.full((max(cap, 1),), -7, dtype=torch.int32, device="cuda"),
                         torch.full((max(cap, 1),), -7, dtype=torch.int32, device="cuda"),
                         torch.full((2 * ncells,), -7, dtype=torch.int32, device="cuda"), 0)
        return r

    out = sentinel_out(no - 1, g.ncells)
    with pytest.raises(G.GridError) as e:
        G.build(g, out=out)
    assert e.value.status == G.GRID_E_CAPACITY and out.npairs == no
    assert bool((out.cells == -7).all()) and bool((out.objs == -7).all()) and bool((out.ranges == -7).all())
    # vertex index out of range (flagged by the count kernel)
    t = g.tris.clone()
    t[5, 1] = g.nverts + 3
    out = sentinel_out(no, g.ncells)
    with pytest.raises(G.GridError) as e:
        G.build(G.GridInput(g.verts, t, g.lo, g.hi, g.res), out=out)
    assert e.value.status == G.GRID_E_BADINDEX
    assert bool((out.cells == -7).all()) and bool((out.ranges == -7).all())
    # NO beyond 2^32 - 1
    verts, tris = _soup([[[0, 0, 0], [1, 1, 1], [0, 1, 0]]] * 5)
    big = G.GridInput.from_scene(_scene(verts, tris, [0, 0, 0], [1, 1, 1], [1024, 1024, 1024]))
    with pytest.raises(G.GridError) as e:
        G.count(big)
    assert e.value.status == G.GRID_E_OVERFLOW
    with pytest.raises(G.GridError) as e:
        G.build(big, cap_pairs=1000)
    assert e.value.status == G.GRID_E_OVERFLOW
    # a workspace used by a failed build serves the next one
    r = G.build(g, cap_pairs=no)
    oc, oo, orr = oracle.build_scene(s)
    c, o, rg = r.numpy()
    assert np.array_equal(c, oc) and np.array_equal(o, oo) and np.array_equal(rg, orr)


def test_build_with_spare_capacity(G):
    # launches are sized by the capacity; the kernels use the NO they count
    for name, n in [("small", 4096), ("mixed", 30_000)]:
        s = scenes.make_scene(name, ntris=n)
        g = G.GridInput.from_scene(s)
        no, _ = G.count(g)
        r = G.build(g, cap_pairs=3 * no + 100_000)
        assert r.npairs == no
        oc, oo, orr = oracle.build_scene(s)
        c, o, rg = r.numpy()
        assert np.array_equal(c, oc) and np.array_equal(o, oo) and np.array_equal(rg, orr)


@pytest.mark.parametrize("fused", [0, 1])
@pytest.mark.parametrize("digit", [4, 8, 9, 10, 11])
def test_build_under_every_tuning(G, fused, digit):
    G.tune_set("fused_expand", fused)
    G.tune_set("max_digit_bits", digit)
    try:
        for name, n in [("mixed", 60_000), ("arch", 60_000)]:
            s = scenes.make_scene(name, ntris=n)
            s.name = f"{name}-fused{fused}-digit{digit}"
            _check_build(G, s)
    finally:
        G.tune_set("fused_expand", 0)
        G.tune_set("max_digit_bits", 9)


@pytest.mark.parametrize("shape", [0, 1, 2, 3, 4])
def test_build_under_every_sort_shape(G, shape):
    G.tune_set("sort_shape", shape)
    G.tune_set("small_tiles", 0)  # these scenes would otherwise all run the small-build shape
    try:
        for name, n in [("mixed", 100_003), ("arch", 100_003)]:
            s = scenes.make_scene(name, ntris=n)
            s.name = f"{name}-shape{shape}"
            _check_build(G, s)
        for digit in (8, 11):
            G.tune_set("max_digit_bits", digit)
            s = scenes.make_scene("arch", ntris=50_000)
            s.name = f"arch-shape{shape}-digit{digit}"
            _check_build(G, s)
    finally:
        G.tune_set("sort_shape", 3)
        G.tune_set("small_tiles", 1)
        G.tune_set("max_digit_bits", 9)


def test_small_builds_take_small_tiles(G):
    # a build with few pairs runs 4096-pair radix tiles whatever sort_shape says,
    # and a large one the knob's shape; both equal the oracle, also on either
    # side of the switch (fewer 16384-pair tiles than the GPU has CUs)
    G.tune_set("sort_shape", 3)
    for n in (4096, 30_000):
        s = scenes.make_scene("arch", ntris=n)
        s.name = f"arch-small-tiles-{n}"
        _check_build(G, s)
    switch = torch.cuda.get_device_properties(0).multi_processor_count * 16384
    below = above = None
    for n in (800_000, 1_200_000, 1_400_000, 1_600_000, 1_800_000, 2_000_000, 2_600_000, 3_200_000):
        s = scenes.make_scene("arch", ntris=n)
        no, _ = G.count(G.GridInput.from_scene(s))
        if no < switch:
            below = s
        elif above is None:
            above = s
    assert below is not None and above is not None
    for s in (below, above):
        s.name = f"arch-tiles-switch-{s.ntris}"
        _check_build(G, s)
    G.tune_set("small_tiles", 0)
    try:
        s = scenes.make_scene("arch", ntris=30_000)
        s.name = "arch-knob-tiles"
        _check_build(G, s)
    finally:
        G.tune_set("small_tiles", 1)


@pytest.mark.parametrize("shape", [3, 4])
def test_build_with_wide_lookback_words(G, shape):
    # radix passes under 2^30 pairs keep 32-bit look-back words; the 64-bit
    # words of larger builds give the same grid
    G.tune_set("wide_lookback", 1)
    G.tune_set("sort_shape", shape)
    G.tune_set("small_tiles", 0)
    try:
        for name, n in [("mixed", 100_003), ("arch", 300_000)]:
            s = scenes.make_scene(name, ntris=n)
            s.name = f"{name}-wide-lookback-shape{shape}"
            _check_build(G, s)
        batch = scenes.make_batch(5, ngrids=7, sizes=np.asarray([3000, 0, 40_000, 1, 900, 12_000, 5]))
        for sc in batch:
            if sc.ntris == 0:
                sc.lo, sc.hi, sc.res = np.zeros(3, np.float32), np.ones(3, np.float32), np.asarray([3, 2, 5], np.uint32)
        res = G.build_batched([G.GridInput.from_scene(sc) for sc in batch])
        for r, sc in zip(res, batch):
            c, o, rg = r.numpy()
            oc, oo, orr = oracle.build_scene(sc)
            assert np.array_equal(c, oc) and np.array_equal(o, oo) and np.array_equal(rg, orr), sc.name
    finally:
        G.tune_set("wide_lookback", 0)
        G.tune_set("sort_shape", 3)
        G.tune_set("small_tiles", 1)


def test_plain_build_object_repeats(G):
    # the marshalled-once build equals G.build and the oracle, call after call
    s = scenes.make_scene("mixed", ntris=30_000)
    g = G.GridInput.from_scene(s)
    no, _ = G.count(g)
    out = G.build(g, cap_pairs=no)
    ref = [x.copy() for x in out.numpy()]
    b = G.PlainBuild(g, out)
    for _ in range(3):
        out.cells.fill_(0)
        r = b()
        assert r.npairs == no
        for x, y in zip(ref, r.numpy()):
            assert np.array_equal(x, y)
    oc, oo, orr = oracle.build_scene(s)
    assert np.array_equal(ref[0], oc) and np.array_equal(ref[1], oo) and np.array_equal(ref[2], orr)


@pytest.mark.parametrize("res", [(512, 512, 1), (1024, 1024, 4)])
def test_huge_triangles_tile_owner_runs(G, res):
    # triangles whose boxes span hundreds of expansion tiles: the count writes
    # the first few tile owners of each, the plan kernel the rest
    rng = np.random.default_rng(11)
    big = [[[0.01, 0.01, 0.01], [0.99, 0.02, 0.98], [0.5, 0.99, 0.5]],
           [[0.98, 0.97, 0.2], [0.03, 0.5, 0.9], [0.6, 0.02, 0.4]]]
    small = rng.uniform(0.0, 1.0, size=(3000, 1, 3)) + rng.uniform(-0.004, 0.004, size=(3000, 3, 3))
    v = np.concatenate([np.asarray(big, np.float64), small, np.asarray(big, np.float64)[::-1]], axis=0)
    verts, tris = scenes.soup_from_vertices(v)
    s = _scene(verts, tris, [0, 0, 0], [1, 1, 1], res, name=f"huge-{res}")
    _check_build(G, s)
    # the same grid inside a batch, between two ordinary grids
    batch = [scenes.make_scene("small", seed=3), s, scenes.make_scene("small", seed=4)]
    outs = G.build_batched([G.GridInput.from_scene(x) for x in batch])
    for r, x in zip(outs, batch):
        c, o, rg = r.numpy()
        oc, oo, orr = oracle.build_scene(x)
        assert np.array_equal(c, oc) and np.array_equal(o, oo) and np.array_equal(rg, orr), x.name
