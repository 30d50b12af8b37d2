"""GPU parity of the compact path (counting scatter with atomics, then in-cell
sorts; the compact-grid construction of the Related Work section, combined
with the sorted path through a statistics pass as the Conclusions propose)
against the oracle, bit for bit: a cell's pairs are distinct objects, so once
each cell is sorted the output is unique and equal to the sorted path's."""
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
    yield _lib
    _lib.tune_set("build_path", 0)


def _say(*a):
    print(*a, flush=True)


def _scene(verts, tris, lo, hi, res, name="adhoc"):
    return scenes.Scene(name, np.ascontiguousarray(verts, np.float32), np.ascontiguousarray(tris, np.uint32),
                        np.asarray(lo, np.float32), np.asarray(hi, np.float32), np.asarray(res, np.uint32))


def _check(G, s, path=1):
    _say("build path", path, s.name, s.ntris, list(map(int, s.res)))
    G.tune_set("build_path", path)
    try:
        g = G.GridInput.from_scene(s)
        r = G.build(g)
        last = G.tune_get("last_path")
    finally:
        G.tune_set("build_path", 0)
    c, o, rg = r.numpy()
    oc, oo, orr = oracle.build_scene(s)
    assert r.npairs == len(oc)
    assert np.array_equal(c, oc)
    assert np.array_equal(o, oo)
    assert np.array_equal(rg, orr)
    return last


@pytest.mark.parametrize("name,n", [("small", None), ("mixed", 100_003), ("arch", 200_001), ("hairball", 30_011)])
def test_compact_equals_oracle(G, name, n):
    assert _check(G, scenes.make_scene(name, seed=1, ntris=n)) == 1


@pytest.mark.parametrize("res", [(1, 1, 1), (3, 1, 1), (300, 200, 1)])
def test_compact_few_cells(G, res):
    s = scenes.make_scene("mixed", seed=4, ntris=20_000)
    _check(G, _scene(s.verts, s.tris, s.lo, s.hi, res, name=f"mixed-res{res}"))


def test_compact_crowded_cells(G):
    # one cell holding more pairs than the LDS sort takes (merged through the
    # scratch buffer), cells of a few hundred (sorted in LDS) and small cells
    rng = np.random.default_rng(5)
    hot = np.array([0.3, 0.3, 0.3]) + rng.uniform(-0.02, 0.02, size=(20_000, 3, 3))
    warm = np.array([0.7, 0.6, 0.2]) + rng.uniform(-0.05, 0.05, size=(900, 3, 3))
    cold = rng.uniform(0.0, 1.0, size=(3000, 1, 3)) + rng.uniform(-0.01, 0.01, size=(3000, 3, 3))
    v = np.concatenate([cold[:1500], hot, warm, cold[1500:]], axis=0)
    verts, tris = scenes.soup_from_vertices(v)
    _check(G, _scene(verts, tris, [0, 0, 0], [1, 1, 1], [4, 5, 6], name="crowded"))


def test_compact_empty_and_capacity(G):
    s = _scene(np.zeros((3, 0), np.float32), np.zeros((0, 3), np.uint32), [0, 0, 0], [1, 1, 1], [3, 2, 5], "empty")
    _check(G, s)
    s = scenes.make_scene("small", seed=2)
    g = G.GridInput.from_scene(s)
    n, _ = G.count(g)
    G.tune_set("build_path", 1)
    try:
        with pytest.raises(G.GridError) as e:
            G.build(g, cap_pairs=n - 1)
        assert e.value.status == G.GRID_E_CAPACITY
    finally:
        G.tune_set("build_path", 0)


def test_statistics_choose_the_path(G):
    # sparse small triangles take the compact path; the dense 1M mixed-style
    # scene (about eight pairs per cell) keeps the sorted path; both exact
    assert _check(G, scenes.make_scene("small", seed=3), path=2) == 1
    assert _check(G, scenes.make_scene("mixed", seed=3, ntris=200_000), path=2) == 0
