"""GPU check of the autotuner: it times several settings, every one of them
reproduces the default grid, and the chosen setting is cached and applied."""
import numpy as np
import pytest

import oracle
from paper_2403_10647_amd import scenes, tune

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_10647_amd import _lib
    _lib.lib()
    return _lib


SPACE = {"max_digit_bits": (8, 9, 11), "sort_shape": (0, 3), "fused_expand": (0, 1)}


def test_tune_plain_and_apply(G, tmp_path):
    s = scenes.make_scene("mixed", seed=5, ntris=40_000)
    g = G.GridInput.from_scene(s)
    path = str(tmp_path / "tune.json")
    best, table = tune.tune_plain(g, reps=2, space=SPACE, cache_path=path, G=G)
    assert len(table) == 12 and all(r["identical"] for r in table)
    assert table[0]["knobs"] == best
    no, _ = G.count(g)
    try:
        got = tune.apply(False, max(1, (g.ncells - 1).bit_length()), no, cache_path=path, G=G)
        assert got == best and all(G.tune_get(k) == v for k, v in best.items())
        c, o, r = G.build(g).numpy()
        oc, oo, orr = oracle.build_scene(s)
        assert np.array_equal(c, oc) and np.array_equal(o, oo) and np.array_equal(r, orr)
    finally:
        for k, v in tune.DEFAULTS.items():
            G.tune_set(k, v)


def test_tune_batched(G, tmp_path):
    batch = scenes.make_batch(6, ngrids=24, sizes=np.random.default_rng(6).integers(100, 20_000, size=24))
    inputs = [G.GridInput.from_scene(s) for s in batch]
    best, table = tune.tune_batched(inputs, reps=2, space=SPACE, cache_path=str(tmp_path / "t.json"), G=G)
    assert all(r["identical"] for r in table)
    assert all(G.tune_get(k) == v for k, v in tune.DEFAULTS.items())   # the tuner restores the knobs


def test_tune_plain_wide_key(G, tmp_path):
    # 160^3 cells = a 22-bit key, where 11-bit digits need a larger workspace
    # than the default setting: the tuner must size for every candidate
    base = scenes.make_scene("mixed", seed=9, ntris=30_000)
    s = scenes.Scene("mixed22", base.verts, base.tris, base.lo, base.hi, np.array([160, 160, 160], np.uint32))
    g = G.GridInput.from_scene(s)
    best, table = tune.tune_plain(g, reps=1, space={"max_digit_bits": (8, 11), "sort_shape": (3,),
                                                    "fused_expand": (0,)}, G=G)
    assert len(table) == 2 and all(r["identical"] for r in table)
    c, o, r = G.build(g).numpy()
    oc, oo, orr = oracle.build_scene(s)
    assert np.array_equal(c, oc) and np.array_equal(o, oo) and np.array_equal(r, orr)


def test_confirm_plain_keeps_the_faster_and_restores_knobs(G):
    # the bench confirms the search's best against the defaults before timing
    # the headline build with it; a 22-bit key sizes the workspace for 11-bit digits
    base = scenes.make_scene("mixed", seed=11, ntris=30_000)
    s = scenes.Scene("mixed22", base.verts, base.tris, base.lo, base.hi, np.array([160, 160, 160], np.uint32))
    g = G.GridInput.from_scene(s)
    cand = {"max_digit_bits": 11, "sort_shape": 0, "fused_expand": 0}
    chosen, med = tune.confirm_plain(g, cand, rounds=2, reps=2, G=G)
    assert chosen in (cand, tune.DEFAULTS)
    assert set(med) == {"default", "tuned"} and all(v > 0 for v in med.values())
    assert chosen == (cand if med["tuned"] < med["default"] else tune.DEFAULTS)
    assert all(G.tune_get(k) == v for k, v in tune.DEFAULTS.items())
    try:
        tune.set_knobs(G, chosen)
        c, o, r = G.build(g).numpy()
        oc, oo, orr = oracle.build_scene(s)
        assert np.array_equal(c, oc) and np.array_equal(o, oo) and np.array_equal(r, orr)
    finally:
        tune.set_knobs(G, tune.DEFAULTS)
