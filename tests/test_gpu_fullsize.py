"""Parity at the full workload sizes, in the launch configuration the benchmark
times: the 1M-triangle mixed scene and the 10M-triangle architectural scene
element by element against the oracle, and every grid of the 512-grid batch
against the oracle."""
import numpy as np
import pytest

import oracle
from paper_2403_10647_amd import scenes

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

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


def _full_check(G, s):
    g = G.GridInput.from_scene(s)
    ws = G.Workspace()
    no, _ = G.count(g, ws)
    out = G.build(g, cap_pairs=no, ws=ws)
    for _ in range(2):                       # the benchmark's repeated builds into one output
        G.build(g, ws=ws, out=out)
    c, o, r = out.numpy()
    _say("oracle", s.name, s.ntris, no)
    oc, oo, orr = oracle.build(s.verts, s.tris, s.lo, s.hi, s.res)   # the oracle sizes its own output
    assert out.npairs == len(oc) == no
    assert np.array_equal(c, oc)
    assert np.array_equal(o, oo)
    assert np.array_equal(r, orr)
    # the invariants the paper's structure implies, checked on the GPU result
    assert r[0] == 0 and r[-1] == no and np.all(r[1:-1:2] == r[2::2])
    return no


def test_mixed_1m_full(G):
    s = scenes.make_scene("mixed", seed=0)
    _say("mixed", s.ntris, list(s.res))
    assert _full_check(G, s) > 10_000_000


def test_arch_10m_full(G):
    s = scenes.make_scene("arch", seed=0)
    _say("arch", s.ntris, list(s.res))
    assert _full_check(G, s) > 40_000_000


def test_arch_10m_full_under_the_tuned_settings(G):
    # the benchmark times this scene with the tuner's choice, which on MI355X
    # is one of these (1024 x 15 radix tiles, 9- to 11-bit kernels): each
    # grid equals the oracle's, element by element
    from paper_2403_10647_amd import tune
    s = scenes.make_scene("arch", seed=0)
    oc, oo, orr = oracle.build(s.verts, s.tris, s.lo, s.hi, s.res)
    g = G.GridInput.from_scene(s)
    ws = G.Workspace()
    no, _ = G.count(g, ws)
    ws.get(tune.max_workspace(G, g, no))
    out = G.build(g, cap_pairs=no, ws=ws)
    try:
        for digit in (9, 10, 11):
            tune.set_knobs(G, {"max_digit_bits": digit, "sort_shape": 4, "fused_expand": 0})
            out.cells.fill_(-1)
            out.objs.fill_(-1)
            out.ranges.fill_(-1)
            b = G.PlainBuild(g, out, ws)             # the benchmark's call: arguments marshalled once
            for _ in range(2):
                b()
            _say("arch tuned", digit, out.npairs)
            c, o, r = out.numpy()
            assert out.npairs == len(oc)
            assert np.array_equal(c, oc) and np.array_equal(o, oo) and np.array_equal(r, orr), digit
    finally:
        tune.set_knobs(G, tune.DEFAULTS)


def test_batch_512_full(G):
    batch = scenes.make_batch(0, ngrids=512)
    _say("batch", sum(s.ntris for s in batch))
    inputs = [G.GridInput.from_scene(s) for s in batch]
    res = G.build_batched(inputs)
    for i, (r, s) in enumerate(zip(res, batch)):
        c, o, rg = r.numpy()
        oc, oo, orr = oracle.build(s.verts, s.tris, s.lo, s.hi, s.res)
        assert np.array_equal(c, oc) and np.array_equal(o, oo) and np.array_equal(rg, orr), i


def _full_culled(G, s):
    g = G.GridInput.from_scene(s)
    ws = G.Workspace()
    nbox, _ = G.count(g, ws)
    out, nb = G.build_culled(g, box_cap=nbox, ws=ws)
    out, nb = G.build_culled(g, box_cap=nbox, ws=ws, out=out)   # repeated into one output
    c, o, r = out.numpy()
    _say("oracle culled", s.name, s.ntris, nbox, out.npairs)
    oc, oo, orr, obox = oracle.build_scene_culled(s)
    assert nb == obox == nbox and out.npairs == len(oc)
    assert np.array_equal(c, oc) and np.array_equal(o, oo) and np.array_equal(r, orr)
    assert r[0] == 0 and r[-1] == out.npairs and np.all(r[1:-1:2] == r[2::2])
    return nbox, out.npairs


@pytest.mark.parametrize("name", ["mixed", "hairball", "arch"])
def test_culled_full(G, name):
    s = scenes.make_scene(name, seed=0)
    _say(name, s.ntris, list(s.res))
    nbox, kept = _full_culled(G, s)
    assert 0 < kept < nbox


def test_raycast_arch_full_sampled(G):
    # the 10M-triangle grid, rays checked one by one against the brute force
    s = scenes.make_scene("arch", seed=0)
    g = G.GridInput.from_scene(s)
    r = G.build(g)
    rays = scenes.make_rays(s, 24, seed=5)
    ht, ho = G.raycast(g, r, torch.from_numpy(rays).cuda())
    ot, oo = oracle.raycast(s.verts, s.tris, s.lo, s.hi, rays)
    assert np.array_equal(ho.cpu().numpy().view(np.uint32), oo)
    assert np.array_equal(ht.cpu().numpy().view(np.uint32), ot.view(np.uint32))
    assert (oo != 0xFFFFFFFF).sum() >= 12
