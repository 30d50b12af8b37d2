"""Randomised GPU parity: many small random scenes (random resolutions with
1-cell axes, tiny and huge triangles, geometry outside the bounds, now and then
NaN or infinite vertices), each built plain and in batches and compared with the
oracle element by element."""
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


def random_scene(seed: int) -> scenes.Scene:
    rng = np.random.default_rng(np.random.SeedSequence(entropy=1234, spawn_key=(seed,)))
    t = int(rng.choice([0, 1, 2, 7, 100, 1000, 4096, 9000]))
    lo = rng.uniform(-5, 5, size=3)
    ext = rng.uniform(0.5, 20, size=3)
    hi = lo + ext
    res = np.asarray([int(rng.choice([1, 2, 3, 17, 64, 100])) for _ in range(3)], np.uint32)
    cen = lo + rng.uniform(-0.2, 1.2, size=(t, 3)) * ext          # some outside the bounds
    size = np.where(rng.random((t, 1)) < 0.1, ext * rng.uniform(0.1, 1.5, size=(t, 3)),
                    ext * rng.uniform(0, 0.05, size=(t, 3)))     # mostly small, some huge
    v = cen[:, None, :] + rng.uniform(-1, 1, size=(t, 3, 3)) * size[:, None, :]
    if t and rng.random() < 0.3:
        bad = rng.integers(0, t, size=max(1, t // 100))
        v[bad, rng.integers(0, 3), rng.integers(0, 3)] = rng.choice([np.nan, np.inf, -np.inf])
    verts, tris = scenes.soup_from_vertices(v)
    return scenes.Scene(f"random{seed}", verts, tris, lo.astype(np.float32), hi.astype(np.float32), res)


def _same(r, s):
    c, o, rg = r.numpy()
    oc, oo, orr = oracle.build_scene(s)
    assert r.npairs == len(oc), s.name
    assert np.array_equal(c, oc), s.name
    assert np.array_equal(o, oo), s.name
    assert np.array_equal(rg, orr), s.name


def test_random_scenes_plain(G):
    ws = G.Workspace()
    for seed in range(60):
        s = random_scene(seed)
        if not np.all(s.hi > s.lo):
            continue
        print("random plain", seed, s.ntris, list(s.res), flush=True)
        _same(G.build(G.GridInput.from_scene(s), ws=ws), s)


def test_random_scenes_batched(G):
    ws = G.Workspace()
    for b in range(6):
        batch = [random_scene(1000 + 10 * b + i) for i in range(10)]
        print("random batch", b, [s.ntris for s in batch], flush=True)
        res = G.build_batched([G.GridInput.from_scene(s) for s in batch], ws=ws)
        for r, s in zip(res, batch):
            _same(r, s)
