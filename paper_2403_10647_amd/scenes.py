"""Seeded synthetic triangle soups shaped like the paper's test scenes.

The paper measures on seven public scenes (Section "Test Procedure", Table 1);
none of them are available here, so these generators stand in for them:

* ``small``  - 4096 small triangles in the unit cube on a fixed 32^3 grid.
* ``mixed``  - 1M triangles, 95% small and 5% large (per-axis half-widths
  log-uniform), the strongly non-homogeneous case the paper targets, where the
  largest boxes cover orders of magnitude more cells than the average one
  (Table 1, "max # cells / item" against "avg # cells / item").
* ``arch``   - a 10M-triangle architectural-style scene (10k wall/floor
  rectangles plus 2000 Gaussian clusters of tiny triangles) in a 100x10x100 box,
  the size class of the paper's 10M-triangle real-time claim (abstract).
* ``batch``  - 512 independent ``mixed``-style grids with log-uniform
  triangle counts in [1e3, 2e5].
* ``uniform`` - ``mixed`` without its large triangles: small triangles spread
  evenly, the homogeneous case (about four cells per triangle).
* ``hairball`` - long, thin, diagonal slivers (strands of random direction,
  lengths log-uniform in [0.3, 3], widths near 1% of the length) in a
  [0, 10]^3 box: the shape of the paper's Hairball scene, whose triangles'
  boxes hold many cells the triangles never touch (Test Results).

This module holds no part of the grid-building arithmetic: it only draws
vertices, picks the grid bounds (the vertices' FP32 bounding box) and the grid
resolution (the harness's cell-size rule, which the paper leaves open in
"Conclusions and Future Work").  Both the oracle and the GPU path consume its
output; neither is imported here.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

__all__ = [
    "Scene", "make_scene", "make_batch", "batch_sizes", "soup_from_vertices",
    "resolution_rule", "aabb_bounds", "SCENE_NAMES", "make_rays",
]

SCENE_NAMES = ("small", "mixed", "arch", "batch", "hairball", "uniform")
_STREAM = {"small": 0, "mixed": 1, "arch": 2, "batch": 3, "serve": 4, "hairball": 5, "uniform": 6, "rays": 7}


@dataclasses.dataclass
class Scene:
    """One grid-build request: a triangle soup plus the grid it is binned into.

    verts : float32 [3, V], structure-of-arrays (x block, y block, z block)
    tris  : uint32 [T, 3], vertex indices
    lo, hi: float32 [3], grid bounds
    res   : uint32 [3], cells per axis
    """
    name: str
    verts: np.ndarray
    tris: np.ndarray
    lo: np.ndarray
    hi: np.ndarray
    res: np.ndarray
    seed: int = 0

    @property
    def ntris(self) -> int:
        return int(self.tris.shape[0])

    @property
    def nverts(self) -> int:
        return int(self.verts.shape[1])

    @property
    def ncells(self) -> int:
        return int(np.prod(self.res.astype(np.int64)))


def _rng(seed: int, *key: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(entropy=seed, spawn_key=tuple(key)))


def soup_from_vertices(v: np.ndarray):
    """[T, 3 vertices, 3 coords] float -> (verts f32 [3, 3T], tris u32 [T, 3]).

    Triangle t owns vertices 3t, 3t+1, 3t+2 (an unindexed soup)."""
    t = v.shape[0]
    verts = np.ascontiguousarray(v.astype(np.float32).reshape(t * 3, 3).T)
    tris = np.arange(3 * t, dtype=np.uint32).reshape(t, 3)
    return verts, tris


def aabb_bounds(verts: np.ndarray):
    """FP32 axis-aligned bounding box of all vertices (the grid bounds); the unit
    cube when there are none, and never empty along an axis."""
    if verts.shape[1] == 0:
        return np.zeros(3, np.float32), np.ones(3, np.float32)
    lo = verts.min(axis=1).astype(np.float32)
    hi = verts.max(axis=1).astype(np.float32)
    hi = np.where(hi > lo, hi, np.nextafter(lo, np.float32(np.inf))).astype(np.float32)
    return lo, hi


def resolution_rule(lo, hi, ntris: int, lam: float, cap: int) -> np.ndarray:
    """res_a = min(cap, max(1, ceil(ext_a * cbrt(lam * N / volume)))), in float64.

    This is the harness's cell-size rule: about ``lam`` cells per triangle,
    cells as close to cubes as the bounds allow."""
    ext = np.maximum(np.asarray(hi, np.float64) - np.asarray(lo, np.float64), 1e-30)
    k = math.pow(lam * max(ntris, 1) / float(np.prod(ext)), 1.0 / 3.0)
    res = [min(cap, max(1, int(math.ceil(e * k)))) for e in ext]
    return np.asarray(res, dtype=np.uint32)


def _small_large(rng: np.random.Generator, n: int, box: float = 10.0):
    """The 95% small / 5% large mix: centroids uniform in [0, box]^3."""
    n_large = n // 20
    n_small = n - n_large
    c = rng.uniform(0.0, box, size=(n, 1, 3))
    off_small = rng.uniform(-0.05, 0.05, size=(n_small, 3, 3))
    h = np.exp(rng.uniform(math.log(0.05), math.log(3.0), size=(n_large, 1, 3)))
    off_large = rng.uniform(-1.0, 1.0, size=(n_large, 3, 3)) * h
    off = np.concatenate([off_small, off_large], axis=0)
    off = off[rng.permutation(n)]
    return c + off


def _small_scene(seed: int, ntris: int = 4096) -> Scene:
    rng = _rng(seed, _STREAM["small"])
    c = rng.uniform(0.0, 1.0, size=(ntris, 1, 3))
    v = c + rng.uniform(-0.02, 0.02, size=(ntris, 3, 3))
    verts, tris = soup_from_vertices(v)
    return Scene("small", verts, tris, np.zeros(3, np.float32), np.ones(3, np.float32),
                 np.full(3, 32, np.uint32), seed)


def _mixed_scene(seed: int, ntris: int = 1_000_000, lam: float = 4.0, cap: int = 512,
                 key=(1,), name: str = "mixed") -> Scene:
    rng = _rng(seed, *key)
    v = _small_large(rng, ntris)
    verts, tris = soup_from_vertices(v)
    lo, hi = aabb_bounds(verts)
    return Scene(name, verts, tris, lo, hi, resolution_rule(lo, hi, ntris, lam, cap), seed)


def _unit_sphere(rng: np.random.Generator, shape):
    u = rng.normal(size=tuple(shape) + (3,))
    n = np.linalg.norm(u, axis=-1, keepdims=True)
    n[n == 0] = 1.0
    return u / n


def _arch_scene(seed: int, ntris: int = 10_000_000, nwalls: int = 10_000,
                nclusters: int = 2000, lam: float = 2.0, cap: int = 1024) -> Scene:
    rng = _rng(seed, _STREAM["arch"])
    box = np.array([100.0, 10.0, 100.0])
    # Walls and floors: axis-aligned rectangles on random x, y or z planes.
    axis = rng.integers(0, 3, size=nwalls)
    plane = rng.uniform(0.0, 1.0, size=nwalls) * box[axis]
    corner = rng.uniform(0.0, 1.0, size=(nwalls, 3)) * box
    side = np.exp(rng.uniform(0.0, math.log(50.0), size=(nwalls, 2)))
    quads = np.empty((nwalls, 4, 3))
    for w in range(3):
        sel = axis == w
        a1, a2 = [x for x in range(3) if x != w]
        c1, c2 = corner[sel, a1], corner[sel, a2]
        e1 = np.minimum(c1 + side[sel, 0], box[a1])
        e2 = np.minimum(c2 + side[sel, 1], box[a2])
        q = quads[sel]
        q[:, :, w] = plane[sel, None]
        q[:, 0, a1], q[:, 0, a2] = c1, c2
        q[:, 1, a1], q[:, 1, a2] = e1, c2
        q[:, 2, a1], q[:, 2, a2] = e1, e2
        q[:, 3, a1], q[:, 3, a2] = c1, e2
        quads[sel] = q
    walls = np.concatenate([quads[:, [0, 1, 2]], quads[:, [0, 2, 3]]], axis=0)
    # Clusters of tiny triangles around Gaussian centres; every triangle lands
    # at a random position of the soup (walls interleaved with clutter).
    nw = walls.shape[0]
    ncl = ntris - nw
    perm = rng.permutation(ntris)
    soup = np.empty((ntris, 3, 3), np.float32)
    soup[perm[:nw]] = walls
    centres = rng.uniform(0.0, 1.0, size=(nclusters, 3)) * box
    chunk = 1 << 20
    for s in range(0, ncl, chunk):
        e = min(ncl, s + chunk)
        n = e - s
        which = rng.integers(0, nclusters, size=n)
        cen = centres[which] + rng.normal(0.0, 0.5, size=(n, 3))
        r = rng.lognormal(math.log(0.02), 0.5, size=(n, 3, 1))
        soup[perm[nw + s:nw + e]] = cen[:, None, :] + r * _unit_sphere(rng, (n, 3))
    verts, tris = soup_from_vertices(soup)
    del soup
    lo, hi = aabb_bounds(verts)
    return Scene("arch", verts, tris, lo, hi, resolution_rule(lo, hi, ntris, lam, cap), seed)


def batch_sizes(seed: int, ngrids: int = 512, tmin: float = 1e3, tmax: float = 2e5,
                stream: int = _STREAM["batch"]) -> np.ndarray:
    """Per-grid triangle counts, log-uniform in [tmin, tmax]."""
    rng = _rng(seed, stream, 0)
    return np.floor(np.exp(rng.uniform(math.log(tmin), math.log(tmax), size=ngrids))).astype(np.int64)


def make_batch(seed: int = 0, ngrids: int = 512, sizes: Optional[np.ndarray] = None,
               stream: int = _STREAM["batch"]) -> List[Scene]:
    """``ngrids`` independent mixed-style scenes, each with its own bounds and resolution."""
    if sizes is None:
        sizes = batch_sizes(seed, ngrids, stream=stream)
    out = []
    for g, n in enumerate(sizes):
        out.append(_mixed_scene(seed, int(n), 4.0, 512, key=(stream, 1, g), name=f"batch{g}"))
    return out


def _hairball_scene(seed: int, ntris: int = 1_000_000, lam: float = 4.0, cap: int = 512) -> Scene:
    """Slivers: vertex a uniform in the box, b = a + L d (L log-uniform in
    [0.3, 3], d uniform on the sphere), c = b + w e with e a unit vector and w
    log-uniform in [0.003, 0.03]."""
    rng = _rng(seed, _STREAM["hairball"])
    a = rng.uniform(0.0, 10.0, size=(ntris, 3))
    length = np.exp(rng.uniform(math.log(0.3), math.log(3.0), size=(ntris, 1)))
    b = a + length * _unit_sphere(rng, (ntris,))
    w = np.exp(rng.uniform(math.log(0.003), math.log(0.03), size=(ntris, 1)))
    c = b + w * _unit_sphere(rng, (ntris,))
    v = np.stack([a, b, c], axis=1)
    verts, tris = soup_from_vertices(v)
    lo, hi = aabb_bounds(verts)
    return Scene("hairball", verts, tris, lo, hi, resolution_rule(lo, hi, ntris, lam, cap), seed)


def _uniform_scene(seed: int, ntris: int = 1_000_000, lam: float = 4.0, cap: int = 512) -> Scene:
    rng = _rng(seed, _STREAM["uniform"])
    v = rng.uniform(0.0, 10.0, size=(ntris, 1, 3)) + rng.uniform(-0.05, 0.05, size=(ntris, 3, 3))
    verts, tris = soup_from_vertices(v)
    lo, hi = aabb_bounds(verts)
    return Scene("uniform", verts, tris, lo, hi, resolution_rule(lo, hi, ntris, lam, cap), seed)


def make_scene(name: str, seed: int = 0, ntris: Optional[int] = None) -> Scene:
    """Build one of the named single-grid scenes (``ntris`` rescales it for tests)."""
    if name == "small":
        return _small_scene(seed, ntris or 4096)
    if name == "mixed":
        return _mixed_scene(seed, ntris or 1_000_000)
    if name == "arch":
        if ntris is None:
            return _arch_scene(seed)
        nwalls = max(2, ntris // 1000)
        return _arch_scene(seed, ntris, nwalls=nwalls, nclusters=max(1, ntris // 5000))
    if name == "hairball":
        return _hairball_scene(seed, ntris or 1_000_000)
    if name == "uniform":
        return _uniform_scene(seed, ntris or 1_000_000)
    raise ValueError(f"unknown scene {name!r}; expected one of small, mixed, arch, hairball, uniform")


def make_rays(scene: Scene, n: int, seed: int = 0, outside: float = 0.3) -> np.ndarray:
    """Seeded rays for queries over a scene's grid, float32 [6, n] (origins x, y,
    z, then directions x, y, z): a share ``outside`` starts outside the grid box
    (one box extent away) and aims at a uniform point inside it; the rest start
    uniformly inside the box with directions uniform on the sphere."""
    rng = _rng(seed, _STREAM["rays"])
    lo = scene.lo.astype(np.float64)
    hi = scene.hi.astype(np.float64)
    ext = hi - lo
    n_out = int(round(n * outside))
    n_in = n - n_out
    o_in = lo + rng.uniform(0.0, 1.0, size=(n_in, 3)) * ext
    d_in = _unit_sphere(rng, (n_in,))
    target = lo + rng.uniform(0.0, 1.0, size=(n_out, 3)) * ext
    o_out = (lo + hi) / 2 + _unit_sphere(rng, (n_out,)) * np.linalg.norm(ext)
    d_out = target - o_out
    o = np.concatenate([o_in, o_out])
    d = np.concatenate([d_in, d_out])
    return np.ascontiguousarray(np.concatenate([o.T, d.T]), np.float32)
