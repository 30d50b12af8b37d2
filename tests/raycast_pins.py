"""Pins of the oracle's ray casting (the closest hit by brute force), against
what geometry fixes, independently of the oracle's FP32 formula:

* hand cases with exact answers: a ray straight onto a triangle at a known
  distance, a miss beside it, the nearer of two stacked triangles from either
  side, a tie between two copies of one triangle (the smaller id), a ray in a
  triangle's plane (grazing: no hit), a degenerate triangle, a hit outside the
  grid box (not counted) and a hit cut off by tmax;
* random rays through random triangles (some outside the grid box) against a
  float64 reference written another way (the plane hit point, then the
  inside-of-every-edge test), wherever that reference's answer is clear of
  edges, grazing angles, near-ties and the box's faces.

``check(fn)`` takes a function (verts, tris, lo, hi, rays, tmax) -> (t, id)."""
import numpy as np

INF = np.float32(np.inf)
NOHIT = np.uint32(0xFFFFFFFF)


def _soup(tri):
    v = np.asarray(tri, np.float64).reshape(-1, 3, 3)
    verts = np.ascontiguousarray(v.transpose(2, 0, 1).reshape(3, -1), np.float32)
    tris = np.arange(3 * v.shape[0], dtype=np.uint32).reshape(-1, 3)
    return verts, tris


def _rays(o, d):
    return np.ascontiguousarray(np.concatenate([np.asarray(o, np.float64).T, np.asarray(d, np.float64).T]), np.float32)


def hand_cases_pass(fn) -> bool:
    lo, hi = np.zeros(3, np.float32), np.ones(3, np.float32)
    a = [[0.0, 0.0, 0.5], [1.0, 0.0, 0.5], [0.0, 1.0, 0.5]]           # z = 0.5
    b = [[0.0, 0.0, 0.25], [1.0, 0.0, 0.25], [0.0, 1.0, 0.25]]        # z = 0.25
    deg = [[0.1, 0.1, 0.75], [0.5, 0.5, 0.75], [0.9, 0.9, 0.75]]      # collinear: no area
    far = [[0.0, 0.0, 1.5], [1.0, 0.0, 1.5], [0.0, 1.0, 1.5]]         # outside the box
    verts, tris = _soup([a, b, a, deg, far])                          # ids 0 and 2 are the same triangle
    o = [[0.2, 0.2, 1.0], [0.8, 0.8, 1.0], [0.2, 0.2, 0.0], [0.3, 0.1, 0.5], [0.3, 0.3, 0.9], [0.2, 0.2, 2.0],
         [0.2, 0.2, 1.0], [0.5, 0.5, 1.0]]
    d = [[0, 0, -1], [0, 0, -1], [0, 0, 1], [1, 0, 0], [0, 0, 1], [0, 0, -1], [0, 0, -2], [0, 0, -1]]
    t, i = fn(verts, tris, lo, hi, _rays(o, d), np.float32(np.inf))
    want_t = [0.5, INF, 0.25, INF, INF, 1.5, 0.25, 0.5]
    want_i = [0, NOHIT, 1, NOHIT, NOHIT, 0, 0, 0]
    if not (np.array_equal(t, np.asarray(want_t, np.float32)) and np.array_equal(i, np.asarray(want_i, np.uint32))):
        return False
    # tmax cuts the first hit off; then the second is the one
    t, i = fn(verts, tris, lo, hi, _rays([[0.2, 0.2, 1.0]], [[0, 0, -1]]), np.float32(0.6))
    return t[0] == np.float32(0.5) and i[0] == 0 and \
        fn(verts, tris, lo, hi, _rays([[0.2, 0.2, 1.0]], [[0, 0, -1]]), np.float32(0.4))[1][0] == NOHIT


def _clip64(o, d, lo, hi, tmax):
    t0, t1 = 0.0, tmax
    for a in range(3):
        if d[a] != 0:
            ta, tb = (lo[a] - o[a]) / d[a], (hi[a] - o[a]) / d[a]
            t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
        elif not (lo[a] <= o[a] <= hi[a]):
            return None
    return (t0, t1) if t0 <= t1 else None


def _hits64(o, d, v):
    """For rays (o, d: [n, 3]) and triangles v [m, 3, 3], in float64: the hit t
    of every pair ([n, m], inf on a miss) and the clearance of the hit point
    from the triangle's edges relative to its size ([n, m]; 0 where the pair is
    grazing or the triangle degenerate, so that such pairs count as unclear)."""
    p0, p1, p2 = v[:, 0], v[:, 1], v[:, 2]
    nrm = np.cross(p1 - p0, p2 - p0)                                  # [m, 3]
    nn = np.linalg.norm(nrm, axis=1)                                  # [m]
    denom = d @ nrm.T                                                 # [n, m]
    dn = np.linalg.norm(d, axis=1)[:, None]
    ok = (nn[None, :] > 0) & (np.abs(denom) >= 1e-3 * nn[None, :] * dn)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = ((p0 * nrm).sum(1)[None, :] - o @ nrm.T) / denom          # n . (p0 - o) / n . d
        x = o[:, None, :] + t[:, :, None] * d[:, None, :]             # [n, m, 3]
        size = np.maximum.reduce([np.linalg.norm(p1 - p0, axis=1), np.linalg.norm(p2 - p1, axis=1),
                                  np.linalg.norm(p0 - p2, axis=1)])
        s = [np.einsum("nmk,mk->nm", np.cross(q1 - q0, x - q0[None]), nrm) / nn[None, :]
             for q0, q1 in ((p0, p1), (p1, p2), (p2, p0))]
        smin = np.minimum.reduce(s)
        clear = np.minimum.reduce([np.abs(z) for z in s]) / size[None, :]
    hit = np.where(ok & (smin >= 0), t, np.inf)
    clear = np.where(ok, clear, 0.0)
    return hit, clear


def random_cases_pass(fn, seed: int = 0) -> bool:
    rng = np.random.default_rng(seed)
    lo, hi = np.array([-1.0, -2.0, 0.5], np.float32), np.array([3.0, 1.5, 4.0], np.float32)
    c = rng.uniform(lo - 0.5, hi + 0.5, size=(80, 1, 3))                # some triangles reach outside the box
    v = c + rng.normal(size=(80, 3, 3)) * 0.6
    verts, tris = _soup(v)
    n = 3000
    o = rng.uniform(lo - 1.0, hi + 1.0, size=(n, 3))
    d = rng.normal(size=(n, 3))
    rays = _rays(o, d)
    t, i = fn(verts, tris, lo, hi, rays, np.float32(np.inf))
    v32 = verts.astype(np.float64).T.reshape(-1, 3, 3)
    O, D = rays[:3].T.astype(np.float64), rays[3:].T.astype(np.float64)
    H, CL = _hits64(O, D, v32)
    checked = hits = 0
    for r in range(n):
        oo, dd = O[r], D[r]
        box = _clip64(oo, dd, lo.astype(np.float64), hi.astype(np.float64), np.inf)
        if box is None:
            checked += 1
            if not (i[r] == NOHIT and t[r] == INF):
                return False
            continue
        t0, t1 = box
        span = max(1.0, abs(t1))
        h = H[r]
        fin = h[np.isfinite(h)]
        # unclear: an edge passes within 1e-4 of the hit point, a hit within 1e-4 of a box face, or a near tie
        if (CL[r] < 1e-4).any() or (np.abs(fin - t0) < 1e-4 * span).any() or (np.abs(fin - t1) < 1e-4 * span).any():
            continue
        ks = np.nonzero(np.isfinite(h) & (h >= t0) & (h <= t1))[0]
        inside = sorted((float(h[k]), int(k)) for k in ks)
        if len(inside) > 1 and inside[1][0] - inside[0][0] < 1e-4 * span:
            continue
        checked += 1
        if not inside:
            if i[r] != NOHIT or t[r] != INF:
                return False
        else:
            hits += 1
            tt, k = inside[0]
            if i[r] != k or abs(float(t[r]) - tt) > 1e-5 * max(1.0, abs(tt)):
                return False
    return checked > 2000 and hits > 300


def check(fn) -> bool:
    return hand_cases_pass(fn) and random_cases_pass(fn)
