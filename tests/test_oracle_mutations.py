"""The oracle's pins catch plausible mistakes.

Each case plants one mistake (a wrong index, a dropped term, a flipped sign, a
swapped operand) into a private copy of the oracle's source, compiles it on the
CPU, and checks that the brute-force, GlobalCoords and FP32 cell-face pins
reject it.  The oracle itself is never modified.
"""
import ctypes as C
import multiprocessing as mp
import os
import subprocess

import numpy as np
import pytest

import fp32_model
import oracle
from brute import brute_pairs, dyadic_scene

SRC = open(oracle._SRC).read()

MUTATIONS = {
    "globalcoords_z_divisor": ("uint32_t z = rid / (m[0] * m[1]);", "uint32_t z = rid / (m[0] * m[2]);"),
    "globalcoords_x_term": ("rid - m[0] * (y + m[1] * z)", "rid - m[0] * (y + m[0] * z)"),
    "globalcoords_y_offset": ("out[1] = box_lo[1] + y;", "out[1] = box_lo[0] + y;"),
    "linearise_transposed": ("return g[0] + res[0] * (g[1] + res[1] * g[2]);",
                             "return g[0] + res[1] * (g[1] + res[0] * g[2]);"),
    "map_round_not_floor": ("float f = std::floor(u);", "float f = std::round(u);"),
    "map_no_low_clamp": ("f = std::fmax(f, 0.0f);", ""),
    "map_wrong_sign": ("float s = p - lo;", "float s = lo - p;"),
    "inv_inverted": ("inv[a] = static_cast<float>(res[a]) / ext;", "inv[a] = ext / static_cast<float>(res[a]);"),
    "extent_off_by_one": ("box_m[3 * static_cast<size_t>(t) + a] = ch - cl + 1;\n      c *= ch - cl + 1;",
                          "box_m[3 * static_cast<size_t>(t) + a] = ch - cl;\n      c *= ch - cl + 1;"),
    "pmin_uses_max": ("float pmin = std::fmin(std::fmin(p0, p1), p2);", "float pmin = std::fmin(std::fmax(p0, p1), p2);"),
    "sort_descending": ("return cells[a] < cells[b];", "return cells[a] > cells[b];"),
    "ranges_begin_after_add": ("ranges[2 * c] = static_cast<uint32_t>(acc);\n    acc += per_cell[c];",
                               "acc += per_cell[c];\n    ranges[2 * c] = static_cast<uint32_t>(acc);"),
    # the cell width w = (hi - lo) / res, and the map divides by it instead of multiplying by inv
    "map_divides_by_cell_width": [("inv[a] = static_cast<float>(res[a]) / ext;", "inv[a] = ext / static_cast<float>(res[a]);"),
                                  ("float u = s * inv;", "float u = s / inv;")],
    # the subtraction and the product carried in double precision
    "map_double_intermediate": ("float s = p - lo;\n  float u = s * inv;\n  float f = std::floor(u);",
                                "double s = static_cast<double>(p) - lo;\n  double u = s * inv;\n"
                                "  float f = static_cast<float>(std::floor(u));"),
    # removal of false intersections
    "cull_edge_axis_component": ("const float ax[3] = {0.0f, e[i][2], -e[i][1]};",
                                 "const float ax[3] = {0.0f, e[i][1], -e[i][2]};"),
    "cull_normal_component": ("e[0][2] * e[1][0] - e[0][0] * e[1][2]", "e[0][2] * e[1][0] - e[0][1] * e[1][2]"),
    "cull_no_normal_axis": ("  if (axis_separates(n, u, b)) return false;\n", ""),
    "cull_margin_shrinks": ("const float above = (tmax + mg) - lo_off;", "const float above = (tmax - mg) - lo_off;"),
    "cull_box_offset_swapped": ("const float below = (tmin - mg) - hi_off;", "const float below = (tmin - mg) - lo_off;"),
    # ray casting
    "ray_det_sign_ignored": ("  if (det < 0.0f) {\n    det = -det;\n    u = -u;\n    v = -v;\n    tn = -tn;\n  }\n", ""),
    "ray_q_cross_swapped": ("cross3(s, e1, q);", "cross3(e1, s, q);"),
    "ray_clip_ignores_box": ("  *t0 = a0;\n  *t1 = a1;\n  return a0 <= a1;", "  *t0 = 0.0f;\n  *t1 = tmax;\n  return true;"),
    "ray_tie_keeps_last": ("th >= t0 && th <= t1 && th < best", "th >= t0 && th <= t1 && th <= best"),
    "ray_t_from_u": ("return tn / det;", "return u / det;"),
}


def _edits(name):
    m = MUTATIONS[name]
    return m if isinstance(m, list) else [m]


def _compile(tmp_path, name, src):
    cpp = tmp_path / f"{name}.cpp"
    so = tmp_path / f"{name}.so"
    cpp.write_text(src)
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-ffp-contract=off", "-fPIC", "-shared", "-o", str(so), str(cpp)])
    L = C.CDLL(str(so))
    P = C.c_void_p
    L.oracle_build.argtypes = [P, C.c_uint32, P, C.c_uint32, P, P, P, P, P, P, C.c_uint64, P]
    L.oracle_build.restype = C.c_int
    L.oracle_global_coords.argtypes = [P, P, C.c_uint32, P]
    L.oracle_count_cells.argtypes = [P, C.c_uint32, P, C.c_uint32, P, P, P, P, P, P]
    L.oracle_count_cells.restype = C.c_int
    L.oracle_make_pairs_culled.argtypes = [P, C.c_uint32, P, C.c_uint32, P, P, P, P, P, P, P, P, P]
    L.oracle_make_pairs_culled.restype = C.c_uint64
    L.oracle_raycast.argtypes = [P, C.c_uint32, P, C.c_uint32, P, P, P, C.c_uint32, C.c_float, P, P]
    return L


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _face_cases():
    """Degenerate triangles at and beside the cell faces of two non-dyadic grids,
    with each corner's cell from the exact rational model of the FP32 map."""
    cases = []
    rng = np.random.default_rng(7)
    for lo, hi, res in (((0.0, -3.7, 11.3), (17.219383, 41.9, 12.05), (112, 333, 77)),
                        ((-51.4, 2.2, 0.1), (60.7, 9.3, 93.3), (1001, 71, 619))):
        lo = np.asarray(lo, np.float32)
        hi = np.asarray(hi, np.float32)
        res = np.asarray(res, np.uint32)
        pts = []
        for a in range(3):
            ks = rng.integers(0, int(res[a]) + 1, size=60)
            p = np.asarray([float(lo[a]) + int(k) * (float(hi[a]) - float(lo[a])) / int(res[a]) for k in ks], np.float32)
            up = np.nextafter(p, np.float32(np.inf))
            dn = np.nextafter(p, np.float32(-np.inf))
            pts.append(np.concatenate([p, up, dn]))
        n = len(pts[0])
        verts = np.ascontiguousarray(np.repeat(np.stack(pts), 3, axis=1), np.float32)   # 3 equal vertices each
        tris = np.arange(3 * n, dtype=np.uint32).reshape(n, 3)
        want = np.asarray([[fp32_model.cell_fp32(pts[a][t], lo[a], hi[a], int(res[a])) for a in range(3)]
                           for t in range(n)], np.uint32)
        cases.append((verts, tris, lo, hi, res, want))
    return cases


_FACE_CASES = None


def _faces_pass(L) -> bool:
    global _FACE_CASES
    if _FACE_CASES is None:
        _FACE_CASES = _face_cases()
    for verts, tris, lo, hi, res, want in _FACE_CASES:
        t = tris.shape[0]
        box_lo = np.zeros((t, 3), np.uint32)
        box_m = np.zeros((t, 3), np.uint32)
        cnt = np.zeros(t, np.uint32)
        st = L.oracle_count_cells(_p(verts), verts.shape[1], _p(tris), t, _p(lo), _p(hi), _p(res),
                                  _p(box_lo), _p(box_m), _p(cnt))
        if st != 0 or not np.array_equal(box_lo, want) or not (box_m == 1).all():
            return False
    return True


def _cull_cases():
    """Scenes of slivers and random triangles on non-dyadic grids, with every box
    cell's exact touch (rational clip of the FP32 grid coordinates by the cell)
    and near-touch (the cell widened by twice the margin)."""
    from fractions import Fraction
    from brute import triangle_touches_box
    from paper_2403_10647_amd import scenes
    cases = []
    for seed in (3, 4):
        rng = np.random.default_rng(seed)
        lo = rng.uniform(-5, 5, size=3).astype(np.float32)
        hi = (lo + rng.uniform(4.1, 8.9, size=3)).astype(np.float32)
        res = rng.integers(6, 12, size=3).astype(np.uint32)
        a = rng.uniform(lo + 0.1, hi - 0.1, size=(20, 3))
        b = rng.uniform(lo + 0.1, hi - 0.1, size=(20, 3))
        w = np.clip(b + rng.normal(size=(20, 3)) * 0.3, lo + 0.05, hi - 0.05)
        verts, tris = scenes.soup_from_vertices(np.stack([a, b, w], axis=1))
        box_lo, box_m, count = oracle.count_cells(verts, tris, lo, hi, res)
        m2 = 2 * Fraction(1, 64)
        want = []
        for t in range(tris.shape[0]):
            u = []
            for j in range(3):
                u.append(tuple(fp32_model.rn32(fp32_model.rn32(fp32_model.exact(verts[ax][tris[t, j]])
                                                               - fp32_model.exact(lo[ax]))
                                               * fp32_model.inv_cell(lo[ax], hi[ax], int(res[ax]))) for ax in range(3)))
            for z in range(int(box_m[t, 2])):
                for y in range(int(box_m[t, 1])):
                    for x in range(int(box_m[t, 0])):
                        c = (int(box_lo[t, 0]) + x, int(box_lo[t, 1]) + y, int(box_lo[t, 2]) + z)
                        cid = c[0] + int(res[0]) * (c[1] + int(res[1]) * c[2])
                        touch = triangle_touches_box(u, c, tuple(v + 1 for v in c))
                        near = triangle_touches_box(u, tuple(v - m2 for v in c), tuple(v + 1 + m2 for v in c))
                        want.append((t, cid, touch, near, int(count[t]) <= 2))
        cases.append((verts, tris, lo, hi, res, box_lo, box_m, count, want))
    return cases


_CULL_CASES = None


def _cull_pass(L) -> bool:
    global _CULL_CASES
    if _CULL_CASES is None:
        _CULL_CASES = _cull_cases()
    for verts, tris, lo, hi, res, box_lo, box_m, count, want in _CULL_CASES:
        nbox = int(count.sum())
        cells = np.zeros(nbox, np.uint32)
        objs = np.zeros(nbox, np.uint32)
        kept = np.zeros(tris.shape[0], np.uint32)
        n = L.oracle_make_pairs_culled(_p(verts), verts.shape[1], _p(tris), tris.shape[0], _p(lo), _p(hi), _p(res),
                                       _p(box_lo), _p(box_m), _p(count), _p(cells), _p(objs), _p(kept))
        got = set(zip(objs[:n].tolist(), cells[:n].tolist()))
        dropped = 0
        for t, cid, touch, near, whole in want:
            k = (t, cid) in got
            if (whole or touch) and not k:
                return False
            if k and not near:
                return False
            dropped += not k
        if dropped == 0:
            return False
    return True


def _raycast_pass(L) -> bool:
    import raycast_pins

    def fn(verts, tris, lo, hi, rays, tmax):
        verts, tris = np.ascontiguousarray(verts, np.float32), np.ascontiguousarray(tris, np.uint32)
        lo, hi = np.ascontiguousarray(lo, np.float32), np.ascontiguousarray(hi, np.float32)
        rays = np.ascontiguousarray(rays, np.float32)
        n = rays.shape[1]
        ht, ho = np.zeros(n, np.float32), np.zeros(n, np.uint32)
        L.oracle_raycast(_p(verts), verts.shape[1], _p(tris), tris.shape[0], _p(lo), _p(hi), _p(rays), n,
                         C.c_float(tmax), _p(ht), _p(ho))
        return ht, ho
    return raycast_pins.check(fn)


def _pins_pass(L) -> bool:
    """Run the brute-force, GlobalCoords, FP32 cell-face, culling and ray-casting pins against library L."""
    if not _faces_pass(L) or not _cull_pass(L) or not _raycast_pass(L):
        return False
    lo5 = np.array([5, 7, 11], np.uint32)
    for m in [(2, 3, 4), (3, 1, 2), (4, 4, 1)]:
        m = np.asarray(m, np.uint32)
        out = np.zeros(3, np.uint32)
        want = [(5 + x, 7 + y, 11 + z) for z in range(m[2]) for y in range(m[1]) for x in range(m[0])]
        for r, w in enumerate(want):
            L.oracle_global_coords(_p(lo5), _p(m), r, _p(out))
            if tuple(out) != w:
                return False
    grids = [((0, 0, 0), (8, 8, 8), (8, 8, 8)), ((-4, 0, 2), (4, 8, 6), (16, 4, 8))]
    for seed in range(3):
        for lo, hi, res in grids:
            lo = np.asarray(lo, np.float32)
            hi = np.asarray(hi, np.float32)
            res = np.asarray(res, np.uint32)
            verts, tris = dyadic_scene(np.random.default_rng(seed), 30, float(lo.min()), float(hi.max()), 1.5)
            want = brute_pairs(verts, tris, lo, hi, res)
            ncell = int(np.prod(res.astype(np.int64)))
            cap = 4 * len(want) + 64
            cells = np.zeros(cap, np.uint32)
            objs = np.zeros(cap, np.uint32)
            rg = np.zeros(2 * ncell, np.uint32)
            no = np.zeros(1, np.uint64)
            st = L.oracle_build(_p(verts), verts.shape[1], _p(tris), tris.shape[0], _p(lo), _p(hi), _p(res),
                                _p(cells), _p(objs), _p(rg), cap, _p(no))
            if st != 0:
                return False
            n = int(no[0])
            if list(zip(cells[:n].tolist(), objs[:n].tolist())) != want:
                return False
            bc = np.asarray([c for c, _ in want], np.int64)
            ar = np.arange(ncell)
            if not (np.array_equal(rg[0::2], np.searchsorted(bc, ar, "left"))
                    and np.array_equal(rg[1::2], np.searchsorted(bc, ar, "right"))):
                return False
    return True


def _child(tmp_path, name, src):
    import faulthandler
    faulthandler.disable()
    os._exit(0 if _pins_pass(_compile(tmp_path, name, src)) else 1)


def _run_pins(tmp_path, name, src) -> int:
    """Exit code of the pins run in a forked child: 0 pass, 1 fail, <0 crash."""
    p = mp.get_context("fork").Process(target=_child, args=(tmp_path, name, src))
    p.start()
    p.join(120)
    if p.is_alive():
        p.kill()
        p.join()
        return -999
    return p.exitcode


def test_unmutated_copy_passes(tmp_path):
    assert _run_pins(tmp_path, "clean", SRC) == 0


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(tmp_path, name):
    src = SRC
    for old, new in _edits(name):
        assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
        src = src.replace(old, new)
    # a crash (e.g. a division by a zero extent) also counts as caught
    assert _run_pins(tmp_path, name, src) != 0, f"planted mistake {name} was not caught"


@pytest.mark.parametrize("name", ["map_divides_by_cell_width", "map_double_intermediate"])
def test_fp32_mutation_survives_dyadic_pins(tmp_path, name):
    # these two mistakes agree with exact arithmetic on dyadic inputs, so only the
    # cell-face pins on non-dyadic grids can catch them: check that they do
    src = SRC
    for old, new in _edits(name):
        src = src.replace(old, new)
    L = _compile(tmp_path, name, src)
    assert not _faces_pass(L)
