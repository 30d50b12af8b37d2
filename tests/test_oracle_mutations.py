"""The oracle's pins catch plausible mistakes.

Each case plants one mistake (a wrong index, a dropped term, a flipped sign, a
swapped operand) into a private copy of the oracle's source, compiles it on the
CPU, and checks that the brute-force and GlobalCoords pins reject it.  The
oracle itself is never modified.
"""
import ctypes as C
import multiprocessing as mp
import os
import subprocess

import numpy as np
import pytest

import oracle
from brute import brute_pairs, dyadic_scene

SRC = open(oracle._SRC).read()

MUTATIONS = {
    "globalcoords_z_divisor": ("uint32_t z = rid / (m[0] * m[1]);", "uint32_t z = rid / (m[0] * m[2]);"),
    "globalcoords_x_term": ("rid - m[0] * (y + m[1] * z)", "rid - m[0] * (y + m[0] * z)"),
    "globalcoords_y_offset": ("out[1] = box_lo[1] + y;", "out[1] = box_lo[0] + y;"),
    "linearise_transposed": ("g[0] + res[0] * (g[1] + res[1] * g[2])", "g[0] + res[1] * (g[1] + res[0] * g[2])"),
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
}


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
    return L


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _pins_pass(L) -> bool:
    """Run the brute-force and GlobalCoords pins against library L."""
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
    old, new = MUTATIONS[name]
    assert SRC.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    # a crash (e.g. a division by a zero extent) also counts as caught
    assert _run_pins(tmp_path, name, SRC.replace(old, new)) != 0, f"planted mistake {name} was not caught"
