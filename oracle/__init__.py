"""Python face of the serial CPU oracle (``oracle.cpp``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are its only users.  The GPU library never imports, links or
runs it, and it never imports the GPU library.  Inputs come from
``paper_2403_10647_amd.scenes`` (draws only, no grid arithmetic).

Every function follows one step of Algorithm 1 of the paper; the C++ file
states the readings of the points the paper leaves open.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

STATUS = {0: "ok", -1: "invalid argument", -3: "overflow", -4: "capacity", -5: "bad index"}


class OracleError(RuntimeError):
    def __init__(self, status: int):
        super().__init__(f"oracle status {status} ({STATUS.get(status, '?')})")
        self.status = status


def build_library(force: bool = False) -> str:
    """Compile oracle.cpp with g++ (no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build_library())
        P = C.c_void_p
        L.oracle_inv_cell.argtypes = [P, P, P, P]
        L.oracle_count_cells.argtypes = [P, C.c_uint32, P, C.c_uint32, P, P, P, P, P, P]
        L.oracle_count_cells.restype = C.c_int
        L.oracle_exclusive_sum.argtypes = [P, C.c_uint32, P]
        L.oracle_exclusive_sum.restype = C.c_uint64
        L.oracle_global_coords.argtypes = [P, P, C.c_uint32, P]
        L.oracle_make_pairs.argtypes = [C.c_uint32, P, P, P, P, P, P]
        L.oracle_sort_pairs.argtypes = [C.c_uint64, P, P]
        L.oracle_ranges.argtypes = [C.c_uint64, P, C.c_uint64, P]
        L.oracle_build.argtypes = [P, C.c_uint32, P, C.c_uint32, P, P, P, P, P, P, C.c_uint64, P]
        L.oracle_build.restype = C.c_int
        L.oracle_grid_coords.argtypes = [P, C.c_uint32, P, P, P, P, P]
        L.oracle_grid_coords.restype = C.c_int
        L.oracle_touches.argtypes = [P, C.c_uint32, C.c_uint32, C.c_uint32]
        L.oracle_touches.restype = C.c_int
        L.oracle_make_pairs_culled.argtypes = [P, C.c_uint32, P, C.c_uint32, P, P, P, P, P, P, P, P, P]
        L.oracle_make_pairs_culled.restype = C.c_uint64
        L.oracle_build_culled.argtypes = [P, C.c_uint32, P, C.c_uint32, P, P, P, P, P, P, C.c_uint64, P, P]
        L.oracle_build_culled.restype = C.c_int
        L.oracle_raycast.argtypes = [P, C.c_uint32, P, C.c_uint32, P, P, P, C.c_uint32, C.c_float, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _grid_args(lo, hi, res):
    return (np.ascontiguousarray(lo, np.float32), np.ascontiguousarray(hi, np.float32),
            np.ascontiguousarray(res, np.uint32))


def inv_cell(lo, hi, res) -> np.ndarray:
    lo, hi, res = _grid_args(lo, hi, res)
    out = np.zeros(3, np.float32)
    lib().oracle_inv_cell(_p(lo), _p(hi), _p(res), _p(out))
    return out


def count_cells(verts, tris, lo, hi, res):
    """CountCells: per-triangle cell box (lo corner, extent m) and cell count."""
    verts = np.ascontiguousarray(verts, np.float32)
    tris = np.ascontiguousarray(tris, np.uint32)
    lo, hi, res = _grid_args(lo, hi, res)
    t = tris.shape[0]
    box_lo = np.zeros((t, 3), np.uint32)
    box_m = np.zeros((t, 3), np.uint32)
    count = np.zeros(t, np.uint32)
    st = lib().oracle_count_cells(_p(verts), verts.shape[1], _p(tris), t, _p(lo), _p(hi), _p(res),
                                  _p(box_lo), _p(box_m), _p(count))
    if st != 0:
        raise OracleError(st)
    return box_lo, box_m, count


def exclusive_sum(count: np.ndarray):
    count = np.ascontiguousarray(count, np.uint32)
    start = np.zeros(count.shape[0], np.uint64)
    no = lib().oracle_exclusive_sum(_p(count), count.shape[0], _p(start))
    return start, int(no)


def global_coords(box_lo, m, rid: int) -> np.ndarray:
    box_lo = np.ascontiguousarray(box_lo, np.uint32)
    m = np.ascontiguousarray(m, np.uint32)
    out = np.zeros(3, np.uint32)
    lib().oracle_global_coords(_p(box_lo), _p(m), int(rid), _p(out))
    return out


def make_pairs(box_lo, box_m, count, res, npairs: int):
    box_lo = np.ascontiguousarray(box_lo, np.uint32)
    box_m = np.ascontiguousarray(box_m, np.uint32)
    count = np.ascontiguousarray(count, np.uint32)
    res = np.ascontiguousarray(res, np.uint32)
    cells = np.zeros(npairs, np.uint32)
    objs = np.zeros(npairs, np.uint32)
    lib().oracle_make_pairs(count.shape[0], _p(box_lo), _p(box_m), _p(count), _p(res), _p(cells), _p(objs))
    return cells, objs


def sort_pairs(cells, objs):
    cells = np.array(cells, np.uint32, copy=True)
    objs = np.array(objs, np.uint32, copy=True)
    lib().oracle_sort_pairs(cells.shape[0], _p(cells), _p(objs))
    return cells, objs


def ranges(sorted_cells, ncells: int) -> np.ndarray:
    sorted_cells = np.ascontiguousarray(sorted_cells, np.uint32)
    out = np.zeros(2 * ncells, np.uint32)
    lib().oracle_ranges(sorted_cells.shape[0], _p(sorted_cells), ncells, _p(out))
    return out


@dataclasses.dataclass
class OracleGrid:
    box_lo: np.ndarray        # [T, 3]
    box_m: np.ndarray         # [T, 3]
    count: np.ndarray         # [T]
    start: np.ndarray         # [T] uint64
    npairs: int
    cells_objorder: Optional[np.ndarray]
    objs_objorder: Optional[np.ndarray]
    cells: np.ndarray         # [NO] sorted
    objs: np.ndarray          # [NO]
    ranges: np.ndarray        # [2R]


def build_stages(verts, tris, lo, hi, res, keep_objorder: bool = True) -> OracleGrid:
    """Run every step of Algorithm 1 and keep each stage's arrays."""
    box_lo, box_m, count = count_cells(verts, tris, lo, hi, res)
    start, no = exclusive_sum(count)
    if no > 0xFFFFFFFF:
        raise OracleError(-3)
    c0, o0 = make_pairs(box_lo, box_m, count, res, no)
    cells, objs = sort_pairs(c0, o0)
    ncells = int(np.prod(np.asarray(res, np.int64)))
    rg = ranges(cells, ncells)
    if not keep_objorder:
        c0 = o0 = None
    return OracleGrid(box_lo, box_m, count, start, no, c0, o0, cells, objs, rg)


def probe_npairs(verts, tris, lo, hi, res) -> int:
    """NO of the grid, without building it."""
    verts = np.ascontiguousarray(verts, np.float32)
    tris = np.ascontiguousarray(tris, np.uint32)
    lo, hi, res = _grid_args(lo, hi, res)
    npairs = np.zeros(1, np.uint64)
    st = lib().oracle_build(_p(verts), verts.shape[1], _p(tris), tris.shape[0], _p(lo), _p(hi), _p(res),
                            None, None, None, 0, _p(npairs))
    if st != 0:
        raise OracleError(st)
    return int(npairs[0])


def build(verts, tris, lo, hi, res, npairs=None):
    """Whole build in one C call: (cells, objs, ranges) sorted by cell.

    ``npairs`` (from probe_npairs) sizes the outputs; it is probed if absent."""
    verts = np.ascontiguousarray(verts, np.float32)
    tris = np.ascontiguousarray(tris, np.uint32)
    lo, hi, res = _grid_args(lo, hi, res)
    if npairs is None:
        npairs = probe_npairs(verts, tris, lo, hi, res)
    no = int(npairs)
    ncells = int(np.prod(res.astype(np.int64)))
    cells = np.zeros(max(no, 1), np.uint32)
    objs = np.zeros(max(no, 1), np.uint32)
    rg = np.zeros(2 * ncells, np.uint32)
    got = np.zeros(1, np.uint64)
    st = lib().oracle_build(_p(verts), verts.shape[1], _p(tris), tris.shape[0], _p(lo), _p(hi), _p(res),
                            _p(cells), _p(objs), _p(rg), no, _p(got))
    if st != 0:
        raise OracleError(st)
    return cells[:no], objs[:no], rg


def build_scene(scene, stages: bool = False):
    if stages:
        return build_stages(scene.verts, scene.tris, scene.lo, scene.hi, scene.res)
    return build(scene.verts, scene.tris, scene.lo, scene.hi, scene.res)


# --- removal of false intersections (Test Results, Hairball; Conclusions) ----------------

def grid_coords(verts, tri, lo, hi, res):
    """Grid coordinates u[j][axis] of one triangle's vertices (the FP32 values the
    cell map floors) and whether the overlap test applies to it."""
    verts = np.ascontiguousarray(verts, np.float32)
    tri = np.ascontiguousarray(tri, np.uint32)
    lo, hi, res = _grid_args(lo, hi, res)
    inv = inv_cell(lo, hi, res)
    u = np.zeros((3, 3), np.float32)
    inside = lib().oracle_grid_coords(_p(verts), verts.shape[1], _p(tri), _p(lo), _p(inv), _p(res), _p(u))
    return u, bool(inside)


def touches(u, cell_xyz) -> bool:
    """The FP32 overlap test of a triangle (grid coordinates u [3, 3]) with a cell."""
    u = np.ascontiguousarray(u, np.float32)
    x, y, z = (int(v) for v in cell_xyz)
    return bool(lib().oracle_touches(_p(u), x, y, z))


def make_pairs_culled(verts, tris, lo, hi, res, box_lo, box_m, count):
    """Object-order pairs with false intersections removed: (cells, objs, kept per triangle)."""
    verts = np.ascontiguousarray(verts, np.float32)
    tris = np.ascontiguousarray(tris, np.uint32)
    lo, hi, res = _grid_args(lo, hi, res)
    box_lo = np.ascontiguousarray(box_lo, np.uint32)
    box_m = np.ascontiguousarray(box_m, np.uint32)
    count = np.ascontiguousarray(count, np.uint32)
    nbox = int(count.astype(np.uint64).sum())
    cells = np.zeros(max(nbox, 1), np.uint32)
    objs = np.zeros(max(nbox, 1), np.uint32)
    kept = np.zeros(tris.shape[0], np.uint32)
    n = lib().oracle_make_pairs_culled(_p(verts), verts.shape[1], _p(tris), tris.shape[0], _p(lo), _p(hi), _p(res),
                                       _p(box_lo), _p(box_m), _p(count), _p(cells), _p(objs), _p(kept))
    return cells[:n], objs[:n], kept


def build_culled(verts, tris, lo, hi, res):
    """Whole build with false intersections removed: (cells, objs, ranges, box pair count)."""
    verts = np.ascontiguousarray(verts, np.float32)
    tris = np.ascontiguousarray(tris, np.uint32)
    lo, hi, res = _grid_args(lo, hi, res)
    no = np.zeros(1, np.uint64)
    nbox = np.zeros(1, np.uint64)
    st = lib().oracle_build_culled(_p(verts), verts.shape[1], _p(tris), tris.shape[0], _p(lo), _p(hi), _p(res),
                                   None, None, None, 0, _p(no), _p(nbox))
    if st != 0:
        raise OracleError(st)
    n = int(no[0])
    ncells = int(np.prod(res.astype(np.int64)))
    cells = np.zeros(max(n, 1), np.uint32)
    objs = np.zeros(max(n, 1), np.uint32)
    rg = np.zeros(2 * ncells, np.uint32)
    st = lib().oracle_build_culled(_p(verts), verts.shape[1], _p(tris), tris.shape[0], _p(lo), _p(hi), _p(res),
                                   _p(cells), _p(objs), _p(rg), n, _p(no), _p(nbox))
    if st != 0:
        raise OracleError(st)
    return cells[:n], objs[:n], rg, int(nbox[0])


def build_scene_culled(scene):
    return build_culled(scene.verts, scene.tris, scene.lo, scene.hi, scene.res)


def raycast(verts, tris, lo, hi, rays, tmax: float = float("inf")):
    """Closest hits by brute force over every triangle (rays: float32 [6, N],
    origins then directions): (hit t float32 [N], hit object uint32 [N])."""
    verts = np.ascontiguousarray(verts, np.float32)
    tris = np.ascontiguousarray(tris, np.uint32)
    lo = np.ascontiguousarray(lo, np.float32)
    hi = np.ascontiguousarray(hi, np.float32)
    rays = np.ascontiguousarray(rays, np.float32)
    n = rays.shape[1]
    ht = np.zeros(n, np.float32)
    ho = np.zeros(n, np.uint32)
    lib().oracle_raycast(_p(verts), verts.shape[1], _p(tris), tris.shape[0], _p(lo), _p(hi), _p(rays), n,
                         C.c_float(tmax), _p(ht), _p(ho))
    return ht, ho
