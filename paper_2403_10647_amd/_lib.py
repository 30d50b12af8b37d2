"""ctypes binding of libgridbuild.so (the C ABI declared in include/gridbuild.h).

Argument marshalling only: PyTorch provides device memory and the stream, and
every step of the build runs in the library's HIP kernels.  There is no other
code path: if the library is missing this module raises.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import threading
from typing import List, Optional, Sequence

import numpy as np
import torch  # must be imported before the library so both share one HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgridbuild.so")

GRID_OK = 0
GRID_E_INVAL = -1
GRID_E_NOMEM = -2
GRID_E_OVERFLOW = -3
GRID_E_CAPACITY = -4
GRID_E_BADINDEX = -5
GRID_E_HIP = -6
GRID_E_INTERNAL = -7

SCAN_EXCLUSIVE_SUM = 0
SCAN_INCLUSIVE_MAX = 1
SCAN_SEGMENTED_EXCLUSIVE_SUM = 2

EXPORTS = (
    "grid_strerror", "grid_workspace_size", "grid_count", "grid_build", "grid_build_static", "grid_build_culled", "grid_expand",
    "grid_workspace_size_culled",
    "grid_workspace_size_batched", "grid_count_batched", "grid_build_batched",
    "grid_sort_workspace_size", "grid_sort_pairs", "grid_scan_workspace_size", "grid_scan_u32",
    "grid_trace_enable", "grid_trace_read", "grid_tune_set", "grid_tune_get", "grid_sort_plan",
    "grid_batch_staging_size", "grid_build_batched_async", "grid_workspace_status", "grid_trace_only",
    "grid_raycast", "grid_count_batched_async", "grid_build_batched_counted",
)

STATIC_SCRATCH_BYTES = 64 << 20   # GRID_STATIC_SCRATCH_BYTES: the static workspace of grid_build_static


class GridError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = lib().grid_strerror(status).decode() if _lib is not None else str(status)
        super().__init__(f"{what}: {msg} (status {status})" if what else f"{msg} (status {status})")


class grid_out(C.Structure):
    _fields_ = [("cells", C.c_void_p), ("objs", C.c_void_p), ("ranges", C.c_void_p),
                ("cap_pairs", C.c_uint64), ("npairs", C.c_uint64)]


class grid_trace_entry(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_uint32), ("total_ms", C.c_double)]


class grid_desc(C.Structure):
    _fields_ = [("verts_soa", C.c_void_p), ("tris", C.c_void_p), ("nverts", C.c_uint32), ("ntris", C.c_uint32),
                ("lo", C.c_float * 3), ("hi", C.c_float * 3), ("res", C.c_uint32 * 3), ("out", grid_out)]


_lib = None
_lock = threading.Lock()


def lib():
    """Load libgridbuild.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2403_10647_amd.build`")
        L = C.CDLL(LIB_PATH)
        P, U32, U64, SZ = C.c_void_p, C.c_uint32, C.c_uint64, C.c_size_t
        F3, U3 = C.POINTER(C.c_float), C.POINTER(C.c_uint32)
        L.grid_strerror.argtypes = [C.c_int]
        L.grid_strerror.restype = C.c_char_p
        L.grid_workspace_size.argtypes = [U32, U64, U3]
        L.grid_workspace_size.restype = SZ
        L.grid_workspace_size_culled.argtypes = [U32, U64, U3]
        L.grid_workspace_size_culled.restype = SZ
        L.grid_count.argtypes = [P, U32, P, U32, F3, F3, U3, P, SZ, P, C.POINTER(C.c_uint64), P]
        L.grid_build.argtypes = [P, U32, P, U32, F3, F3, U3, P, SZ, C.POINTER(grid_out), P]
        L.grid_build_static.argtypes = [P, U32, P, U32, F3, F3, U3, C.POINTER(grid_out), P]
        L.grid_build_culled.argtypes = [P, U32, P, U32, F3, F3, U3, P, SZ, U64, C.POINTER(grid_out),
                                        C.POINTER(C.c_uint64), P]
        L.grid_expand.argtypes = [P, U32, P, U32, F3, F3, U3, P, SZ, P, P, U64, C.POINTER(C.c_uint64), P]
        L.grid_workspace_size_batched.argtypes = [C.POINTER(grid_desc), U32]
        L.grid_workspace_size_batched.restype = SZ
        L.grid_count_batched.argtypes = [C.POINTER(grid_desc), U32, P, SZ, P]
        L.grid_build_batched.argtypes = [C.POINTER(grid_desc), U32, P, SZ, P]
        L.grid_sort_workspace_size.argtypes = [U64, U32]
        L.grid_sort_workspace_size.restype = SZ
        L.grid_sort_pairs.argtypes = [P, P, P, P, U64, U32, P, SZ, P]
        L.grid_scan_workspace_size.argtypes = [U64]
        L.grid_scan_workspace_size.restype = SZ
        L.grid_scan_u32.argtypes = [P, P, P, U64, C.c_int, P, SZ, C.POINTER(C.c_uint64), P]
        L.grid_batch_staging_size.argtypes = [U32]
        L.grid_batch_staging_size.restype = SZ
        L.grid_build_batched_async.argtypes = [C.POINTER(grid_desc), U32, P, SZ, P, SZ, P]
        L.grid_build_batched_async.restype = C.c_int
        L.grid_count_batched_async.argtypes = [C.POINTER(grid_desc), U32, P, SZ, P, SZ, P, C.POINTER(C.c_uint64), P]
        L.grid_count_batched_async.restype = C.c_int
        L.grid_build_batched_counted.argtypes = [C.POINTER(grid_desc), U32, P, SZ, P, SZ, P]
        L.grid_build_batched_counted.restype = C.c_int
        L.grid_workspace_status.argtypes = [P, C.POINTER(C.c_uint64), P]
        L.grid_workspace_status.restype = C.c_int
        L.grid_tune_set.argtypes = [C.c_char_p, C.c_int]
        L.grid_tune_get.argtypes = [C.c_char_p, C.POINTER(C.c_int)]
        L.grid_tune_set.restype = C.c_int
        L.grid_sort_plan.argtypes = [U32, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.grid_sort_plan.restype = C.c_int
        L.grid_tune_get.restype = C.c_int
        L.grid_raycast.argtypes = [P, U32, P, U32, F3, F3, U3, P, P, P, U32, C.c_float, P, P, P]
        L.grid_raycast.restype = C.c_int
        L.grid_trace_enable.argtypes = [C.c_int]
        L.grid_trace_only.argtypes = [C.c_char_p]
        L.grid_trace_only.restype = C.c_int
        L.grid_trace_read.argtypes = [C.POINTER(grid_trace_entry), C.c_int, C.POINTER(C.c_int)]
        for name in ("grid_trace_enable", "grid_trace_read", "grid_count", "grid_build", "grid_build_static", "grid_build_culled", "grid_expand", "grid_count_batched", "grid_build_batched",
                     "grid_sort_pairs", "grid_scan_u32"):
            getattr(L, name).restype = C.c_int
        _lib = L
        return _lib


def _check(st: int, what: str):
    if st != GRID_OK:
        raise GridError(st, what)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _f3(x):
    return (C.c_float * 3)(*[float(v) for v in x])


def _u3(x):
    return (C.c_uint32 * 3)(*[int(v) for v in x])


class Workspace:
    """A growable device byte buffer (a torch tensor) handed to the library."""

    def __init__(self, device="cuda"):
        self.device = torch.device(device)
        self.buf: Optional[torch.Tensor] = None

    def get(self, nbytes: int) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = None
            self.buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)
        return self.buf

    def ptr_size(self, nbytes: int):
        b = self.get(nbytes)
        return C.c_void_p(b.data_ptr()), C.c_size_t(b.numel())


_default_ws = {}


def default_workspace(device=None) -> Workspace:
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    key = (dev.type, dev.index)
    if key not in _default_ws:
        _default_ws[key] = Workspace(dev)
    return _default_ws[key]


@dataclasses.dataclass
class GridInput:
    """Device-resident grid request: verts FP32 [3, V], tris int32 [T, 3]."""
    verts: torch.Tensor
    tris: torch.Tensor
    lo: Sequence[float]
    hi: Sequence[float]
    res: Sequence[int]

    @property
    def ntris(self) -> int:
        return int(self.tris.shape[0])

    @property
    def nverts(self) -> int:
        return int(self.verts.shape[1])

    @property
    def ncells(self) -> int:
        return int(np.prod(np.asarray(self.res, np.int64)))

    @staticmethod
    def from_scene(scene, device="cuda") -> "GridInput":
        v = torch.from_numpy(np.ascontiguousarray(scene.verts, np.float32)).to(device)
        t = torch.from_numpy(np.ascontiguousarray(scene.tris).view(np.int32)).to(device)
        return GridInput(v, t, list(map(float, scene.lo)), list(map(float, scene.hi)), list(map(int, scene.res)))


@dataclasses.dataclass
class GridResult:
    cells: torch.Tensor      # int32 view of uint32 [npairs]
    objs: torch.Tensor       # int32 view of uint32 [npairs]
    ranges: torch.Tensor     # int32 view of uint32 [2R]
    npairs: int

    def numpy(self):
        c = self.cells[: self.npairs].cpu().numpy().view(np.uint32)
        o = self.objs[: self.npairs].cpu().numpy().view(np.uint32)
        r = self.ranges.cpu().numpy().view(np.uint32)
        return c, o, r


def _input_args(g: GridInput):
    """The C arguments of a grid (checked once, then kept while the tensors stay the same)."""
    key = (g.verts.data_ptr(), g.tris.data_ptr(), g.verts.shape, g.tris.shape, tuple(g.lo), tuple(g.hi), tuple(g.res))
    cached = getattr(g, "_c_args", None)
    if cached is not None and cached[0] == key:
        return cached[1]
    assert g.verts.dtype == torch.float32 and g.verts.is_contiguous() and g.verts.dim() == 2 and g.verts.shape[0] == 3
    assert g.tris.dtype == torch.int32 and g.tris.is_contiguous() and (g.tris.numel() == 0 or g.tris.shape[1] == 3)
    args = (C.c_void_p(g.verts.data_ptr()), C.c_uint32(g.nverts), C.c_void_p(g.tris.data_ptr()),
            C.c_uint32(g.ntris), _f3(g.lo), _f3(g.hi), _u3(g.res))
    object.__setattr__(g, "_c_args", (key, args))
    return args


_ws_sizes: dict = {}


def workspace_size(ntris: int, cap_pairs: int, res) -> int:
    # the radix digit width sets the look-back words the workspace holds
    key = (int(ntris), int(cap_pairs), tuple(int(r) for r in res), tune_get("max_digit_bits"))
    n = _ws_sizes.get(key)
    if n is None:
        n = _ws_sizes[key] = int(lib().grid_workspace_size(ntris, cap_pairs, _u3(res)))
    return n


def workspace_size_culled(ntris: int, box_cap: int, res) -> int:
    """Workspace of grid_build_culled: the plain build's plus each triangle's test record."""
    return int(lib().grid_workspace_size_culled(ntris, box_cap, _u3(res)))


def count(g: GridInput, ws: Optional[Workspace] = None, with_start: bool = False, stream=None):
    """CountCells + ExclusiveSum: (NO, start[T] or None)."""
    L = lib()
    ws = ws or default_workspace(g.verts.device)
    wp, wn = ws.ptr_size(workspace_size(g.ntris, 0, g.res))
    start = torch.empty(max(g.ntris, 1), dtype=torch.int32, device=g.verts.device) if with_start else None
    no = C.c_uint64(0)
    st = L.grid_count(*_input_args(g), wp, wn, C.c_void_p(start.data_ptr()) if start is not None else None,
                      C.byref(no), _stream(stream))
    _check(st, "grid_count")
    return int(no.value), (start[: g.ntris] if start is not None else None)


def build(g: GridInput, cap_pairs: Optional[int] = None, ws: Optional[Workspace] = None, out: Optional[GridResult] = None,
          stream=None) -> GridResult:
    """The whole build.  With no capacity given, counts first to size the outputs."""
    L = lib()
    ws = ws or default_workspace(g.verts.device)
    if out is None:
        if cap_pairs is None:
            cap_pairs, _ = count(g, ws, stream=stream)
        dev = g.verts.device
        out = GridResult(torch.empty(max(cap_pairs, 1), dtype=torch.int32, device=dev),
                         torch.empty(max(cap_pairs, 1), dtype=torch.int32, device=dev),
                         torch.empty(2 * g.ncells, dtype=torch.int32, device=dev), 0)
    cap = int(out.cells.numel()) if cap_pairs is None else int(cap_pairs)
    wp, wn = ws.ptr_size(workspace_size(g.ntris, cap, g.res))
    o = grid_out(out.cells.data_ptr(), out.objs.data_ptr(), out.ranges.data_ptr(), cap, 0)
    st = L.grid_build(*_input_args(g), wp, wn, C.byref(o), _stream(stream))
    out.npairs = int(o.npairs)
    _check(st, "grid_build")
    return out


def build_static(g: GridInput, out: GridResult, stream=None) -> GridResult:
    """The whole build in the library's static device scratch (grid_build_static):
    no workspace argument and no allocation.  out's buffers set the capacity."""
    cap = int(out.cells.numel())
    o = grid_out(out.cells.data_ptr(), out.objs.data_ptr(), out.ranges.data_ptr(), cap, 0)
    st = lib().grid_build_static(*_input_args(g), C.byref(o), _stream(stream))
    out.npairs = int(o.npairs)
    _check(st, "grid_build_static")
    return out


def build_culled(g: GridInput, box_cap: Optional[int] = None, out: Optional[GridResult] = None,
                 ws: Optional[Workspace] = None, stream=None):
    """The build with false intersections removed: (GridResult of the kept pairs, box pair count).
    With no box capacity given, counts first; with no outputs, sizes them for the box pairs."""
    L = lib()
    ws = ws or default_workspace(g.verts.device)
    if box_cap is None:
        box_cap, _ = count(g, ws, stream=stream)
    if out is None:
        dev = g.verts.device
        out = GridResult(torch.empty(max(box_cap, 1), dtype=torch.int32, device=dev),
                         torch.empty(max(box_cap, 1), dtype=torch.int32, device=dev),
                         torch.empty(2 * g.ncells, dtype=torch.int32, device=dev), 0)
    wp, wn = ws.ptr_size(workspace_size_culled(g.ntris, box_cap, g.res))
    o = grid_out(out.cells.data_ptr(), out.objs.data_ptr(), out.ranges.data_ptr(), int(out.cells.numel()), 0)
    nbox = C.c_uint64(0)
    st = L.grid_build_culled(*_input_args(g), wp, wn, C.c_uint64(box_cap), C.byref(o), C.byref(nbox), _stream(stream))
    out.npairs = int(o.npairs)
    _check(st, "grid_build_culled")
    return out, int(nbox.value)


class PlainBuild:
    """grid_build of one input into one output, its C arguments marshalled once.

    For repeated builds of the same buffers (frames of a scene, benchmarks):
    each call is one C call.  The input tensors, the outputs and the workspace
    must stay alive and in place while the object is used: a workspace that
    later grows for another build moves, so size it first for all its users."""

    def __init__(self, g: GridInput, out: GridResult, ws: Optional[Workspace] = None, stream=None):
        self.g, self.out = g, out
        self.ws = ws or default_workspace(g.verts.device)
        cap = int(out.cells.numel())
        wp, wn = self.ws.ptr_size(workspace_size(g.ntris, cap, g.res))
        self._o = grid_out(out.cells.data_ptr(), out.objs.data_ptr(), out.ranges.data_ptr(), cap, 0)
        self._fn = lib().grid_build
        self._args = (*_input_args(g), wp, wn, C.byref(self._o), _stream(stream))

    def __call__(self) -> GridResult:
        st = self._fn(*self._args)
        self.out.npairs = int(self._o.npairs)
        if st != GRID_OK:
            raise GridError(st, "grid_build")
        return self.out


class CulledBuild:
    """grid_build_culled of one input into one output, its C arguments marshalled once
    (the same rules as PlainBuild).  Returns (GridResult, box pair count)."""

    def __init__(self, g: GridInput, out: GridResult, box_cap: int, ws: Optional[Workspace] = None, stream=None):
        self.g, self.out = g, out
        self.ws = ws or default_workspace(g.verts.device)
        wp, wn = self.ws.ptr_size(workspace_size_culled(g.ntris, box_cap, g.res))
        self._o = grid_out(out.cells.data_ptr(), out.objs.data_ptr(), out.ranges.data_ptr(), int(out.cells.numel()), 0)
        self._nbox = C.c_uint64(0)
        self._fn = lib().grid_build_culled
        self._args = (*_input_args(g), wp, wn, C.c_uint64(box_cap), C.byref(self._o), C.byref(self._nbox),
                      _stream(stream))

    def __call__(self):
        st = self._fn(*self._args)
        self.out.npairs = int(self._o.npairs)
        if st != GRID_OK:
            raise GridError(st, "grid_build_culled")
        return self.out, int(self._nbox.value)


def expand(g: GridInput, ws: Optional[Workspace] = None, stream=None):
    """Object-order (cells, objs) lists."""
    L = lib()
    ws = ws or default_workspace(g.verts.device)
    no, _ = count(g, ws, stream=stream)
    dev = g.verts.device
    cells = torch.empty(max(no, 1), dtype=torch.int32, device=dev)
    objs = torch.empty(max(no, 1), dtype=torch.int32, device=dev)
    wp, wn = ws.ptr_size(workspace_size(g.ntris, no, g.res))
    n = C.c_uint64(0)
    st = L.grid_expand(*_input_args(g), wp, wn, C.c_void_p(cells.data_ptr()), C.c_void_p(objs.data_ptr()), no,
                       C.byref(n), _stream(stream))
    _check(st, "grid_expand")
    return cells[:no], objs[:no]


def _desc_dtype() -> np.dtype:
    """numpy view of grid_desc (same offsets), to fill descriptor arrays by column."""
    o = grid_desc.out.offset
    names = ["verts_soa", "tris", "nverts", "ntris", "lo", "hi", "res", "cells", "objs", "ranges", "cap_pairs", "npairs"]
    formats = ["<u8", "<u8", "<u4", "<u4", ("<f4", 3), ("<f4", 3), ("<u4", 3), "<u8", "<u8", "<u8", "<u8", "<u8"]
    offsets = [grid_desc.verts_soa.offset, grid_desc.tris.offset, grid_desc.nverts.offset, grid_desc.ntris.offset,
               grid_desc.lo.offset, grid_desc.hi.offset, grid_desc.res.offset, o + grid_out.cells.offset,
               o + grid_out.objs.offset, o + grid_out.ranges.offset, o + grid_out.cap_pairs.offset,
               o + grid_out.npairs.offset]
    return np.dtype({"names": names, "formats": formats, "offsets": offsets, "itemsize": C.sizeof(grid_desc)})


_DESC_DTYPE = _desc_dtype()


def _desc_view(arr) -> np.ndarray:
    return np.frombuffer((C.c_char * C.sizeof(arr)).from_buffer(arr), dtype=_DESC_DTYPE)


_FEW = 16   # descriptor arrays up to this length are filled element by element


def _desc_bytes(g: GridInput) -> bytes:
    """A grid's descriptor without outputs, kept while its tensors and bounds stay the same."""
    key = (g.verts.data_ptr(), g.tris.data_ptr(), g.verts.shape, g.tris.shape, tuple(g.lo), tuple(g.hi), tuple(g.res))
    cached = getattr(g, "_c_desc", None)
    if cached is not None and cached[0] == key:
        return cached[1]
    d = grid_desc()
    d.verts_soa = g.verts.data_ptr()
    d.tris = g.tris.data_ptr()
    d.nverts = g.nverts
    d.ntris = g.ntris
    d.lo[:] = [float(x) for x in g.lo]
    d.hi[:] = [float(x) for x in g.hi]
    d.res[:] = [int(x) for x in g.res]
    b = bytes(d)
    object.__setattr__(g, "_c_desc", (key, b))
    return b


def _set_outputs(arr, cells: List[int], objs: List[int], ranges: List[int], caps: List[int]):
    """Write output addresses and pair capacities into a descriptor array."""
    if len(arr) <= _FEW:
        for d, c, o, r, k in zip(arr, cells, objs, ranges, caps):
            out = d.out
            out.cells = c
            out.objs = o
            out.ranges = r
            out.cap_pairs = k
        return
    a = _desc_view(arr)
    a["cells"] = cells
    a["objs"] = objs
    a["ranges"] = ranges
    a["cap_pairs"] = caps


def _descs(inputs: List[GridInput], outs: Optional[List[GridResult]] = None):
    """ctypes array of grid_desc for the inputs (and outputs): short arrays from each grid's kept
    descriptor, long ones column by column."""
    n = len(inputs)
    if 0 < n <= _FEW:
        arr = (grid_desc * n).from_buffer_copy(b"".join(_desc_bytes(g) for g in inputs))
        if outs is not None:
            _set_outputs(arr, [o.cells.data_ptr() for o in outs], [o.objs.data_ptr() for o in outs],
                         [o.ranges.data_ptr() for o in outs], [o.cells.numel() for o in outs])
        return arr
    arr = (grid_desc * n)()
    if n == 0:
        return arr
    a = _desc_view(arr)
    a["verts_soa"] = [g.verts.data_ptr() for g in inputs]
    a["tris"] = [g.tris.data_ptr() for g in inputs]
    a["nverts"] = [g.nverts for g in inputs]
    a["ntris"] = [g.ntris for g in inputs]
    a["lo"] = np.asarray([g.lo for g in inputs], np.float32)
    a["hi"] = np.asarray([g.hi for g in inputs], np.float32)
    a["res"] = np.asarray([g.res for g in inputs], np.uint32)
    if outs is not None:
        a["cells"] = [o.cells.data_ptr() for o in outs]
        a["objs"] = [o.objs.data_ptr() for o in outs]
        a["ranges"] = [o.ranges.data_ptr() for o in outs]
        a["cap_pairs"] = [o.cells.numel() for o in outs]
    return arr


def count_batched(inputs: List[GridInput], ws: Optional[Workspace] = None, stream=None) -> List[int]:
    L = lib()
    ws = ws or default_workspace(inputs[0].verts.device)
    arr = _descs(inputs)
    wp, wn = ws.ptr_size(L.grid_workspace_size_batched(arr, len(inputs)))
    st = L.grid_count_batched(arr, len(inputs), wp, wn, _stream(stream))
    _check(st, "grid_count_batched")
    return _desc_view(arr)["npairs"].tolist()


def alloc_results(inputs: List[GridInput], caps: List[int]) -> List[GridResult]:
    dev = inputs[0].verts.device
    return [GridResult(torch.empty(max(c, 1), dtype=torch.int32, device=dev),
                       torch.empty(max(c, 1), dtype=torch.int32, device=dev),
                       torch.empty(2 * g.ncells, dtype=torch.int32, device=dev), 0)
            for g, c in zip(inputs, caps)]


def build_batched(inputs: List[GridInput], outs: Optional[List[GridResult]] = None, ws: Optional[Workspace] = None,
                  stream=None) -> List[GridResult]:
    L = lib()
    ws = ws or default_workspace(inputs[0].verts.device)
    if outs is None:
        outs = alloc_results(inputs, count_batched(inputs, ws, stream))
    arr = _descs(inputs, outs)
    wp, wn = ws.ptr_size(L.grid_workspace_size_batched(arr, len(inputs)))
    st = L.grid_build_batched(arr, len(inputs), wp, wn, _stream(stream))
    for o, n in zip(outs, _desc_view(arr)["npairs"].tolist()):
        o.npairs = n
    _check(st, "grid_build_batched")
    return outs


class BatchedBuild:
    """grid_build_batched of fixed inputs into fixed outputs, descriptors marshalled once.

    For repeated batched builds of the same buffers; each call is one C call.
    The tensors and the workspace must stay alive and in place while it is used
    (a workspace that later grows for another build moves)."""

    def __init__(self, inputs: List[GridInput], outs: List[GridResult], ws: Optional[Workspace] = None, stream=None):
        self.inputs, self.outs = inputs, outs
        self.ws = ws or default_workspace(inputs[0].verts.device)
        self._arr = _descs(inputs, outs)
        self._view = _desc_view(self._arr)
        wp, wn = self.ws.ptr_size(lib().grid_workspace_size_batched(self._arr, len(inputs)))
        self._fn = lib().grid_build_batched
        self._args = (self._arr, len(inputs), wp, wn, _stream(stream))

    def __call__(self) -> List[GridResult]:
        st = self._fn(*self._args)
        for o, n in zip(self.outs, self._view["npairs"].tolist()):
            o.npairs = n
        _check(st, "grid_build_batched")
        return self.outs


def sort_pairs(keys: torch.Tensor, vals: torch.Tensor, nbits: int, ws: Optional[Workspace] = None, stream=None):
    """Stable radix sort of int32-viewed uint32 (keys, vals) in place by the low nbits bits."""
    L = lib()
    n = keys.numel()
    ws = ws or default_workspace(keys.device)
    ka = torch.empty_like(keys)
    va = torch.empty_like(vals)
    wp, wn = ws.ptr_size(L.grid_sort_workspace_size(n, nbits))
    st = L.grid_sort_pairs(C.c_void_p(keys.data_ptr()), C.c_void_p(vals.data_ptr()), C.c_void_p(ka.data_ptr()),
                           C.c_void_p(va.data_ptr()), n, nbits, wp, wn, _stream(stream))
    _check(st, "grid_sort_pairs")
    return keys, vals


def scan_u32(x: torch.Tensor, op: int, flags: Optional[torch.Tensor] = None, ws: Optional[Workspace] = None,
             stream=None):
    L = lib()
    n = x.numel()
    ws = ws or default_workspace(x.device)
    out = torch.empty_like(x)
    tot = C.c_uint64(0)
    wp, wn = ws.ptr_size(L.grid_scan_workspace_size(n))
    st = L.grid_scan_u32(C.c_void_p(x.data_ptr()), C.c_void_p(flags.data_ptr()) if flags is not None else None,
                         C.c_void_p(out.data_ptr()), n, op, wp, wn, C.byref(tot), _stream(stream))
    _check(st, "grid_scan_u32")
    return out, int(tot.value)


def raycast(g: GridInput, grid: GridResult, rays: torch.Tensor, tmax: float = float("inf"), stream=None):
    """Closest hits of rays (float32 [6, N] on the device: origins, then directions)
    over a built grid of g: (hit t float32 [N], hit object int32 [N], 0xFFFFFFFF if none)."""
    assert rays.dtype == torch.float32 and rays.is_contiguous() and rays.dim() == 2 and rays.shape[0] == 6
    n = int(rays.shape[1])
    ht = torch.empty(max(n, 1), dtype=torch.float32, device=rays.device)
    ho = torch.empty(max(n, 1), dtype=torch.int32, device=rays.device)
    st = lib().grid_raycast(*_input_args(g), C.c_void_p(grid.ranges.data_ptr()), C.c_void_p(grid.objs.data_ptr()),
                            C.c_void_p(rays.data_ptr()), n, C.c_float(tmax), C.c_void_p(ht.data_ptr()),
                            C.c_void_p(ho.data_ptr()), _stream(stream))
    _check(st, "grid_raycast")
    return ht[:n], ho[:n]


def trace_enable(on: bool = True):
    _check(lib().grid_trace_enable(1 if on else 0), "grid_trace_enable")


def trace_only(name: Optional[str]):
    """Trace only the launches of kernel ``name`` (None: every kernel)."""
    _check(lib().grid_trace_only(name.encode() if name is not None else None), "grid_trace_only")


def trace_read() -> dict:
    """{kernel: (launches, total_ms)} since the last read (waits for the launches)."""
    arr = (grid_trace_entry * 64)()
    n = C.c_int(0)
    _check(lib().grid_trace_read(arr, 64, C.byref(n)), "grid_trace_read")
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(min(n.value, 64))}


def tune_set(key: str, value: int):
    _check(lib().grid_tune_set(key.encode(), int(value)), f"grid_tune_set({key})")


def tune_get(key: str) -> int:
    v = C.c_int(0)
    _check(lib().grid_tune_get(key.encode(), C.byref(v)), f"grid_tune_get({key})")
    return int(v.value)


def sort_plan(nbits: int):
    """(passes, [digit widths], kernel digit bits) for an nbits-bit key under the current knobs."""
    p, k = C.c_uint32(0), C.c_uint32(0)
    w = (C.c_uint32 * 4)()
    _check(lib().grid_sort_plan(nbits, C.byref(p), w, C.byref(k)), "grid_sort_plan")
    return int(p.value), [int(w[i]) for i in range(p.value)], int(k.value)


def build_batched_async(inputs: List[GridInput], outs: List[GridResult], npairs: List[int], ws: Workspace,
                        staging: torch.Tensor, stream=None):
    """Launch a batched build without waiting.

    ``npairs`` are the grids' pair counts from count_batched; each output must hold at least that
    many pairs.  ``staging`` is a pinned host uint8 tensor of at least grid_batch_staging_size(n)
    bytes that must stay untouched until the stream passes this call.  Errors found on the device
    are read later with workspace_status(ws)."""
    L = lib()
    arr = _descs(inputs, outs)
    n = len(inputs)
    need = int(L.grid_batch_staging_size(n))
    assert staging.is_pinned() and staging.numel() >= need
    wp, wn = ws.ptr_size(L.grid_workspace_size_batched(arr, n))
    st = L.grid_build_batched_async(arr, n, wp, wn, C.c_void_p(staging.data_ptr()), C.c_size_t(staging.numel()),
                                    _stream(stream))
    _check(st, "grid_build_batched_async")
    for o, c in zip(outs, npairs):
        o.npairs = int(c)


# bits of the status word grid_count_batched_async leaves after the per-grid counts
COUNT_BAD_INDEX = 1
COUNT_INTERNAL = 2
COUNT_OVER_WORKSPACE = 4
COUNT_OVER_32BIT = 8


def count_batched_async(inputs: List[GridInput], ws: Workspace, ws_bytes: int, staging: torch.Tensor,
                        counts: torch.Tensor, stream=None, descs=None) -> int:
    """Enqueue the count of a batch into ``ws`` (the first half of a batched build split around its
    count) and return the pair capacity of the workspace's layout for this batch.

    ``counts`` is a pinned int64 tensor of at least len(inputs) + 1 entries: once the stream has
    passed this call it holds each grid's NO and then the status word (COUNT_* bits).  ``staging``
    is a pinned uint8 tensor of at least 2 * grid_batch_staging_size(n) bytes, kept for
    build_batched_counted.  ``descs``: the inputs' descriptor array when the caller already holds it."""
    L = lib()
    n = len(inputs)
    assert staging.is_pinned() and staging.numel() >= 2 * int(L.grid_batch_staging_size(n))
    assert counts.is_pinned() and counts.dtype == torch.int64 and counts.numel() >= n + 1
    assert ws.buf is not None and ws.buf.numel() >= ws_bytes
    cap = C.c_uint64(0)
    st = L.grid_count_batched_async(descs if descs is not None else _descs(inputs), n, C.c_void_p(ws.buf.data_ptr()), C.c_size_t(ws_bytes),
                                    C.c_void_p(staging.data_ptr()), C.c_size_t(staging.numel()),
                                    C.c_void_p(counts.data_ptr()), C.byref(cap), _stream(stream))
    _check(st, "grid_count_batched_async")
    return int(cap.value)


def build_batched_counted(inputs: List[GridInput], outs: Optional[List[GridResult]], npairs: List[int], ws: Workspace,
                          ws_bytes: int, staging: torch.Tensor, stream=None, descs=None):
    """Enqueue the rest of a batched build counted by count_batched_async into the same workspace, with
    the same inputs, ``ws_bytes``, staging and stream.  Each output must hold at least its grid's NO
    (``npairs``).  Errors found on the device are read later with workspace_status(ws).  ``descs``: the
    descriptor array with the outputs already written (then ``outs`` may be None)."""
    L = lib()
    n = len(inputs)
    st = L.grid_build_batched_counted(descs if descs is not None else _descs(inputs, outs), n, C.c_void_p(ws.buf.data_ptr()), C.c_size_t(ws_bytes),
                                      C.c_void_p(staging.data_ptr()), C.c_size_t(staging.numel()), _stream(stream))
    _check(st, "grid_build_batched_counted")
    for o, c in zip(outs or [], npairs):
        o.npairs = int(c)


def workspace_status(ws: Workspace, stream=None):
    """(status, total NO) of the last build launched on ws (waits for the stream)."""
    tot = C.c_uint64(0)
    st = lib().grid_workspace_status(C.c_void_p(ws.buf.data_ptr()), C.byref(tot), _stream(stream))
    return int(st), int(tot.value)
