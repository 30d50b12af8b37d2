"""Host-side checks of the C ABI that need no GPU.

The library loads on a machine without a GPU; every function declared in
include/gridbuild.h is exported; and argument validation, workspace sizing and
error strings are host logic that runs before any device call.
"""
import ctypes as C
import os
import re

import pytest

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gridbuild.h")


@pytest.fixture(scope="module")
def G():
    from paper_2403_10647_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2403_10647_amd import build
        build.build()
    _lib.lib()
    return _lib


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(grid_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_function_is_exported(G):
    names = declared_functions()
    assert len(names) >= 14
    L = G.lib()
    for n in names:
        assert hasattr(L, n), f"{n} declared in gridbuild.h but not exported"
    assert set(names) == set(G.EXPORTS)


def test_strerror(G):
    L = G.lib()
    for st in (0, -1, -2, -3, -4, -5, -6, -7):
        assert L.grid_strerror(st) != b"unknown status"
    assert L.grid_strerror(-4) == b"pair capacity too small"
    assert L.grid_strerror(12345) == b"unknown status"


def test_workspace_sizes_grow(G):
    a = G.workspace_size(1000, 4000, [32, 32, 32])
    b = G.workspace_size(1000, 400000, [32, 32, 32])
    c = G.workspace_size(100000, 400000, [32, 32, 32])
    assert 0 < a < b < c
    L = G.lib()
    # culled builds add one 176-byte test record per triangle
    assert G.workspace_size_culled(1000, 4000, [32, 32, 32]) >= a + 176 * 1000 - 256   # one empty region fewer
    assert G.workspace_size_culled(100000, 400000, [32, 32, 32]) >= c + 176 * 100000 - 256
    assert L.grid_workspace_size_culled(10, 10, None) == 0
    assert L.grid_sort_workspace_size(1 << 20, 25) > L.grid_sort_workspace_size(1 << 20, 8) > 0
    assert L.grid_sort_workspace_size(10, 33) == 0
    assert L.grid_scan_workspace_size(1 << 20) > L.grid_scan_workspace_size(10) > 0


def _args(G, lo=(0, 0, 0), hi=(1, 1, 1), res=(4, 4, 4)):
    return (C.c_void_p(16), C.c_uint32(3), C.c_void_p(16), C.c_uint32(1), G._f3(lo), G._f3(hi), G._u3(res))


@pytest.mark.parametrize("lo,hi,res", [
    ((0, 0, 0), (0, 1, 1), (4, 4, 4)),          # lo == hi
    ((0, 2, 0), (1, 1, 1), (4, 4, 4)),          # lo > hi
    ((0, 0, 0), (1, 1, 1), (0, 4, 4)),          # res 0
    ((0, 0, 0), (1, 1, 1), (4, 4, 1025)),       # res above 1024
    ((float("nan"), 0, 0), (1, 1, 1), (4, 4, 4)),
    ((0, 0, 0), (float("inf"), 1, 1), (4, 4, 4)),
])
def test_invalid_grids_rejected_on_host(G, lo, hi, res):
    L = G.lib()
    out = G.grid_out(16, 16, 16, 10, 0)
    st = L.grid_build(*_args(G, lo, hi, res), C.c_void_p(16), 1 << 30, C.byref(out), None)
    assert st == G.GRID_E_INVAL
    no = C.c_uint64(0)
    st = L.grid_count(*_args(G, lo, hi, res), C.c_void_p(16), 1 << 30, None, C.byref(no), None)
    assert st == G.GRID_E_INVAL


def test_null_and_small_workspace_rejected(G):
    L = G.lib()
    out = G.grid_out(16, 16, 16, 10, 0)
    assert L.grid_build(*_args(G), None, 1 << 30, C.byref(out), None) == G.GRID_E_INVAL
    assert L.grid_build(*_args(G), C.c_void_p(16), 64, C.byref(out), None) == G.GRID_E_NOMEM
    bad = G.grid_out(16, 0, 16, 10, 0)         # objs missing
    assert L.grid_build(*_args(G), C.c_void_p(16), 1 << 30, C.byref(bad), None) == G.GRID_E_INVAL
    assert L.grid_build(*_args(G), C.c_void_p(16), 1 << 30, None, None) == G.GRID_E_INVAL
    no = C.c_uint64(0)
    assert L.grid_count(*_args(G), C.c_void_p(16), 1 << 30, None, None, None) == G.GRID_E_INVAL


def test_primitives_validate_on_host(G):
    L = G.lib()
    tot = C.c_uint64(7)
    P = C.c_void_p(16)
    assert L.grid_scan_u32(P, None, P, 10, 3, P, 1 << 20, C.byref(tot), None) == G.GRID_E_INVAL
    assert L.grid_scan_u32(P, None, P, 10, 2, P, 1 << 20, C.byref(tot), None) == G.GRID_E_INVAL  # flags missing
    assert L.grid_scan_u32(P, None, P, 0, 0, P, 1 << 20, C.byref(tot), None) == G.GRID_OK and tot.value == 0
    assert L.grid_scan_u32(P, None, P, 1000, 0, P, 8, C.byref(tot), None) == G.GRID_E_NOMEM
    assert L.grid_sort_pairs(P, P, P, P, 10, 33, P, 1 << 20, None) == G.GRID_E_INVAL
    assert L.grid_sort_pairs(P, P, P, P, 0, 16, P, 1 << 20, None) == G.GRID_OK
    assert L.grid_sort_pairs(P, P, P, P, 10, 0, P, 1 << 20, None) == G.GRID_OK
    assert L.grid_sort_pairs(P, P, P, P, 100000, 16, P, 64, None) == G.GRID_E_NOMEM


def test_batched_validation_on_host(G):
    L = G.lib()
    assert L.grid_build_batched(None, 0, C.c_void_p(16), 1 << 20, None) == G.GRID_E_INVAL
    arr = (G.grid_desc * 2)()
    for d in arr:
        d.verts_soa, d.tris, d.nverts, d.ntris = 16, 16, 3, 1
        d.lo[:] = [0, 0, 0]
        d.hi[:] = [1, 1, 1]
        d.res[:] = [4, 4, 4]
        d.out.cells, d.out.objs, d.out.ranges, d.out.cap_pairs = 16, 16, 16, 4
    arr[1].res[:] = [4, 0, 4]
    assert L.grid_workspace_size_batched(arr, 2) == 0
    assert L.grid_build_batched(arr, 2, C.c_void_p(16), 1 << 20, None) == G.GRID_E_INVAL
    arr[1].res[:] = [4, 4, 4]
    assert L.grid_workspace_size_batched(arr, 2) > 0
    assert L.grid_build_batched(arr, 2, C.c_void_p(16), 64, None) == G.GRID_E_NOMEM


def test_split_batched_build_validates_on_host(G):
    # the count and the resumed build of a batched build split around its count:
    # argument checks, the workspace capacity and the counted-table match all
    # come before anything is enqueued
    L = G.lib()
    arr = (G.grid_desc * 2)()
    for d in arr:
        d.verts_soa, d.tris, d.nverts, d.ntris = 16, 16, 3, 1
        d.lo[:] = [0, 0, 0]
        d.hi[:] = [1, 1, 1]
        d.res[:] = [4, 4, 4]
        d.out.cells, d.out.objs, d.out.ranges, d.out.cap_pairs = 16, 16, 16, 4
    half = L.grid_batch_staging_size(2)
    staging = (C.c_ubyte * (2 * half))()
    counts = (C.c_uint64 * 3)()
    cap = C.c_uint64(123)
    P = C.c_void_p(16)
    count = L.grid_count_batched_async
    assert count(None, 0, P, 1 << 20, staging, 2 * half, counts, C.byref(cap), None) == G.GRID_E_INVAL
    assert count(arr, 2, P, 1 << 20, None, 2 * half, counts, C.byref(cap), None) == G.GRID_E_INVAL
    assert count(arr, 2, P, 1 << 20, staging, 2 * half, None, C.byref(cap), None) == G.GRID_E_INVAL
    assert count(arr, 2, P, 1 << 20, staging, half, counts, C.byref(cap), None) == G.GRID_E_NOMEM  # one table only
    assert count(arr, 2, P, 64, staging, 2 * half, counts, C.byref(cap), None) == G.GRID_E_NOMEM  # not even the count
    assert count(arr, 2, None, 1 << 20, staging, 2 * half, counts, C.byref(cap), None) == G.GRID_E_INVAL
    assert cap.value == 123                        # nothing reported on failure
    arr[1].res[:] = [4, 0, 4]
    assert count(arr, 2, P, 1 << 20, staging, 2 * half, counts, C.byref(cap), None) == G.GRID_E_INVAL
    arr[1].res[:] = [4, 4, 4]
    resume = L.grid_build_batched_counted
    assert resume(arr, 2, P, 1 << 20, staging, half, None) == G.GRID_E_NOMEM
    # the first half of the staging is not the table of these grids (all zero): refused
    assert resume(arr, 2, P, 1 << 20, staging, 2 * half, None) == G.GRID_E_INVAL
    arr[0].out.objs = 0                            # an output missing
    assert resume(arr, 2, P, 1 << 20, staging, 2 * half, None) == G.GRID_E_INVAL


def test_trace_read_without_launches(G):
    G.trace_enable(True)
    assert G.trace_read() == {}
    G.trace_enable(False)


def test_trace_only_validates_names(G):
    G.trace_only("onesweep")
    G.trace_only(None)
    with pytest.raises(G.GridError):
        G.trace_only("")
    with pytest.raises(G.GridError):
        G.trace_only("x" * 48)


@pytest.mark.parametrize("digit", [4, 5, 6, 7, 8, 9, 10, 11])
def test_sort_plan_is_valid_for_every_width(G, digit):
    # regression: a narrow digit limit on a wide key once asked for more than
    # four passes, overflowing the plan and running digits wider than the kernel
    G.tune_set("max_digit_bits", digit)
    try:
        for nbits in range(1, 33):
            passes, widths, kbits = G.sort_plan(nbits)
            assert 1 <= passes <= 4
            assert sum(widths) == nbits
            assert all(1 <= w <= kbits for w in widths) and 8 <= kbits <= 11
            assert passes == min(4, -(-nbits // digit))
            assert max(widths) - min(widths) <= 1          # balanced digits (25 bits: 8, 8, 9)
            assert list(widths) == sorted(widths)          # the wider digits on top
            assert kbits == max(8, max(widths))
        assert G.sort_plan(0)[0] == 0
    finally:
        G.tune_set("max_digit_bits", 9)


def test_tune_rejects_bad_values(G):
    with pytest.raises(G.GridError):
        G.tune_set("max_digit_bits", 3)
    with pytest.raises(G.GridError):
        G.tune_set("max_digit_bits", 12)
    with pytest.raises(G.GridError):
        G.tune_set("no_such_knob", 1)
    with pytest.raises(G.GridError):
        G.tune_set("per_object_pairs", 2)
    with pytest.raises(G.GridError):
        G.tune_set("small_tiles", 2)
    with pytest.raises(G.GridError):
        G.tune_set("wide_lookback", 2)
    assert G.tune_get("max_digit_bits") == 9 and G.tune_get("fused_expand") in (0, 1)
    assert G.tune_get("per_object_pairs") == 0 and G.tune_get("small_tiles") == 1
    assert G.tune_get("wide_lookback") == 0


def test_workspace_size_follows_the_digit_width(G):
    # a 22-bit key (160^3 cells): 11-bit digits need more look-back words than
    # 8-bit ones, and the binding must not serve a size computed under another width
    from paper_2403_10647_amd import tune
    res = [160, 160, 160]
    old = G.tune_get("max_digit_bits")
    try:
        G.tune_set("max_digit_bits", 8)
        a = G.workspace_size(1_000_000, 33_000_000, res)
        G.tune_set("max_digit_bits", 11)
        b = G.workspace_size(1_000_000, 33_000_000, res)
    finally:
        G.tune_set("max_digit_bits", old)
    assert b > a

    class _G:   # the tuner's sizing over its candidates, on the host only
        tune_get = staticmethod(G.tune_get)
        tune_set = staticmethod(G.tune_set)
        workspace_size = staticmethod(G.workspace_size)

    class _g:
        ntris = 1_000_000
    _g.res = res
    assert tune.max_workspace(_G, _g, 33_000_000) == b
    assert G.tune_get("max_digit_bits") == old


def test_static_build_rejects_oversize_before_device_work(G):
    """grid_build_static sizes its workspace on the host and refuses a build that
    would not fit its static scratch (no device call is made)."""
    m = re.search(r"#define GRID_STATIC_SCRATCH_BYTES \((\d+)ull << (\d+)\)", open(HEADER).read())
    assert m and int(m.group(1)) << int(m.group(2)) == G.STATIC_SCRATCH_BYTES
    o = G.grid_out(None, None, 1, 20_000_000, 0)
    res = G._u3([32, 32, 32])
    L = G.lib()
    assert G.workspace_size(4096, 20_000_000, [32, 32, 32]) > G.STATIC_SCRATCH_BYTES
    st = L.grid_build_static(None, 0, None, 4096, G._f3([0, 0, 0]), G._f3([1, 1, 1]), res, C.byref(o), None)
    assert st == G.GRID_E_NOMEM
    bad = G._u3([0, 32, 32])
    assert L.grid_build_static(None, 0, None, 0, G._f3([0, 0, 0]), G._f3([1, 1, 1]), bad, C.byref(o), None) \
        == G.GRID_E_INVAL
    assert L.grid_build_static(None, 0, None, 0, G._f3([0, 0, 0]), G._f3([1, 1, 1]), res, None, None) == G.GRID_E_INVAL


def test_culled_build_argument_checks(G):
    """grid_build_culled rejects null outputs, a null box-count pointer and bad
    grids before any device work."""
    L = G.lib()
    res = G._u3([4, 4, 4])
    lo, hi = G._f3([0, 0, 0]), G._f3([1, 1, 1])
    nb = C.c_uint64(0)
    o = G.grid_out(None, None, 1, 0, 0)
    assert L.grid_build_culled(None, 0, None, 0, lo, hi, res, None, 0, 0, None, C.byref(nb), None) == G.GRID_E_INVAL
    assert L.grid_build_culled(None, 0, None, 0, lo, hi, res, None, 0, 0, C.byref(o), None, None) == G.GRID_E_INVAL
    # a box capacity with no pair arrays to write the kept pairs into
    assert L.grid_build_culled(None, 0, None, 0, lo, hi, res, None, 0, 10, C.byref(o), C.byref(nb), None) \
        == G.GRID_E_INVAL
    assert L.grid_build_culled(None, 0, None, 0, lo, hi, G._u3([0, 4, 4]), None, 0, 0, C.byref(o), C.byref(nb),
                               None) == G.GRID_E_INVAL
