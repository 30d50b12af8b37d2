/* The library's host-side logic under AddressSanitizer and
 * UndefinedBehaviorSanitizer (host code only; no device is needed): argument
 * checks, workspace sizing, radix-sort plans, tuning knobs and error strings,
 * every call returning before any device work.  Exits 0 on success. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "gridbuild.h"

#define CHECK(c, msg) do { if (!(c)) { fprintf(stderr, "FAIL: %s\n", msg); return 1; } } while (0)

int main() {
  for (int st = -8; st <= 1; ++st) CHECK(grid_strerror(st) != nullptr, "strerror");
  const uint32_t res[3] = {524, 74, 524}, bad_res[3] = {0, 4, 4}, big_res[3] = {1025, 1, 1};
  const float lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, nan_hi[3] = {1, NAN, 1}, inf_lo[3] = {-INFINITY, 0, 0};
  size_t prev = 0;
  for (uint64_t cap = 0; cap <= (uint64_t{1} << 28); cap = cap ? cap * 4 : 1) {
    const size_t w = grid_workspace_size(1u << 20, cap, res);
    CHECK(w >= prev, "workspace grows with the capacity");
    prev = w;
  }
  CHECK(grid_workspace_size(10, 10, nullptr) == 0, "null res");
  for (uint32_t b = 0; b <= 32; ++b) {
    uint32_t passes = 0, widths[4] = {0, 0, 0, 0}, kb = 0;
    CHECK(grid_sort_plan(b, &passes, widths, &kb) == GRID_OK, "plan");
    uint32_t sum = 0;
    for (uint32_t p = 0; p < passes; ++p) sum += widths[p];
    CHECK(sum == b && passes <= 4, "plan covers the key");
  }
  CHECK(grid_sort_plan(33, nullptr, nullptr, nullptr) == GRID_E_INVAL, "plan bounds");
  CHECK(grid_tune_set("no_such_knob", 1) == GRID_E_INVAL && grid_tune_set(nullptr, 1) == GRID_E_INVAL, "knob");
  CHECK(grid_tune_set("max_digit_bits", 3) == GRID_E_INVAL && grid_tune_set("max_digit_bits", 12) == GRID_E_INVAL,
        "digit range");
  int v = 0;
  CHECK(grid_tune_get("max_digit_bits", &v) == GRID_OK && v == 9, "default digit");
  grid_out out{};
  uint32_t dummy[4];
  out.ranges = dummy;
  uint64_t nb = 0, no = 0;
  CHECK(grid_build(nullptr, 0, nullptr, 0, lo, hi, bad_res, nullptr, 0, &out, nullptr) == GRID_E_INVAL, "res 0");
  CHECK(grid_build(nullptr, 0, nullptr, 0, lo, hi, big_res, nullptr, 0, &out, nullptr) == GRID_E_INVAL, "res 1025");
  CHECK(grid_build(nullptr, 0, nullptr, 0, lo, nan_hi, res, nullptr, 0, &out, nullptr) == GRID_E_INVAL, "NaN hi");
  CHECK(grid_build(nullptr, 0, nullptr, 0, inf_lo, hi, res, nullptr, 0, &out, nullptr) == GRID_E_INVAL, "inf lo");
  CHECK(grid_build(nullptr, 0, nullptr, 0, hi, lo, res, nullptr, 0, &out, nullptr) == GRID_E_INVAL, "lo >= hi");
  CHECK(grid_build(nullptr, 0, nullptr, 5, lo, hi, res, dummy, 16, &out, nullptr) == GRID_E_INVAL, "null inputs");
  CHECK(grid_build(nullptr, 0, nullptr, 0, lo, hi, res, dummy, 16, &out, nullptr) == GRID_E_NOMEM, "small workspace");
  CHECK(grid_build_culled(nullptr, 0, nullptr, 0, lo, hi, res, nullptr, 0, 0, &out, nullptr, nullptr) ==
            GRID_E_INVAL, "culled: null box count");
  CHECK(grid_build_culled(nullptr, 0, nullptr, 0, lo, hi, res, dummy, 16, 5, &out, &nb, nullptr) == GRID_E_INVAL,
        "culled: no pair arrays");
  out.cap_pairs = uint64_t{1} << 30;
  out.cells = dummy;
  out.objs = dummy;
  CHECK(grid_build_static(nullptr, 0, nullptr, 0, lo, hi, res, &out, nullptr) == GRID_E_NOMEM, "static: too big");
  CHECK(grid_count(nullptr, 0, nullptr, 0, lo, hi, res, nullptr, 0, nullptr, nullptr, nullptr) == GRID_E_INVAL,
        "count: null npairs");
  CHECK(grid_count(nullptr, 0, nullptr, 0, lo, hi, res, dummy, 16, nullptr, &no, nullptr) == GRID_E_NOMEM,
        "count: small workspace");
  grid_desc d[2];
  memset(d, 0, sizeof(d));
  for (int g = 0; g < 2; ++g) {
    for (int a = 0; a < 3; ++a) { d[g].lo[a] = 0; d[g].hi[a] = 1; d[g].res[a] = 8; }
    d[g].out.ranges = dummy;
  }
  CHECK(grid_workspace_size_batched(d, 2) > 0, "batched sizing");
  d[1].res[2] = 0;
  CHECK(grid_workspace_size_batched(d, 2) == 0, "batched sizing rejects a bad grid");
  CHECK(grid_build_batched(d, 0, dummy, 16, nullptr) == GRID_E_INVAL, "batched: no grids");
  // the batched build split around its count: everything here is refused on the host
  d[1].res[2] = 8;
  d[0].ntris = d[1].ntris = 1;
  d[0].verts_soa = d[1].verts_soa = reinterpret_cast<const float*>(dummy);
  d[0].tris = d[1].tris = reinterpret_cast<const uint32_t*>(dummy);
  const size_t half = grid_batch_staging_size(2);
  static unsigned char staging[1 << 12];
  uint64_t counts[3] = {0, 0, 0}, cap = 7;
  CHECK(2 * half <= sizeof(staging), "staging size");
  CHECK(grid_count_batched_async(d, 2, dummy, 16, staging, 2 * half, counts, &cap, nullptr) == GRID_E_NOMEM,
        "split count: workspace below the count");
  CHECK(grid_count_batched_async(d, 2, dummy, 1 << 20, staging, half, counts, &cap, nullptr) == GRID_E_NOMEM,
        "split count: one staging table");
  CHECK(grid_count_batched_async(d, 2, dummy, 1 << 20, staging, 2 * half, nullptr, &cap, nullptr) == GRID_E_INVAL,
        "split count: no counts");
  CHECK(cap == 7, "split count: no capacity reported on failure");
  memset(staging, 0, sizeof(staging));
  for (int g = 0; g < 2; ++g) { d[g].out.cells = dummy; d[g].out.objs = dummy; d[g].out.cap_pairs = 4; }
  CHECK(grid_build_batched_counted(d, 2, dummy, 1 << 20, staging, 2 * half, nullptr) == GRID_E_INVAL,
        "split build: grids other than the counted ones");
  CHECK(grid_build_batched_counted(d, 2, dummy, 1 << 20, staging, half, nullptr) == GRID_E_NOMEM,
        "split build: one staging table");
  uint64_t tot = 0;
  CHECK(grid_scan_u32(nullptr, nullptr, nullptr, 0, GRID_SCAN_EXCLUSIVE_SUM, nullptr, 0, &tot, nullptr) == GRID_OK,
        "scan of nothing");
  CHECK(grid_scan_u32(nullptr, nullptr, nullptr, 5, 7, nullptr, 0, &tot, nullptr) == GRID_E_INVAL, "scan op");
  CHECK(grid_sort_pairs(nullptr, nullptr, nullptr, nullptr, 10, 33, nullptr, 0, nullptr) == GRID_E_INVAL, "bits");
  CHECK(grid_sort_pairs(nullptr, nullptr, nullptr, nullptr, 0, 20, nullptr, 0, nullptr) == GRID_OK, "sort nothing");
  CHECK(grid_trace_only("") == GRID_E_INVAL && grid_trace_only(nullptr) == GRID_OK, "trace filter");
  printf("ok\n");
  return 0;
}
