// Host side of the gfx950 grid builder: argument checks, workspace layout,
// the radix-sort plan and the launch sequence behind the C ABI of gridbuild.h.
#include "gridbuild.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "compact.hpp"
#include "cull.hpp"
#include "raycast.hpp"
#include "kernels.hpp"
#include "ranges.hpp"
#include "scan.hpp"
#include "sort.hpp"

using namespace gb;

namespace {

// ---- launch shapes ----------------------------------------------------------
constexpr int kCountBlock = 1024, kCountK = 8;          // 8192 triangles per count tile
constexpr int kExpandBlock = 512, kExpandK = 8;         // 4096 pairs per expansion tile
constexpr int kExpandTile = kExpandBlock * kExpandK;
constexpr int kExpandTileShift = 12;                    // tfo/tfg hold one entry per expansion tile
constexpr int kSortBlock = 512, kSortK = 16;            // radix tile shape 0 and the standalone sort: 8192 pairs
constexpr int kSortTile = kSortBlock * kSortK;
constexpr int kSortTileMin = 4096;                      // smallest tile of any radix-pass or expansion shape
constexpr int kRangesBlock = 256, kRangesK = 16;        // 4096 merge items per range tile
constexpr int kMergeTile = kRangesBlock * kRangesK;
constexpr int kScanBlock = 256, kScanK = 8;
constexpr int kMakePairsBlock = 256;                    // per-object pair generation: one thread per object
constexpr int kPlanBlock = 1024;
constexpr int kCellScanBlock = 256, kCellScanK = 16;     // compact builds: 4096 cells per scan tile
constexpr int kCellScanTile = kCellScanBlock * kCellScanK;
constexpr uint64_t kCompactMaxPairs = uint64_t{1} << 18;  // build_path = 2: compact up to this many pairs ...
constexpr double kCompactMaxPairsPerCell = 2.0;          // ... at or below this density
constexpr int kMaxRadixBits = 11;
constexpr int kKeyMapBits = 13;                         // batched key map: at most 8192 buckets
static_assert((1 << kExpandTileShift) == kExpandTile, "expansion tile must be a power of two");
static_assert(kExpandTile >= kSortTileMin && kSortTile >= kSortTileMin, "tile tables are sized by the smallest tile");

#define GB_TRY(expr)                             \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) return GRID_E_HIP;     \
  } while (0)
#define GB_LAUNCHED() GB_TRY(hipGetLastError())

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }
uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

uint32_t bits_for(uint64_t n) {  // smallest b with 2^b >= n
  uint32_t b = 0;
  while ((uint64_t{1} << b) < n) ++b;
  return b;
}

int device_cus() {
  static std::mutex mu;
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  std::lock_guard<std::mutex> lock(mu);
  if (cache[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cache[dev] = n;
  }
  return cache[dev];
}

// ---- optional per-kernel timing --------------------------------------------------
// When enabled, every launch is bracketed by a pair of HIP events recorded on
// the launch's own stream; grid_trace_read() folds them into per-kernel totals.
struct TraceRec {
  const char* name;
  hipEvent_t a, b;
};
struct Tracer {
  std::mutex mu;
  bool on = false;
  char only[48] = {0};  // when set, only launches of this kernel are traced
  std::vector<TraceRec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
Tracer& tracer() {
  static Tracer t;
  return t;
}

// A span scope brackets several launches (a build's radix passes) and is
// recorded only when selected by name, so that it never overlaps the
// per-kernel totals of a full trace.
class TraceScope {
 public:
  TraceScope(hipStream_t s, const char* name, bool span = false) : s_(s) {
    Tracer& t = tracer();
    if (!t.on) return;
    std::lock_guard<std::mutex> lock(t.mu);
    if ((t.only[0] || span) && std::strncmp(t.only, name, sizeof(t.only)) != 0) return;
    rec_.name = name;
    rec_.a = t.get();
    rec_.b = t.get();
    if (rec_.a && rec_.b && hipEventRecord(rec_.a, s_) == hipSuccess) active_ = true;
  }
  ~TraceScope() {
    if (!active_) return;
    Tracer& t = tracer();
    std::lock_guard<std::mutex> lock(t.mu);
    if (hipEventRecord(rec_.b, s_) == hipSuccess) t.recs.push_back(rec_);
  }

 private:
  hipStream_t s_;
  TraceRec rec_{};
  bool active_ = false;
};

// ---- radix-sort plan ----------------------------------------------------------
struct Plan {
  SortPlan sp;
  int rb;  // template radix bits (8..11)
};

// Tunables (grid_tune_set): the widest digit a radix pass may use, and whether
// the first radix pass regenerates its keys from the expansion (fused) or the
// expansion writes the object-order pairs and every pass reads arrays.
int g_max_digit_bits = 9;
int g_fused_expand = 0;
// Plain builds only, and only while the first radix pass reads arrays: 1 makes
// one thread per object write all of that object's pairs (the sorted-grid
// style the paper measures its per-pair expansion against), for comparison.
int g_per_object_pairs = 0;
// Plain builds: 0 = the sorted path (count, expansion, radix sort, ranges),
// 1 = the compact path (counting scatter with atomics and in-cell sorts),
// 2 = chosen per build from the count's statistics (one extra readback).
int g_build_path = 0;
int g_last_path = 0;  // the path the last plain build took
int g_sort_shape = 3;  // radix passes from arrays: 0 = 512 x 16, 1 = 256 x 16, 2 = 1024 x 8, 3 = 1024 x 16,
                       // 4 = 1024 x 15

int sort_shape_tile(int shape) { return shape == 1 ? 4096 : shape == 3 ? 16384 : shape == 4 ? 15360 : 8192; }
// 1: a build whose pairs would fill fewer 16384-pair tiles than the GPU has
// CUs runs its passes from arrays in 256 x 16 tiles, whatever sort_shape says.
int g_small_tiles = 1;

Plan make_plan(uint32_t bits, int max_digit = -1) {
  Plan p{};
  const int md = std::min(kMaxRadixBits, std::max(4, max_digit > 0 ? max_digit : g_max_digit_bits));
  if (bits == 0) {
    p.sp.passes = 0;
    p.rb = 8;
    return p;
  }
  // at most 4 passes (the plan's arrays and the histogram slots): a narrow
  // digit limit on a wide key widens the digits instead (32 bits / 4 = 8)
  const uint32_t passes = std::min<uint32_t>(4, (bits + md - 1) / md);
  // widths as even as possible: a wider digit costs its pass more counters,
  // look-back words and shorter scatter runs.  The wider digits are the top
  // ones (25 bits: 8, 8, 9): keys below a cell count that is not a power of
  // two take fewer values in the top digit than its width allows, so the
  // wide pass gets longer runs than it would on the low digit
  const uint32_t base = bits / passes, extra = bits % passes;
  p.sp.passes = passes;
  uint32_t shift = 0;
  for (uint32_t i = 0; i < passes; ++i) {
    p.sp.shift[i] = shift;
    p.sp.width[i] = base + (i >= passes - extra ? 1u : 0u);
    shift += p.sp.width[i];
  }
  p.rb = std::max(8, static_cast<int>(base + (extra ? 1u : 0u)));
  return p;
}

// ---- workspace layout -----------------------------------------------------------
// (tfo_work_cap, the tile-owner runs the count can leave to the plan kernel, is in tiles.hpp)

struct Layout {
  size_t ctl, hist, count_status, cull_status, cell_status, zero_end;
  size_t start, box, tfo, tfg, tfo_work, cull_rec, sort_status, keys_alt, vals_alt, keys_alt2, vals_alt2, run, npairs_out, splits,
      tile_grid, table, sink, kmap, ksink, total;
  uint32_t ntfo, ncount_tiles, nsort_tiles_cap, nmerge_tiles_cap;
};

Layout make_layout(uint64_t ntris, uint64_t cap_pairs, uint64_t ncells_plus_grids, const Plan& plan,
                   uint32_t ngrids, bool batched, bool culled = false) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + std::max<size_t>(bytes, 1));
    return at;
  };
  L.ncount_tiles = static_cast<uint32_t>(ceil_div(ntris, kCountBlock * kCountK));
  L.nsort_tiles_cap = static_cast<uint32_t>(ceil_div(cap_pairs, kSortTileMin));
  L.ntfo = L.nsort_tiles_cap + 1;
  L.nmerge_tiles_cap = static_cast<uint32_t>(ceil_div(ncells_plus_grids + cap_pairs, kMergeTile) + ngrids);
  L.ctl = take(sizeof(Control));
  L.hist = take(static_cast<size_t>(kHistCopies) * 4 * kRadixMax * sizeof(uint32_t));
  L.count_status = take(std::max<size_t>(L.ncount_tiles, 1) * 8);
  L.cull_status = take(static_cast<size_t>(L.ntfo) * 8);  // culled builds: one word per expansion tile
  L.cell_status = take(batched ? 0 : (ceil_div(ncells_plus_grids, kCellScanTile) + 1) * 8);  // compact builds
  L.zero_end = o;
  L.start = take(ntris * 4);
  L.box = take(ntris * 8);
  L.tfo = take(static_cast<size_t>(L.ntfo) * 4);
  L.tfg = take(batched ? static_cast<size_t>(L.ntfo) * 4 : 0);
  L.tfo_work = take(tfo_work_cap(L.ntfo) * sizeof(uint4));
  L.cull_rec = take(culled ? ntris * sizeof(CullRecord) : 0);  // culled builds: each triangle's test
  L.sort_status = take(static_cast<size_t>(plan.sp.passes) * L.nsort_tiles_cap * (size_t{1} << plan.rb) * 8);
  L.keys_alt = take(cap_pairs * 4);
  L.vals_alt = take(cap_pairs * 4);
  // batched builds scatter their last pass into per-grid outputs, so the
  // passes before it ping-pong between two workspace buffers
  L.keys_alt2 = take(batched ? cap_pairs * 4 : 0);
  L.vals_alt2 = take(batched ? cap_pairs * 4 : 0);
  L.run = take((ngrids + 1) * sizeof(GridRun));
  L.npairs_out = take((ngrids + 1) * 8);  // per-grid NO, then the count's status word
  L.splits = take(static_cast<size_t>(L.nmerge_tiles_cap) * 4);
  L.tile_grid = take(batched ? static_cast<size_t>(L.nmerge_tiles_cap) * 4 : 0);
  L.table = take(batched ? ngrids * sizeof(GridDev) : 0);
  L.sink = take(batched ? ngrids * sizeof(GridSink) : 0);
  L.kmap = take(batched ? (size_t{1} << kKeyMapBits) * sizeof(uint2) : 0);
  L.ksink = take(batched ? (size_t{1} << kKeyMapBits) * sizeof(GridSink) : 0);
  L.total = o + 256;
  return L;
}

template <class T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// ---- argument checks --------------------------------------------------------------
bool finite(float x) { return std::isfinite(x); }

int check_grid(const float lo[3], const float hi[3], const uint32_t res[3]) {
  if (!lo || !hi || !res) return GRID_E_INVAL;
  for (int a = 0; a < 3; ++a) {
    if (!finite(lo[a]) || !finite(hi[a]) || !(lo[a] < hi[a])) return GRID_E_INVAL;
    if (res[a] < 1 || res[a] > 1024) return GRID_E_INVAL;
  }
  return GRID_OK;
}

uint64_t ncells_of(const uint32_t res[3]) { return static_cast<uint64_t>(res[0]) * res[1] * res[2]; }

GridDev make_grid(const float* verts, uint32_t nverts, const uint32_t* tris, uint32_t ntris, const float lo[3],
                  const float hi[3], const uint32_t res[3]) {
  GridDev g{};
  g.verts = verts;
  g.tris = tris;
  g.nverts = nverts;
  g.ntris = ntris;
  for (int a = 0; a < 3; ++a) {
    g.res[a] = res[a];
    g.lo[a] = lo[a];
    const float ext = hi[a] - lo[a];              // FP32, as the grid contract states
    g.inv[a] = static_cast<float>(res[a]) / ext;  // IEEE division on the host
  }
  return g;
}

// ---- the launch sequence ------------------------------------------------------------
__global__ void zero_kernel(uint64_t* p, uint64_t nwords) {
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < nwords;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    p[i] = 0;
}

int launch_zero(void* ws, size_t bytes, hipStream_t s) {
  const uint64_t words = bytes / 8;
  const uint32_t blocks = static_cast<uint32_t>(std::min<uint64_t>(ceil_div(words, 256), 1024));
  TraceScope ts(s, "zero");
  zero_kernel<<<std::max(blocks, 1u), 256, 0, s>>>(static_cast<uint64_t*>(ws), words);
  GB_LAUNCHED();
  return GRID_OK;
}

__global__ void fill_u32_kernel(uint32_t* p, uint64_t n, uint32_t v) {
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

struct Build {
  void* ws;
  Layout L;
  Plan plan;
  GridSet gs;
  uint32_t ntris;
  bool batched;
  uint64_t batch_cells;  // batched: cells of all grids (the sort-key space)
  hipStream_t s;
  bool culled;           // plain builds: false intersections removed before the sort
  uint64_t out_cap;      // culled builds: pairs the caller's outputs hold
  uint64_t layout_cap = ~uint64_t{0};  // pairs the workspace layout holds, checked by the plan
  bool no_alloc = false;  // the build may not allocate, not even host memory for its readback
  int sort_shape = 3;     // tile shape of the radix passes from arrays (build_sort_shape)
};

template <bool B>
int launch_count(Build& b) {
  if (b.ntris == 0) return GRID_OK;
  CountArgs a{};
  a.gs = b.gs;
  a.ntris = b.ntris;
  a.start = at<uint32_t>(b.ws, b.L.start);
  a.box = at<uint64_t>(b.ws, b.L.box);
  a.tfo = at<uint32_t>(b.ws, b.L.tfo);
  a.tfg = at<uint32_t>(b.ws, b.L.tfg);
  a.ntfo = b.L.ntfo;
  a.tile_shift = kExpandTileShift;
  a.status = at<uint64_t>(b.ws, b.L.count_status);
  a.tfo_work = at<uint4>(b.ws, b.L.tfo_work);
  a.tfo_work_cap = tfo_work_cap(b.L.ntfo);
  a.ctl = at<Control>(b.ws, b.L.ctl);
  TraceScope ts(b.s, "count_scan");
  count_kernel<kCountBlock, kCountK, B><<<b.L.ncount_tiles, kCountBlock, 0, b.s>>>(a);
  GB_LAUNCHED();
  return GRID_OK;
}

template <bool B>
int launch_plan(Build& b) {
  PlanArgs a{};
  a.gs = b.gs;
  a.start = at<uint32_t>(b.ws, b.L.start);
  a.ntris = b.ntris;
  a.merge_tile = kMergeTile;
  a.run = at<GridRun>(b.ws, b.L.run);
  a.npairs_out = at<uint64_t>(b.ws, b.L.npairs_out);
  a.cap_flag = &at<Control>(b.ws, b.L.ctl)->cap_flag;
  a.cap_total = b.layout_cap;
  a.tfo = at<uint32_t>(b.ws, b.L.tfo);
  a.tfg = at<uint32_t>(b.ws, b.L.tfg);
  a.tfo_work = at<uint4>(b.ws, b.L.tfo_work);
  a.tfo_work_cap = tfo_work_cap(b.L.ntfo);
  a.ctl = at<Control>(b.ws, b.L.ctl);
  TraceScope ts(b.s, "plan");
  plan_kernel<kPlanBlock, B><<<1, kPlanBlock, 0, b.s>>>(a);
  GB_LAUNCHED();
  return GRID_OK;
}

ExpandArgs expand_args(const Build& b) {
  ExpandArgs e{};
  e.gs = b.gs;
  e.start = at<uint32_t>(b.ws, b.L.start);
  e.box = at<uint64_t>(b.ws, b.L.box);
  e.tfo = at<uint32_t>(b.ws, b.L.tfo);
  e.tfg = at<uint32_t>(b.ws, b.L.tfg);
  e.ntris = b.ntris;
  e.ctl = at<Control>(b.ws, b.L.ctl);
  return e;
}

uint32_t persistent_blocks(uint64_t tiles, int per_cu) {
  const uint64_t cap = static_cast<uint64_t>(device_cus()) * per_cu;
  return static_cast<uint32_t>(std::max<uint64_t>(1, std::min<uint64_t>(tiles, cap)));
}

// Workgroups of `kernel` that fit on the device at once (occupancy query,
// cached per kernel), so a persistent grid is exactly one resident wave.
template <class F>
uint32_t resident_blocks(F kernel, int block, uint64_t tiles) {
  static std::mutex mu;
  static std::vector<std::pair<const void*, int>> cache;
  const void* key = reinterpret_cast<const void*>(kernel);
  int per_cu = 0;
  {
    std::lock_guard<std::mutex> lock(mu);
    for (auto& e : cache)
      if (e.first == key) per_cu = e.second;
    if (per_cu == 0) {
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess || per_cu <= 0)
        per_cu = 1;
      cache.emplace_back(key, per_cu);
    }
  }
  return persistent_blocks(tiles, per_cu);
}

int pass_bits(uint32_t width);

// Tile size of radix pass p under the current knobs (a regenerating first pass
// reads the expansion's tiles; the others take the sort_shape tile).
bool fused_first_pass(const Build& b) { return g_fused_expand != 0 && !b.culled; }

uint32_t pass_tile(const Build& b, uint32_t p) {
  return (fused_first_pass(b) && p == 0) ? static_cast<uint32_t>(kExpandTile)
                                         : static_cast<uint32_t>(sort_shape_tile(b.sort_shape));
}

// Radix tile shape for a build of at most cap_pairs pairs: the sort_shape
// knob's, unless the pairs would fill fewer 16384-pair tiles than the GPU has
// CUs.  Each tile's phases take about the same time whatever its size, so a
// build with few tiles finishes sooner with more, smaller tiles spread over
// more CUs (a 17K-pair pass: 15 against 20 us).
int build_sort_shape(uint64_t cap_pairs) {
  if (g_small_tiles && ceil_div(cap_pairs, 16384) < static_cast<uint64_t>(device_cus())) return 1;
  return g_sort_shape;
}

// The look-back words each radix pass of b's plan will use (kernels built for
// RB-bit digits lay the passes out RB-wide).
StatusClear status_clear(const Build& b, int RB) {
  StatusClear c{};
  c.status = at<uint64_t>(b.ws, b.L.sort_status);
  c.stride = static_cast<uint64_t>(b.L.nsort_tiles_cap) * (RB > 0 ? (1u << RB) : 1u);
  c.passes = RB > 0 ? b.plan.sp.passes : 0;
  for (uint32_t p = 0; p < c.passes; ++p) {
    c.tile[p] = pass_tile(b, p);
    c.radix[p] = 1u << pass_bits(b.plan.sp.width[p]);
  }
  return c;
}

template <int RB, bool B>
int launch_expand(Build& b, uint32_t* cells, uint32_t* objs, uint64_t npairs) {
  if (npairs == 0) return GRID_OK;
  if (!cells || !objs) return GRID_E_INVAL;
  ExpandOutArgs a{};
  a.ex = expand_args(b);
  a.cells = cells;
  a.objs = objs;
  a.plan = b.plan.sp;
  a.hist = at<uint32_t>(b.ws, b.L.hist);
  a.clear = status_clear(b, RB);
  a.vec16 = ((reinterpret_cast<uintptr_t>(cells) | reinterpret_cast<uintptr_t>(objs)) & 15u) == 0;
  a.ctl = at<Control>(b.ws, b.L.ctl);
  if constexpr (!B) {
    if (g_per_object_pairs) {
      TraceScope ts(b.s, RB > 0 ? "makepairs_hist" : "makepairs");
      const uint32_t blocks = static_cast<uint32_t>(std::max<uint64_t>(1, ceil_div(b.ntris, kMakePairsBlock)));
      makepairs_kernel<kMakePairsBlock, RB><<<blocks, kMakePairsBlock, 0, b.s>>>(a);  // one thread per object
      GB_LAUNCHED();
      return GRID_OK;
    }
  }
  {
    TraceScope ts(b.s, RB > 0 ? "expand_hist" : "expand");
    auto kern = expand_kernel<kExpandBlock, kExpandK, RB, B>;
    kern<<<resident_blocks(kern, kExpandBlock, ceil_div(npairs, kExpandTile)), kExpandBlock, 0, b.s>>>(a);
    GB_LAUNCHED();
  }
  if constexpr (B) {
    // the tiles that straddle grids, skipped above (a batch of one grid has none)
    if (b.gs.ngrids < 2) return GRID_OK;
    TraceScope ts(b.s, "expand_straddle");
    auto kern = expand_straddle_kernel<kExpandBlock, kExpandK, RB>;
    kern<<<static_cast<uint32_t>(std::min<uint64_t>(ceil_div(npairs, kExpandTile), 1024)), kExpandBlock, 0, b.s>>>(a);
    GB_LAUNCHED();
  }
  return GRID_OK;
}

// The compact path of a plain build (after the count and the plan): counts
// per cell, their scan into the range table, the counting scatter and the
// in-cell sorts.  out->ranges serves as the per-cell counters throughout.
int launch_compact(Build& b, const grid_out* out) {
  CompactArgs a{};
  a.ex = expand_args(b);
  a.ranges = out->ranges;
  a.cells = out->cells;
  a.objs = out->objs;
  a.cap = out->cap_pairs;
  a.ncells = ncells_of(b.gs.one.res);
  a.status = at<uint64_t>(b.ws, b.L.cell_status);
  a.big = at<uint2>(b.ws, b.L.vals_alt);                       // the radix buffers are free on this path
  a.big_cap = static_cast<uint32_t>(std::min<uint64_t>(out->cap_pairs / 2, 0xFFFFFFFFull));
  a.scratch = at<uint32_t>(b.ws, b.L.keys_alt);
  a.ctl = at<Control>(b.ws, b.L.ctl);
  const uint64_t cap = out->cap_pairs;
  {
    TraceScope ts(b.s, "compact_zero");
    const uint64_t n = 2 * a.ncells;
    fill_u32_kernel<<<static_cast<uint32_t>(std::max<uint64_t>(1, std::min<uint64_t>(ceil_div(n, 256), 4096))), 256, 0,
                      b.s>>>(out->ranges, n, 0u);
    GB_LAUNCHED();
  }
  if (cap > 0) {
    TraceScope ts(b.s, "compact_count");
    auto kern = compact_count_kernel<kExpandBlock, kExpandK>;
    kern<<<resident_blocks(kern, kExpandBlock, ceil_div(cap, kExpandTile)), kExpandBlock, 0, b.s>>>(a);
    GB_LAUNCHED();
  }
  {
    TraceScope ts(b.s, "compact_scan");
    auto kern = compact_scan_kernel<kCellScanBlock, kCellScanK>;
    kern<<<resident_blocks(kern, kCellScanBlock, ceil_div(a.ncells, kCellScanTile)), kCellScanBlock, 0, b.s>>>(a);
    GB_LAUNCHED();
  }
  if (cap > 0) {
    {
      TraceScope ts(b.s, "compact_scatter");
      auto kern = compact_scatter_kernel<kExpandBlock, kExpandK>;
      kern<<<resident_blocks(kern, kExpandBlock, ceil_div(cap, kExpandTile)), kExpandBlock, 0, b.s>>>(a);
      GB_LAUNCHED();
    }
    {
      TraceScope ts(b.s, "compact_sort_small");
      compact_sort_small_kernel<256><<<static_cast<uint32_t>(std::max<uint64_t>(1, std::min<uint64_t>(ceil_div(a.ncells, 256), 8192))),
                                      256, 0, b.s>>>(a);
      GB_LAUNCHED();
    }
    {
      TraceScope ts(b.s, "compact_sort_big");
      compact_sort_big_kernel<256><<<1024, 256, 0, b.s>>>(a);
      GB_LAUNCHED();
    }
  }
  return GRID_OK;
}

// The path a plain build takes when it is left to the statistics (knob
// build_path = 2): the compact path's atomics cost more per pair than the
// sorted path's passes, so it only pays where launches dominate, small sparse
// grids (measured on MI355X: 0.78-0.90 of the sorted time up to 150K pairs,
// 1.24 at 0.9M, 3.7-10 beyond).
int choose_path(uint64_t npairs, uint64_t ncells) {
  if (npairs == 0) return 0;
  return npairs <= kCompactMaxPairs && static_cast<double>(npairs) <= kCompactMaxPairsPerCell * ncells ? 1 : 0;
}

// Culled builds: the expansion that tests every box pair and keeps the pairs
// whose triangle touches the cell (into cells/objs, at most dest_cap of them),
// then the kept count made the build's pair count.
template <int RB>
int launch_cull(Build& b, uint32_t* cells, uint32_t* objs, uint64_t dest_cap, uint64_t box_cap) {
  if (box_cap > 0) {
    if (!cells || !objs) return GRID_E_INVAL;
    CullRecordArgs r{};
    r.grid = b.gs.one;
    r.box = at<uint64_t>(b.ws, b.L.box);
    r.rec = at<CullRecord>(b.ws, b.L.cull_rec);
    r.ntris = b.ntris;
    r.ctl = at<Control>(b.ws, b.L.ctl);
    if (b.ntris > 0) {
      TraceScope tr(b.s, "cull_record");
      cull_record_kernel<256><<<static_cast<uint32_t>(std::min<uint64_t>(ceil_div(b.ntris, 256), 8192)), 256, 0,
                                b.s>>>(r);
      GB_LAUNCHED();
    }
    CullArgs a{};
    a.rec = reinterpret_cast<const float4*>(r.rec);
    a.o.ex = expand_args(b);
    a.o.cells = cells;
    a.o.objs = objs;
    a.o.plan = b.plan.sp;
    a.o.hist = at<uint32_t>(b.ws, b.L.hist);
    a.o.clear = status_clear(b, RB);
    a.o.ctl = at<Control>(b.ws, b.L.ctl);
    a.dest_cap = dest_cap;
    a.status = at<uint64_t>(b.ws, b.L.cull_status);
    TraceScope ts(b.s, RB > 0 ? "expand_cull_hist" : "expand_cull");
    auto kern = expand_cull_kernel<kExpandBlock, kExpandK, RB>;
    kern<<<resident_blocks(kern, kExpandBlock, ceil_div(box_cap, kExpandTile)), kExpandBlock, 0, b.s>>>(a);
    GB_LAUNCHED();
  }
  CullCommitArgs c{};
  c.ctl = at<Control>(b.ws, b.L.ctl);
  c.run = at<GridRun>(b.ws, b.L.run);
  c.out_cap = b.out_cap;
  c.ncells = ncells_of(b.gs.one.res);
  c.merge_tile = kMergeTile;
  TraceScope ts(b.s, "cull_commit");
  cull_commit_kernel<<<1, kWave, 0, b.s>>>(c);
  GB_LAUNCHED();
  return GRID_OK;
}

// Each pass runs the kernel built for its own digit width (8..11 bits), so an
// 8-bit pass of a 25-bit key does not pay for 9-bit ranking.
int pass_bits(uint32_t width) { return std::max(8, static_cast<int>(width)); }

// Passes that read arrays come in two builds, by look-back word width.
template <int Blk, int K, int RB, int Src, int Snk, bool B>
void launch_onesweep(const SortPassArgs& a, uint32_t ntiles, hipStream_t s) {
  if constexpr (Src == kFromArrays) {
    if (a.narrow) {
      auto k = onesweep_kernel<Blk, K, RB, Src, Snk, B, true>;
      k<<<resident_blocks(k, Blk, ntiles), Blk, 0, s>>>(a);
      return;
    }
  }
  auto k = onesweep_kernel<Blk, K, RB, Src, Snk, B, false>;
  k<<<resident_blocks(k, Blk, ntiles), Blk, 0, s>>>(a);
}

// A pass that reads arrays runs in the tile shape the sort_shape knob picks.
template <int RB, int Snk, bool B>
void launch_shaped(const SortPassArgs& a, uint32_t ntiles, hipStream_t s, int shape) {
  switch (shape) {
    case 1: launch_onesweep<256, 16, RB, kFromArrays, Snk, B>(a, ntiles, s); break;
    case 2: launch_onesweep<1024, 8, RB, kFromArrays, Snk, B>(a, ntiles, s); break;
    case 3: launch_onesweep<1024, 16, RB, kFromArrays, Snk, B>(a, ntiles, s); break;
    case 4: launch_onesweep<1024, 15, RB, kFromArrays, Snk, B>(a, ntiles, s); break;
    default: launch_onesweep<kSortBlock, kSortK, RB, kFromArrays, Snk, B>(a, ntiles, s); break;
  }
}

template <int RB, bool B>
int launch_pass_rb(const SortPassArgs& a, bool regen, bool to_grids, uint32_t ntiles, hipStream_t s, int shape) {
  if (regen) {
    // regenerating passes read the expansion, whose tiles are kExpandTile pairs
    if (to_grids) launch_onesweep<kExpandBlock, kExpandK, RB, kFromExpansion, kToGrids, B>(a, ntiles, s);
    else launch_onesweep<kExpandBlock, kExpandK, RB, kFromExpansion, kToArrays, B>(a, ntiles, s);
  } else if (to_grids) {
    if constexpr (B) launch_shaped<RB, kToGrids, B>(a, ntiles, s, shape);
    else return GRID_E_INVAL;  // plain builds end in the caller's arrays
  } else {
    launch_shaped<RB, kToArrays, B>(a, ntiles, s, shape);
  }
  GB_LAUNCHED();
  return GRID_OK;
}

template <bool B>
int launch_pass(SortPassArgs a, int rb, bool regen, bool to_grids, uint32_t ntiles, hipStream_t s, int shape) {
  switch (rb) {
    case 8: return launch_pass_rb<8, B>(a, regen, to_grids, ntiles, s, shape);
    case 9: return launch_pass_rb<9, B>(a, regen, to_grids, ntiles, s, shape);
    case 10: return launch_pass_rb<10, B>(a, regen, to_grids, ntiles, s, shape);
    case 11: return launch_pass_rb<11, B>(a, regen, to_grids, ntiles, s, shape);
    default: return GRID_E_INVAL;
  }
}

// Destination of writer i of the sort sequence (i = -1: the unfused
// expansion, i = 0..P-1: the radix passes).  Plain builds end in the caller's
// arrays; batched builds end in the per-grid outputs (nullptr here).
struct Dest {
  uint32_t* k;
  uint32_t* v;
};
Dest sort_dest(const Build& b, bool batched, int i, uint32_t P, uint32_t* out_k, uint32_t* out_v) {
  uint32_t* ak = at<uint32_t>(b.ws, b.L.keys_alt);
  uint32_t* av = at<uint32_t>(b.ws, b.L.vals_alt);
  if (batched) {
    if (i == static_cast<int>(P) - 1) return {nullptr, nullptr};
    const bool first = ((i + 1) % 2) == 0;  // -1 -> alt, 0 -> alt2, 1 -> alt, ...
    if (!g_fused_expand) return first ? Dest{ak, av} : Dest{at<uint32_t>(b.ws, b.L.keys_alt2), at<uint32_t>(b.ws, b.L.vals_alt2)};
    return (i % 2 == 0) ? Dest{ak, av} : Dest{at<uint32_t>(b.ws, b.L.keys_alt2), at<uint32_t>(b.ws, b.L.vals_alt2)};
  }
  const bool to_out = ((static_cast<int>(P) - 1 - i) % 2) == 0;
  return to_out ? Dest{out_k, out_v} : Dest{ak, av};
}

// Batched builds: the per-grid sinks and the key map of the last radix pass.
int launch_sink(Build& b) {
  const uint32_t kbits = bits_for(b.batch_cells);
  SinkArgs a{};
  a.gs = b.gs;
  a.run = at<GridRun>(b.ws, b.L.run);
  a.cap_flag = &at<Control>(b.ws, b.L.ctl)->cap_flag;
  a.sink = at<GridSink>(b.ws, b.L.sink);
  a.kmap = at<uint2>(b.ws, b.L.kmap);
  a.ksink = at<GridSink>(b.ws, b.L.ksink);
  a.kshift = kbits > static_cast<uint32_t>(kKeyMapBits) ? kbits - kKeyMapBits : 0;
  a.ncells = b.batch_cells;
  a.nbuckets = static_cast<uint32_t>(((b.batch_cells - 1) >> a.kshift) + 1);
  if (b.batch_cells == 0 || a.nbuckets > (1u << kKeyMapBits)) return GRID_E_INVAL;
  const uint32_t items = std::max(a.nbuckets, b.gs.ngrids);
  TraceScope ts(b.s, "sink");
  sink_kernel<256><<<static_cast<uint32_t>(std::min<uint64_t>(ceil_div(items, 256), 1024)), 256, 0, b.s>>>(a);
  GB_LAUNCHED();
  return GRID_OK;
}

// Radix passes of fewer pairs than this use 32-bit look-back words (a 30-bit
// value each): half the stores and polls of 64-bit words.  The wide_lookback
// knob keeps 64-bit words for every build.
constexpr uint64_t kNarrowLimit = uint64_t{1} << 30;
int g_wide_lookback = 0;
uint32_t narrow_words(uint64_t max_pairs) { return !g_wide_lookback && max_pairs < kNarrowLimit ? 1u : 0u; }

template <int RB, bool B>
int launch_sort_rb(Build& b, uint32_t* out_cells, uint32_t* out_objs, uint64_t npairs) {
  const SortPlan& sp = b.plan.sp;
  if constexpr (B) {
    int st = launch_sink(b);
    if (st) return st;
  }
  const uint32_t ntiles = static_cast<uint32_t>(ceil_div(npairs, kExpandTile));
  Control* ctl = at<Control>(b.ws, b.L.ctl);
  const uint32_t P = sp.passes;
  const bool fused = fused_first_pass(b);
  b.sort_shape = build_sort_shape(npairs);  // before anything sizes or clears the passes' look-back words
  const uint32_t* in_k = nullptr;
  const uint32_t* in_v = nullptr;
  if (fused) {
    HistArgs h{};
    h.ex = expand_args(b);
    h.plan = sp;
    h.hist = at<uint32_t>(b.ws, b.L.hist);
    h.clear = status_clear(b, RB);
    h.ctl = ctl;
    TraceScope ts(b.s, "hist");
    auto kern = hist_kernel<kExpandBlock, kExpandK, RB, B>;
    kern<<<resident_blocks(kern, kExpandBlock, ntiles), kExpandBlock, 0, b.s>>>(h);
    GB_LAUNCHED();
  } else {
    const Dest d = sort_dest(b, B, -1, P, out_cells, out_objs);
    int st;
    if (!B && b.culled) {
      // the kept pairs go where the expansion's would: the caller's arrays or the workspace's
      const uint64_t dest_cap = d.k == out_cells ? b.out_cap : npairs;
      st = launch_cull<RB>(b, d.k, d.v, dest_cap, npairs);
    } else {
      st = launch_expand<RB, B>(b, d.k, d.v, npairs);
    }
    if (st) return st;
    in_k = d.k;
    in_v = d.v;
  }
  {
    TraceScope span(b.s, "radix_passes", true);  // all of the build's passes, between two events
    for (uint32_t p = 0; p < P; ++p) {
      const Dest d = sort_dest(b, B, static_cast<int>(p), P, out_cells, out_objs);
      const bool last = p + 1 == P;
      if ((!B || !last) && (!d.k || !d.v)) return GRID_E_INVAL;  // never launch a pass without a destination
      SortPassArgs a{};
      a.keys_in = in_k;
      a.vals_in = in_v;
      a.keys_out = d.k;
      a.vals_out = d.v;
      a.ex = expand_args(b);
      a.hist = at<uint32_t>(b.ws, b.L.hist) + p * kRadixMax;
      a.hist_copies = kHistCopies;
      a.hist_stride = 4 * kRadixMax;
      a.status = at<uint64_t>(b.ws, b.L.sort_status) + static_cast<uint64_t>(p) * b.L.nsort_tiles_cap * (1u << RB);
      a.n = npairs;
      a.n_from_ctl = 1;  // the pass reads NO from the control block
      a.narrow = narrow_words(npairs);  // NO <= the capacity npairs
      a.shift = sp.shift[p];
      a.width = sp.width[p];
      a.counter = kCtrSort0 + p;
      a.sink = at<GridSink>(b.ws, b.L.sink);
      a.kmap = at<uint2>(b.ws, b.L.kmap);
      a.ksink = at<GridSink>(b.ws, b.L.ksink);
      {
        const uint32_t kbits = bits_for(b.batch_cells);
        a.kshift = kbits > static_cast<uint32_t>(kKeyMapBits) ? kbits - kKeyMapBits : 0;
      }
      a.ctl = ctl;
      const bool regen = fused && p == 0;
      const uint32_t pass_tiles = static_cast<uint32_t>(ceil_div(npairs, pass_tile(b, p)));
      TraceScope ts(b.s, regen ? "onesweep_expand" : (B && last) ? "onesweep_grids" : "onesweep");
      int st = launch_pass<B>(a, pass_bits(sp.width[p]), regen, B && last, pass_tiles, b.s, b.sort_shape);
      if (st) return st;
      GB_LAUNCHED();
      in_k = d.k;
      in_v = d.v;
    }
  }
  return GRID_OK;
}

bool plan_ok(const Plan& p) {
  if (p.sp.passes > 4) return false;
  for (uint32_t i = 0; i < p.sp.passes; ++i)
    if (p.sp.width[i] < 1 || static_cast<int>(p.sp.width[i]) > p.rb || p.sp.shift[i] + p.sp.width[i] > 32) return false;
  return p.rb >= 8 && p.rb <= kMaxRadixBits;
}

template <bool B>
int launch_sort(Build& b, uint32_t* out_cells, uint32_t* out_objs, uint64_t npairs) {
  if (!plan_ok(b.plan)) return GRID_E_INVAL;  // never launch digits wider than the kernel's counters
  switch (b.plan.rb) {
    case 8: return launch_sort_rb<8, B>(b, out_cells, out_objs, npairs);
    case 9: return launch_sort_rb<9, B>(b, out_cells, out_objs, npairs);
    case 10: return launch_sort_rb<10, B>(b, out_cells, out_objs, npairs);
    case 11: return launch_sort_rb<11, B>(b, out_cells, out_objs, npairs);
    default: return GRID_E_INVAL;
  }
}

template <bool B>
int launch_ranges(Build& b, uint64_t merge_items_cap) {
  RangesArgs a{};
  a.gs = b.gs;
  a.run = at<GridRun>(b.ws, b.L.run);
  a.splits = at<uint32_t>(b.ws, b.L.splits);
  a.tile_grid = at<uint32_t>(b.ws, b.L.tile_grid);
  a.merge_tile = kMergeTile;
  a.ctl = at<Control>(b.ws, b.L.ctl);
  const uint64_t tiles = ceil_div(merge_items_cap, kMergeTile) + b.gs.ngrids;
  {
  TraceScope ts(b.s, "split");
  split_kernel<256, B><<<static_cast<uint32_t>(std::max<uint64_t>(1, std::min<uint64_t>(ceil_div(tiles, 256), 4096))),
                         256, 0, b.s>>>(a);
  GB_LAUNCHED();
  }
  TraceScope ts(b.s, "ranges");
  auto kern = ranges_kernel<kRangesBlock, kRangesK, B>;
  kern<<<resident_blocks(kern, kRangesBlock, tiles), kRangesBlock, 0, b.s>>>(a);
  GB_LAUNCHED();
  return GRID_OK;
}

struct HostCtl {
  uint64_t npairs;
  uint32_t error;
  uint32_t cap_flag;
  uint64_t box_npairs;
};

// Status of the device-side error bits (0 when none is set).
int device_error(uint32_t error) {
  if (error & kErrBadIndex) return GRID_E_BADINDEX;
  if (error & kErrInternal) return GRID_E_INTERNAL;
  return GRID_OK;
}

// Host end of the control block's readback: one pinned block per host thread,
// allocated by that thread's first synchronous build and kept until the
// process ends.  A copy into pinned memory is one DMA; a copy into pageable
// memory goes through the runtime's staging buffer and costs about 28 us more
// per build.  nullptr (and the pageable path) if the allocation fails.
Control* pinned_ctl() {
  static thread_local Control* pin = nullptr;
  static thread_local bool tried = false;
  if (!tried) {
    tried = true;
    if (hipHostMalloc(reinterpret_cast<void**>(&pin), sizeof(Control), hipHostMallocDefault) != hipSuccess) {
      pin = nullptr;
      (void)hipGetLastError();  // not left for the next launch check to report
    }
  }
  return pin;
}

int read_ctl(const Build& b, HostCtl* h) {
  Control local;
  Control* c = b.no_alloc ? nullptr : pinned_ctl();
  if (!c) c = &local;
  GB_TRY(hipMemcpyAsync(c, at<Control>(b.ws, b.L.ctl), sizeof(Control), hipMemcpyDeviceToHost, b.s));
  GB_TRY(hipStreamSynchronize(b.s));
  h->npairs = c->npairs;
  h->error = c->error;
  h->cap_flag = c->cap_flag;
  h->box_npairs = c->box_npairs;
  return GRID_OK;
}

int prepare_plain(Build& b, const float* verts, uint32_t nverts, const uint32_t* tris, uint32_t ntris,
                  const float lo[3], const float hi[3], const uint32_t res[3], void* ws, size_t ws_bytes,
                  uint64_t cap_pairs, hipStream_t s, bool culled = false) {
  int st = check_grid(lo, hi, res);
  if (st != GRID_OK) return st;
  if (!ws) return GRID_E_INVAL;
  if (ntris > 0 && (!verts || !tris)) return GRID_E_INVAL;
  if (ntris >= (1u << 31)) return GRID_E_INVAL;
  b.ws = ws;
  b.s = s;
  b.ntris = ntris;
  b.batched = false;
  b.plan = make_plan(bits_for(ncells_of(res)));
  b.L = make_layout(ntris, cap_pairs, ncells_of(res) + 1, b.plan, 1, false, culled);
  if (ws_bytes < b.L.total) return GRID_E_NOMEM;
  b.gs = GridSet{};
  b.gs.one = make_grid(verts, nverts, tris, ntris, lo, hi, res);
  b.gs.one.cap_pairs = cap_pairs;
  b.gs.ngrids = 1;
  return GRID_OK;
}

int count_phase_plain(Build& b, HostCtl* h) {
  int st = launch_zero(b.ws, b.L.zero_end, b.s);
  if (st) return st;
  if ((st = launch_count<false>(b))) return st;
  if ((st = read_ctl(b, h))) return st;
  if (h->error) return device_error(h->error);
  if (h->npairs > 0xFFFFFFFFull) return GRID_E_OVERFLOW;
  return GRID_OK;
}

}  // namespace

extern "C" {

const char* grid_strerror(int status) {
  switch (status) {
    case GRID_OK: return "ok";
    case GRID_E_INVAL: return "invalid argument";
    case GRID_E_NOMEM: return "workspace too small";
    case GRID_E_OVERFLOW: return "pair count exceeds 2^32 - 1";
    case GRID_E_CAPACITY: return "pair capacity too small";
    case GRID_E_BADINDEX: return "vertex index out of range";
    case GRID_E_HIP: return "HIP runtime error";
    case GRID_E_INTERNAL: return "internal consistency check failed";
    default: return "unknown status";
  }
}

size_t grid_workspace_size(uint32_t ntris, uint64_t cap_pairs, const uint32_t res[3]) {
  if (!res) return 0;
  const uint64_t nc = ncells_of(res);
  return make_layout(ntris, cap_pairs, nc + 1, make_plan(bits_for(nc)), 1, false).total;
}

size_t grid_workspace_size_culled(uint32_t ntris, uint64_t box_cap, const uint32_t res[3]) {
  if (!res) return 0;
  const uint64_t nc = ncells_of(res);
  return make_layout(ntris, box_cap, nc + 1, make_plan(bits_for(nc)), 1, false, true).total;
}

int grid_count(const float* verts_soa, uint32_t nverts, const uint32_t* tris, uint32_t ntris, const float lo[3],
               const float hi[3], const uint32_t res[3], void* ws, size_t ws_bytes, uint32_t* start_out,
               uint64_t* npairs, void* stream) {
  if (!npairs) return GRID_E_INVAL;
  Build b{};
  // the count needs no pair buffers: size the layout for zero pairs
  int st = prepare_plain(b, verts_soa, nverts, tris, ntris, lo, hi, res, ws, ws_bytes, 0,
                         static_cast<hipStream_t>(stream));
  if (st) return st;
  HostCtl h{};
  st = count_phase_plain(b, &h);
  *npairs = h.npairs;
  if (st == GRID_OK && start_out && ntris > 0) {
    GB_TRY(hipMemcpyAsync(start_out, at<uint32_t>(ws, b.L.start), static_cast<size_t>(ntris) * 4,
                          hipMemcpyDeviceToDevice, b.s));
    GB_TRY(hipStreamSynchronize(b.s));
  }
  return st;
}

}  // extern "C"

namespace {

int build_plain(const float* verts_soa, uint32_t nverts, const uint32_t* tris, uint32_t ntris, const float lo[3],
                const float hi[3], const uint32_t res[3], void* ws, size_t ws_bytes, grid_out* out, hipStream_t stream,
                bool no_alloc) {
  if (!out || !out->ranges || (out->cap_pairs > 0 && (!out->cells || !out->objs))) return GRID_E_INVAL;
  Build b{};
  int st = prepare_plain(b, verts_soa, nverts, tris, ntris, lo, hi, res, ws, ws_bytes, out->cap_pairs, stream);
  if (st) return st;
  b.no_alloc = no_alloc;
  b.gs.one.out_cells = out->cells;
  b.gs.one.out_objs = out->objs;
  b.gs.one.out_ranges = out->ranges;
  // the capacity bounds every launch; the kernels read the real NO on the device
  const uint64_t cap = out->cap_pairs;
  if ((st = launch_zero(b.ws, b.L.zero_end, b.s))) return st;
  if ((st = launch_count<false>(b))) return st;
  if ((st = launch_plan<false>(b))) return st;
  int path = g_build_path;
  if (path == 2) {
    // the statistics pass: the count's totals, read back once, choose the path
    Control c;
    GB_TRY(hipMemcpyAsync(&c, at<Control>(b.ws, b.L.ctl), sizeof(Control), hipMemcpyDeviceToHost, b.s));
    GB_TRY(hipStreamSynchronize(b.s));
    path = choose_path(c.npairs, ncells_of(res));
  }
  g_last_path = path;
  if (path == 1) {
    if ((st = launch_compact(b, out))) return st;
  } else if (b.plan.sp.passes == 0) {
    if ((st = launch_expand<0, false>(b, out->cells, out->objs, cap))) return st;
  } else if (cap > 0) {
    if ((st = launch_sort<false>(b, out->cells, out->objs, cap))) return st;
  }
  if (path != 1 && (st = launch_ranges<false>(b, ncells_of(res) + 1 + cap))) return st;
  HostCtl h{};
  if ((st = read_ctl(b, &h))) return st;
  out->npairs = h.npairs;
  if (h.error) return device_error(h.error);
  if (h.npairs > 0xFFFFFFFFull) return GRID_E_OVERFLOW;
  if (h.npairs > cap) return GRID_E_CAPACITY;
  return GRID_OK;
}

}  // namespace

extern "C" {

int grid_build(const float* verts_soa, uint32_t nverts, const uint32_t* tris, uint32_t ntris, const float lo[3],
               const float hi[3], const uint32_t res[3], void* ws, size_t ws_bytes, grid_out* out, void* stream) {
  return build_plain(verts_soa, nverts, tris, ntris, lo, hi, res, ws, ws_bytes, out, static_cast<hipStream_t>(stream),
                     false);
}

int grid_build_culled(const float* verts_soa, uint32_t nverts, const uint32_t* tris, uint32_t ntris,
                      const float lo[3], const float hi[3], const uint32_t res[3], void* ws, size_t ws_bytes,
                      uint64_t box_cap, grid_out* out, uint64_t* box_npairs, void* stream) {
  if (!out || !box_npairs || !out->ranges) return GRID_E_INVAL;
  if (box_cap > 0 && (!out->cells || !out->objs)) return GRID_E_INVAL;
  Build b{};
  // the layout (expansion tiles, workspace pair buffers) is sized for the box pairs
  int st = prepare_plain(b, verts_soa, nverts, tris, ntris, lo, hi, res, ws, ws_bytes, box_cap,
                         static_cast<hipStream_t>(stream), true);
  if (st) return st;
  b.culled = true;
  b.out_cap = out->cap_pairs;
  b.gs.one.out_cells = out->cells;
  b.gs.one.out_objs = out->objs;
  b.gs.one.out_ranges = out->ranges;
  if ((st = launch_zero(b.ws, b.L.zero_end, b.s))) return st;
  if ((st = launch_count<false>(b))) return st;
  if ((st = launch_plan<false>(b))) return st;  // checks the box pairs against box_cap
  if (b.plan.sp.passes == 0 || box_cap == 0) {
    if ((st = launch_cull<0>(b, out->cells, out->objs, out->cap_pairs, box_cap))) return st;
  } else {
    if ((st = launch_sort<false>(b, out->cells, out->objs, box_cap))) return st;
  }
  if ((st = launch_ranges<false>(b, ncells_of(res) + 1 + std::min(box_cap, out->cap_pairs)))) return st;
  HostCtl h{};
  if ((st = read_ctl(b, &h))) return st;
  if (h.error) return device_error(h.error);
  *box_npairs = h.box_npairs;
  if (h.box_npairs > 0xFFFFFFFFull) return GRID_E_OVERFLOW;
  if (h.box_npairs > box_cap) {  // nothing was kept: the box pairs did not fit the workspace
    out->npairs = 0;
    return GRID_E_CAPACITY;
  }
  out->npairs = h.npairs;
  if (h.npairs > out->cap_pairs) return GRID_E_CAPACITY;
  return GRID_OK;
}

int grid_expand(const float* verts_soa, uint32_t nverts, const uint32_t* tris, uint32_t ntris, const float lo[3],
                const float hi[3], const uint32_t res[3], void* ws, size_t ws_bytes, uint32_t* cells, uint32_t* objs,
                uint64_t cap_pairs, uint64_t* npairs, void* stream) {
  if (!npairs || (cap_pairs > 0 && (!cells || !objs))) return GRID_E_INVAL;
  Build b{};
  int st = prepare_plain(b, verts_soa, nverts, tris, ntris, lo, hi, res, ws, ws_bytes, cap_pairs,
                         static_cast<hipStream_t>(stream));
  if (st) return st;
  HostCtl h{};
  st = count_phase_plain(b, &h);
  *npairs = h.npairs;
  if (st) return st;
  if (h.npairs > cap_pairs) return GRID_E_CAPACITY;
  if ((st = launch_plan<false>(b))) return st;  // the tile-owner runs of huge objects
  if ((st = launch_expand<0, false>(b, cells, objs, h.npairs))) return st;
  GB_TRY(hipStreamSynchronize(b.s));
  return GRID_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------
// The build whose workspace is a static device array (no allocation anywhere).
// ---------------------------------------------------------------------------------
// Each device that loads the library holds its own copy of this array.  In host
// code its name is only a host-side stand-in: kernels and copies get the device
// address that hipGetSymbolAddress returns for the current device.
__device__ __align__(256) unsigned char scratch[GRID_STATIC_SCRATCH_BYTES];

namespace {

// Device address of the current device's scratch array, looked up once per
// device (with that device current) and kept for later calls.
int static_scratch(void** out) {
  static std::mutex mu;
  static void* addr[64] = {};
  int dev = -1;
  GB_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return GRID_E_HIP;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    GB_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return GRID_E_HIP;
    addr[dev] = p;
  }
  *out = addr[dev];
  return GRID_OK;
}

}  // namespace

extern "C" {

int grid_build_static(const float* verts_soa, uint32_t nverts, const uint32_t* tris, uint32_t ntris,
                      const float lo[3], const float hi[3], const uint32_t res[3], grid_out* out, void* stream) {
  if (!out || check_grid(lo, hi, res) != GRID_OK) return GRID_E_INVAL;
  // the same sizing grid_build checks its workspace against, before any device work
  const size_t need = grid_workspace_size(ntris, out->cap_pairs, res);
  if (need == 0 || need > GRID_STATIC_SCRATCH_BYTES) return GRID_E_NOMEM;
  void* ws = nullptr;
  int st = static_scratch(&ws);
  if (st) return st;
  return build_plain(verts_soa, nverts, tris, ntris, lo, hi, res, ws, GRID_STATIC_SCRATCH_BYTES, out,
                     static_cast<hipStream_t>(stream), true);
}

}  // extern "C"

// ---------------------------------------------------------------------------------
// Batched builds.
// ---------------------------------------------------------------------------------
namespace {

struct BatchSetup {
  std::vector<GridDev> table;
  uint64_t ntris = 0, cap = 0, cells = 0;  // cells: the batch's cell space (sum of the grids' cells)
};

// Sort keys of a batch number the cells of all its grids in one space (each
// grid's cells follow the previous grid's), so a batch fits when its total
// cell count does not exceed 2^32.
constexpr uint64_t kMaxBatchCells = uint64_t{1} << 32;

int setup_batch(const grid_desc* grids, uint32_t ngrids, BatchSetup* bs, bool need_out) {
  if (!grids || ngrids == 0) return GRID_E_INVAL;
  bs->table.resize(ngrids);
  for (uint32_t g = 0; g < ngrids; ++g) {
    const grid_desc& d = grids[g];
    int st = check_grid(d.lo, d.hi, d.res);
    if (st) return st;
    if (d.ntris > 0 && (!d.verts_soa || !d.tris)) return GRID_E_INVAL;
    if (need_out && (!d.out.ranges || (d.out.cap_pairs > 0 && (!d.out.cells || !d.out.objs)))) return GRID_E_INVAL;
    GridDev gd = make_grid(d.verts_soa, d.nverts, d.tris, d.ntris, d.lo, d.hi, d.res);
    gd.out_cells = d.out.cells;
    gd.out_objs = d.out.objs;
    gd.out_ranges = d.out.ranges;
    gd.cap_pairs = need_out ? d.out.cap_pairs : ~uint64_t{0};
    gd.tri_base = static_cast<uint32_t>(bs->ntris);
    gd.cell_base = bs->cells;
    bs->table[g] = gd;
    bs->ntris += d.ntris;
    bs->cap += d.out.cap_pairs;
    bs->cells += ncells_of(d.res);
  }
  if (bs->ntris >= (1u << 31)) return GRID_E_INVAL;
  return GRID_OK;
}

// Largest run of grids starting at g0 whose cells fit in one 32-bit key space.
uint32_t batch_chunk(const grid_desc* grids, uint32_t ngrids, uint32_t g0) {
  uint64_t cells = 0;
  uint32_t n = 0;
  while (g0 + n < ngrids) {
    const uint64_t c = cells + ncells_of(grids[g0 + n].res);
    if (c > kMaxBatchCells) break;
    cells = c;
    ++n;
  }
  return std::max(n, 1u);
}

// The pair capacity a batched layout is made for: the sum of the grids' output
// capacities, or (builds split into a count and a resumed build) the most pairs
// the workspace holds, which both halves derive alike from the same inputs.
constexpr int64_t kCapFromDescs = -1;
constexpr int64_t kCapFromWorkspace = -2;

// Largest pair capacity whose batched layout fits in ws_bytes (-1: not even an empty one).
int64_t batch_pair_capacity(const BatchSetup& bs, uint32_t ngrids, size_t ws_bytes) {
  const Plan plan = make_plan(std::max(1u, bits_for(bs.cells)));
  auto need = [&](uint64_t cap) { return make_layout(bs.ntris, cap, bs.cells + ngrids, plan, ngrids, true).total; };
  if (need(0) > ws_bytes) return -1;
  uint64_t lo = 0, hi = uint64_t{1} << 32;  // the batch's pair indices are 32-bit
  while (hi - lo > 1) {
    const uint64_t mid = lo + (hi - lo) / 2;
    if (need(mid) <= ws_bytes) lo = mid; else hi = mid;
  }
  return static_cast<int64_t>(lo);
}

// Everything of a grid's table entry that the count reads (not its outputs).
bool same_geometry(const GridDev& a, const GridDev& b) {
  return a.verts == b.verts && a.tris == b.tris && a.nverts == b.nverts && a.ntris == b.ntris &&
         a.tri_base == b.tri_base && a.cell_base == b.cell_base && std::memcmp(a.res, b.res, sizeof a.res) == 0 &&
         std::memcmp(a.lo, b.lo, sizeof a.lo) == 0 && std::memcmp(a.inv, b.inv, sizeof a.inv) == 0;
}

// counted: when given, the table the batch was counted with (a resumed build),
// which the new table must match grid for grid before anything is enqueued.
int prepare_batched(Build& b, BatchSetup& bs, const grid_desc* grids, uint32_t ngrids, void* ws, size_t ws_bytes,
                    hipStream_t s, bool need_out, void* staging = nullptr, size_t staging_bytes = 0,
                    int64_t layout = kCapFromDescs, const GridDev* counted = nullptr) {
  int st = setup_batch(grids, ngrids, &bs, need_out);
  if (st) return st;
  if (bs.cells > kMaxBatchCells) return GRID_E_INVAL;
  if (!ws) return GRID_E_INVAL;
  if (counted) {
    for (uint32_t g = 0; g < ngrids; ++g)
      if (!same_geometry(bs.table[g], counted[g])) return GRID_E_INVAL;
  }
  uint64_t cap = bs.cap;
  if (layout == kCapFromWorkspace) {
    const int64_t c = batch_pair_capacity(bs, ngrids, ws_bytes);
    if (c < 0) return GRID_E_NOMEM;
    cap = static_cast<uint64_t>(c);
    b.layout_cap = cap;
  }
  b.ws = ws;
  b.s = s;
  b.ntris = static_cast<uint32_t>(bs.ntris);
  b.batched = true;
  b.plan = make_plan(std::max(1u, bits_for(bs.cells)));
  b.batch_cells = bs.cells;
  b.L = make_layout(bs.ntris, cap, bs.cells + ngrids, b.plan, ngrids, true);
  if (ws_bytes < b.L.total) return GRID_E_NOMEM;
  b.gs = GridSet{};
  b.gs.table = at<GridDev>(ws, b.L.table);
  b.gs.ngrids = ngrids;
  if (staging) {
    // caller-owned pinned memory: the copy stays asynchronous
    if (staging_bytes < ngrids * sizeof(GridDev)) return GRID_E_NOMEM;
    std::memcpy(staging, bs.table.data(), ngrids * sizeof(GridDev));
    GB_TRY(hipMemcpyAsync(at<GridDev>(ws, b.L.table), staging, ngrids * sizeof(GridDev), hipMemcpyHostToDevice, s));
  } else {
    // the caller synchronises before bs goes away (the count readback)
    GB_TRY(hipMemcpyAsync(at<GridDev>(ws, b.L.table), bs.table.data(), ngrids * sizeof(GridDev),
                          hipMemcpyHostToDevice, s));
  }
  return GRID_OK;
}

int count_phase_batched(Build& b, uint32_t ngrids, std::vector<uint64_t>& npairs, HostCtl* h) {
  int st = launch_zero(b.ws, b.L.zero_end, b.s);
  if (st) return st;
  if ((st = launch_count<true>(b))) return st;
  if ((st = launch_plan<true>(b))) return st;
  npairs.resize(ngrids);
  GB_TRY(hipMemcpyAsync(npairs.data(), at<uint64_t>(b.ws, b.L.npairs_out), ngrids * 8, hipMemcpyDeviceToHost, b.s));
  if ((st = read_ctl(b, h))) return st;
  if (h->error) return device_error(h->error);
  if (h->npairs > 0xFFFFFFFFull) return GRID_E_OVERFLOW;
  return GRID_OK;
}

size_t batched_ws_one(const grid_desc* grids, uint32_t ngrids, bool need_out) {
  BatchSetup bs;
  if (setup_batch(grids, ngrids, &bs, need_out)) return 0;
  return make_layout(bs.ntris, bs.cap, bs.cells + ngrids, make_plan(std::max(1u, bits_for(bs.cells))), ngrids,
                     true).total;
}

}  // namespace

extern "C" {

size_t grid_workspace_size_batched(const grid_desc* grids, uint32_t ngrids) {
  if (!grids) return 0;
  size_t need = 0;
  for (uint32_t g0 = 0; g0 < ngrids;) {
    const uint32_t n = batch_chunk(grids, ngrids, g0);
    const size_t one = batched_ws_one(grids + g0, n, false);
    if (one == 0) return 0;
    need = std::max(need, one);
    g0 += n;
  }
  return need;
}

int grid_count_batched(grid_desc* grids, uint32_t ngrids, void* ws, size_t ws_bytes, void* stream) {
  if (!grids || ngrids == 0) return GRID_E_INVAL;
  for (uint32_t g0 = 0; g0 < ngrids;) {
    const uint32_t n = batch_chunk(grids, ngrids, g0);
    Build b{};
    BatchSetup bs;
    int st = prepare_batched(b, bs, grids + g0, n, ws, ws_bytes, static_cast<hipStream_t>(stream), false);
    if (st) return st;
    std::vector<uint64_t> np;
    HostCtl h{};
    st = count_phase_batched(b, n, np, &h);
    if (st) return st;
    for (uint32_t g = 0; g < n; ++g) grids[g0 + g].out.npairs = np[g];
    g0 += n;
  }
  return GRID_OK;
}

int grid_build_batched(grid_desc* grids, uint32_t ngrids, void* ws, size_t ws_bytes, void* stream) {
  if (!grids || ngrids == 0) return GRID_E_INVAL;
  for (uint32_t g0 = 0; g0 < ngrids;) {
    const uint32_t n = batch_chunk(grids, ngrids, g0);
    Build b{};
    BatchSetup bs;
    int st = prepare_batched(b, bs, grids + g0, n, ws, ws_bytes, static_cast<hipStream_t>(stream), true);
    if (st) return st;
    std::vector<uint64_t> np;
    HostCtl h{};
    st = count_phase_batched(b, n, np, &h);
    if (st) return st;
    bool cap_ok = true;
    for (uint32_t g = 0; g < n; ++g) {
      grids[g0 + g].out.npairs = np[g];
      if (np[g] > grids[g0 + g].out.cap_pairs) cap_ok = false;
    }
    if (!cap_ok) return GRID_E_CAPACITY;
    if (h.npairs > 0) {
      if (b.plan.sp.passes == 0) return GRID_E_INVAL;  // cannot happen: the grid bits alone need a pass
      if ((st = launch_sort<true>(b, nullptr, nullptr, h.npairs))) return st;
    }
    if ((st = launch_ranges<true>(b, bs.cells + n + h.npairs))) return st;
    g0 += n;
  }
  return GRID_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------
// Building blocks: the radix sort and the scans on their own.
// ---------------------------------------------------------------------------------
namespace {

struct SortLayout {
  size_t ctl, hist, status, total;
  uint32_t ntiles;
};

SortLayout sort_layout(uint64_t n, const Plan& plan) {
  SortLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + std::max<size_t>(bytes, 1));
    return at;
  };
  L.ntiles = static_cast<uint32_t>(ceil_div(n, kSortTile));
  L.ctl = take(sizeof(Control));
  L.hist = take(4 * kRadixMax * sizeof(uint32_t));
  L.status = take(static_cast<size_t>(plan.sp.passes) * L.ntiles * (size_t{1} << plan.rb) * 8);
  L.total = o + 256;
  return L;
}

template <int RB>
int sort_arrays_rb(uint32_t* keys, uint32_t* vals, uint32_t* ka, uint32_t* va, uint64_t n, const Plan& plan,
                   void* ws, const SortLayout& L, hipStream_t s) {
  Control* ctl = at<Control>(ws, L.ctl);
  const uint64_t stride = static_cast<uint64_t>(L.ntiles) * (1u << RB);
  {
    HistArrayArgs h{};
    h.keys = keys;
    h.n = n;
    h.plan = plan.sp;
    h.hist = at<uint32_t>(ws, L.hist);
    h.sort_status = at<uint64_t>(ws, L.status);
    h.status_stride = stride;
    h.ctl = ctl;
    TraceScope ts(s, "hist_array");
    hist_array_kernel<kSortBlock, kSortK, RB><<<persistent_blocks(L.ntiles, 3), kSortBlock, 0, s>>>(h);
    GB_LAUNCHED();
  }
  uint32_t* src_k = keys;
  uint32_t* src_v = vals;
  uint32_t* dst_k = ka;
  uint32_t* dst_v = va;
  for (uint32_t p = 0; p < plan.sp.passes; ++p) {
    SortPassArgs a{};
    a.keys_in = src_k;
    a.vals_in = src_v;
    a.keys_out = dst_k;
    a.vals_out = dst_v;
    a.hist = at<uint32_t>(ws, L.hist) + p * kRadixMax;
    a.hist_copies = 1;
    a.hist_stride = 0;
    a.status = at<uint64_t>(ws, L.status) + p * stride;
    a.n = n;
    a.narrow = narrow_words(n);
    a.n_from_ctl = 0;
    a.shift = plan.sp.shift[p];
    a.width = plan.sp.width[p];
    a.counter = kCtrSort0 + p;
    a.ctl = ctl;
    TraceScope ts(s, "onesweep");
    if (a.narrow)
      onesweep_kernel<kSortBlock, kSortK, RB, kFromArrays, kToArrays, false, true>
          <<<persistent_blocks(L.ntiles, 2), kSortBlock, 0, s>>>(a);
    else
      onesweep_kernel<kSortBlock, kSortK, RB, kFromArrays, kToArrays, false, false>
          <<<persistent_blocks(L.ntiles, 2), kSortBlock, 0, s>>>(a);
    GB_LAUNCHED();
    std::swap(src_k, dst_k);
    std::swap(src_v, dst_v);
  }
  if (src_k != keys) {
    GB_TRY(hipMemcpyAsync(keys, src_k, n * 4, hipMemcpyDeviceToDevice, s));
    GB_TRY(hipMemcpyAsync(vals, src_v, n * 4, hipMemcpyDeviceToDevice, s));
  }
  return GRID_OK;
}

size_t scan_layout_status(uint64_t n) { return align_up(sizeof(Control)); }
uint32_t scan_tiles(uint64_t n) { return static_cast<uint32_t>(ceil_div(n, kScanBlock * kScanK)); }

}  // namespace

extern "C" {

size_t grid_sort_workspace_size(uint64_t n, uint32_t nbits) {
  if (nbits > 32) return 0;
  return sort_layout(n, make_plan(nbits)).total;
}

int grid_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt, uint64_t n,
                    uint32_t nbits, void* ws, size_t ws_bytes, void* stream) {
  if (nbits > 32 || n > 0xFFFFFFFFull) return GRID_E_INVAL;
  if (n == 0 || nbits == 0) return GRID_OK;
  if (!keys || !vals || !keys_alt || !vals_alt || !ws) return GRID_E_INVAL;
  const Plan plan = make_plan(nbits);
  if (!plan_ok(plan)) return GRID_E_INVAL;
  const SortLayout L = sort_layout(n, plan);
  if (ws_bytes < L.total) return GRID_E_NOMEM;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int st = launch_zero(ws, L.status, s);  // control block and histograms
  if (st) return st;
  switch (plan.rb) {
    case 8: return sort_arrays_rb<8>(keys, vals, keys_alt, vals_alt, n, plan, ws, L, s);
    case 9: return sort_arrays_rb<9>(keys, vals, keys_alt, vals_alt, n, plan, ws, L, s);
    case 10: return sort_arrays_rb<10>(keys, vals, keys_alt, vals_alt, n, plan, ws, L, s);
    case 11: return sort_arrays_rb<11>(keys, vals, keys_alt, vals_alt, n, plan, ws, L, s);
    default: return GRID_E_INVAL;
  }
}

size_t grid_scan_workspace_size(uint64_t n) {
  return scan_layout_status(n) + align_up(std::max<uint64_t>(scan_tiles(n), 1) * 8) + 256;
}

int grid_scan_u32(const uint32_t* in, const uint32_t* flags, uint32_t* out, uint64_t n, int op, void* ws,
                  size_t ws_bytes, uint64_t* total, void* stream) {
  if (!total || op < 0 || op > 2) return GRID_E_INVAL;
  *total = 0;
  if (n == 0) return GRID_OK;
  if (!in || !out || !ws || (op == GRID_SCAN_SEGMENTED_EXCLUSIVE_SUM && !flags)) return GRID_E_INVAL;
  if (ws_bytes < grid_scan_workspace_size(n)) return GRID_E_NOMEM;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t status_off = scan_layout_status(n);
  const uint32_t tiles = scan_tiles(n);
  int st = launch_zero(ws, status_off + static_cast<size_t>(tiles) * 8, s);
  if (st) return st;
  ScanArgs a{};
  a.in = in;
  a.flags = flags;
  a.out = out;
  a.n = n;
  a.status = at<uint64_t>(ws, status_off);
  a.ctl = at<Control>(ws, 0);
  if (op == GRID_SCAN_EXCLUSIVE_SUM)
    scan_kernel<kScanBlock, kScanK, ScanSum, 0><<<tiles, kScanBlock, 0, s>>>(a);
  else if (op == GRID_SCAN_INCLUSIVE_MAX)
    scan_kernel<kScanBlock, kScanK, ScanMax, 1><<<tiles, kScanBlock, 0, s>>>(a);
  else
    scan_kernel<kScanBlock, kScanK, ScanSeg, 2><<<tiles, kScanBlock, 0, s>>>(a);
  GB_LAUNCHED();
  Control c;
  GB_TRY(hipMemcpyAsync(&c, ws, sizeof(Control), hipMemcpyDeviceToHost, s));
  GB_TRY(hipStreamSynchronize(s));
  uint64_t t = c.scratch[0];
  if (op == GRID_SCAN_SEGMENTED_EXCLUSIVE_SUM) t &= ScanSeg::kSum;
  *total = t;
  return GRID_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------
// Kernel timing.
// ---------------------------------------------------------------------------------
extern "C" {

int grid_trace_enable(int on) {
  Tracer& t = tracer();
  std::lock_guard<std::mutex> lock(t.mu);
  t.on = on != 0;
  return GRID_OK;
}

int grid_trace_only(const char* name) {
  Tracer& t = tracer();
  std::lock_guard<std::mutex> lock(t.mu);
  if (!name) {
    t.only[0] = 0;
    return GRID_OK;
  }
  if (std::strlen(name) == 0 || std::strlen(name) >= sizeof(t.only)) return GRID_E_INVAL;
  std::strncpy(t.only, name, sizeof(t.only) - 1);
  t.only[sizeof(t.only) - 1] = 0;
  return GRID_OK;
}

int grid_trace_read(grid_trace_entry* out, int max_entries, int* n_entries) {
  if (!n_entries || (max_entries > 0 && !out)) return GRID_E_INVAL;
  Tracer& t = tracer();
  std::lock_guard<std::mutex> lock(t.mu);
  std::vector<grid_trace_entry> agg;
  int status = GRID_OK;
  for (TraceRec& r : t.recs) {
    float ms = 0.0f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) status = GRID_E_HIP;
    grid_trace_entry* e = nullptr;
    for (auto& x : agg)
      if (std::strncmp(x.name, r.name, sizeof(x.name)) == 0) e = &x;
    if (!e) {
      agg.push_back(grid_trace_entry{});
      e = &agg.back();
      std::strncpy(e->name, r.name, sizeof(e->name) - 1);
    }
    e->launches += 1;
    e->total_ms += ms;
    t.pool.push_back(r.a);
    t.pool.push_back(r.b);
  }
  t.recs.clear();
  *n_entries = static_cast<int>(agg.size());
  for (int i = 0; i < static_cast<int>(agg.size()) && i < max_entries; ++i) out[i] = agg[i];
  return status;
}

}  // extern "C"

// ---------------------------------------------------------------------------------
// Tuning knobs.
// ---------------------------------------------------------------------------------
extern "C" {

int grid_tune_set(const char* key, int value) {
  if (!key) return GRID_E_INVAL;
  if (std::strcmp(key, "max_digit_bits") == 0) {
    if (value < 4 || value > kMaxRadixBits) return GRID_E_INVAL;
    g_max_digit_bits = value;
    return GRID_OK;
  }
  if (std::strcmp(key, "fused_expand") == 0) {
    if (value != 0 && value != 1) return GRID_E_INVAL;
    g_fused_expand = value;
    return GRID_OK;
  }
  if (std::strcmp(key, "sort_shape") == 0) {
    if (value < 0 || value > 4) return GRID_E_INVAL;
    g_sort_shape = value;
    return GRID_OK;
  }
  if (std::strcmp(key, "small_tiles") == 0) {
    if (value != 0 && value != 1) return GRID_E_INVAL;
    g_small_tiles = value;
    return GRID_OK;
  }
  if (std::strcmp(key, "wide_lookback") == 0) {
    if (value != 0 && value != 1) return GRID_E_INVAL;
    g_wide_lookback = value;
    return GRID_OK;
  }
  if (std::strcmp(key, "per_object_pairs") == 0) {
    if (value != 0 && value != 1) return GRID_E_INVAL;
    g_per_object_pairs = value;
    return GRID_OK;
  }
  if (std::strcmp(key, "build_path") == 0) {
    if (value < 0 || value > 2) return GRID_E_INVAL;
    g_build_path = value;
    return GRID_OK;
  }
  return GRID_E_INVAL;
}

int grid_sort_plan(uint32_t nbits, uint32_t* passes, uint32_t widths[4], uint32_t* kernel_digit_bits) {
  if (nbits > 32 || !passes || !widths || !kernel_digit_bits) return GRID_E_INVAL;
  const Plan p = make_plan(nbits);
  if (!plan_ok(p) && nbits > 0) return GRID_E_INVAL;
  *passes = p.sp.passes;
  for (int i = 0; i < 4; ++i) widths[i] = i < static_cast<int>(p.sp.passes) ? p.sp.width[i] : 0;
  *kernel_digit_bits = static_cast<uint32_t>(p.rb);
  return GRID_OK;
}

int grid_tune_get(const char* key, int* value) {
  if (!key || !value) return GRID_E_INVAL;
  if (std::strcmp(key, "max_digit_bits") == 0) { *value = g_max_digit_bits; return GRID_OK; }
  if (std::strcmp(key, "fused_expand") == 0) { *value = g_fused_expand; return GRID_OK; }
  if (std::strcmp(key, "sort_shape") == 0) { *value = g_sort_shape; return GRID_OK; }
  if (std::strcmp(key, "small_tiles") == 0) { *value = g_small_tiles; return GRID_OK; }
  if (std::strcmp(key, "wide_lookback") == 0) { *value = g_wide_lookback; return GRID_OK; }
  if (std::strcmp(key, "per_object_pairs") == 0) { *value = g_per_object_pairs; return GRID_OK; }
  if (std::strcmp(key, "build_path") == 0) { *value = g_build_path; return GRID_OK; }
  if (std::strcmp(key, "last_path") == 0) { *value = g_last_path; return GRID_OK; }
  return GRID_E_INVAL;
}

}  // extern "C"

// ---------------------------------------------------------------------------------
// Batched builds without a host readback.
// ---------------------------------------------------------------------------------
extern "C" {

size_t grid_batch_staging_size(uint32_t ngrids) { return static_cast<size_t>(ngrids) * sizeof(GridDev); }

int grid_build_batched_async(const grid_desc* grids, uint32_t ngrids, void* ws, size_t ws_bytes, void* host_staging,
                             size_t staging_bytes, void* stream) {
  if (!grids || ngrids == 0 || !host_staging) return GRID_E_INVAL;
  if (batch_chunk(grids, ngrids, 0) != ngrids) return GRID_E_INVAL;  // packed keys must fit in 32 bits
  Build b{};
  BatchSetup bs;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int st = prepare_batched(b, bs, grids, ngrids, ws, ws_bytes, s, true, host_staging, staging_bytes);
  if (st) return st;
  if ((st = launch_zero(b.ws, b.L.zero_end, s))) return st;
  if ((st = launch_count<true>(b))) return st;
  if ((st = launch_plan<true>(b))) return st;
  // sizes on the host are the capacities; the kernels read the true counts
  if (bs.cap > 0) {
    if (b.plan.sp.passes == 0) return GRID_E_INVAL;
    if ((st = launch_sort<true>(b, nullptr, nullptr, bs.cap))) return st;
  }
  return launch_ranges<true>(b, bs.cells + ngrids + bs.cap);
}

int grid_count_batched_async(const grid_desc* grids, uint32_t ngrids, void* ws, size_t ws_bytes, void* host_staging,
                             size_t staging_bytes, uint64_t* counts_host, uint64_t* pair_cap, void* stream) {
  if (!grids || ngrids == 0 || !host_staging || !counts_host) return GRID_E_INVAL;
  if (batch_chunk(grids, ngrids, 0) != ngrids) return GRID_E_INVAL;  // packed keys must fit in 32 bits
  const size_t half = grid_batch_staging_size(ngrids);
  if (staging_bytes < 2 * half) return GRID_E_NOMEM;
  Build b{};
  BatchSetup bs;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // outputs are not known yet: the count checks only the workspace's capacity
  int st = prepare_batched(b, bs, grids, ngrids, ws, ws_bytes, s, false, host_staging, half, kCapFromWorkspace);
  if (st) return st;
  if (pair_cap) *pair_cap = b.layout_cap;
  if ((st = launch_zero(b.ws, b.L.zero_end, s))) return st;
  if ((st = launch_count<true>(b))) return st;
  if ((st = launch_plan<true>(b))) return st;
  GB_TRY(hipMemcpyAsync(counts_host, at<uint64_t>(b.ws, b.L.npairs_out), (ngrids + 1) * sizeof(uint64_t),
                        hipMemcpyDeviceToHost, s));
  return GRID_OK;
}

int grid_build_batched_counted(const grid_desc* grids, uint32_t ngrids, void* ws, size_t ws_bytes, void* host_staging,
                               size_t staging_bytes, void* stream) {
  if (!grids || ngrids == 0 || !host_staging) return GRID_E_INVAL;
  if (batch_chunk(grids, ngrids, 0) != ngrids) return GRID_E_INVAL;
  const size_t half = grid_batch_staging_size(ngrids);
  if (staging_bytes < 2 * half) return GRID_E_NOMEM;
  Build b{};
  BatchSetup bs;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // the first half of the staging still holds the table the batch was counted with
  int st = prepare_batched(b, bs, grids, ngrids, ws, ws_bytes, s, true, static_cast<char*>(host_staging) + half, half,
                           kCapFromWorkspace, static_cast<const GridDev*>(host_staging));
  if (st) return st;
  // launch sizes: the outputs' capacities (the kernels read the true counts);
  // a grid beyond its capacity is caught by the sink kernel, pairs beyond the
  // workspace by the count's plan, and either way no kernel writes anything
  const uint64_t n = std::min<uint64_t>(bs.cap, b.layout_cap);
  if (n > 0) {
    if (b.plan.sp.passes == 0) return GRID_E_INVAL;
    if ((st = launch_sort<true>(b, nullptr, nullptr, n))) return st;
  } else if ((st = launch_sink(b))) {
    return st;
  }
  return launch_ranges<true>(b, bs.cells + ngrids + n);
}

int grid_workspace_status(const void* ws, uint64_t* npairs_total, void* stream) {
  if (!ws) return GRID_E_INVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Control c;  // the control block opens every workspace
  GB_TRY(hipMemcpyAsync(&c, ws, sizeof(Control), hipMemcpyDeviceToHost, s));
  GB_TRY(hipStreamSynchronize(s));
  if (npairs_total) *npairs_total = c.npairs;
  if (c.error) return device_error(c.error);
  if (c.cap_flag & 2u) return GRID_E_OVERFLOW;
  if (c.cap_flag & 1u) return GRID_E_CAPACITY;
  return GRID_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------
// Ray casting over a built grid.
// ---------------------------------------------------------------------------------
extern "C" {

int grid_raycast(const float* verts_soa, uint32_t nverts, const uint32_t* tris, uint32_t ntris, const float lo[3],
                 const float hi[3], const uint32_t res[3], const uint32_t* ranges, const uint32_t* objs,
                 const float* rays, uint32_t nrays, float tmax, float* hit_t, uint32_t* hit_obj, void* stream) {
  int st = check_grid(lo, hi, res);
  if (st) return st;
  if (nrays == 0) return GRID_OK;
  if (!rays || !hit_t || !hit_obj || !ranges || (ntris > 0 && (!verts_soa || !tris))) return GRID_E_INVAL;
  if (!(tmax >= 0.0f)) return GRID_E_INVAL;
  RaycastArgs a{};
  a.g = make_grid(verts_soa, nverts, tris, ntris, lo, hi, res);
  for (int k = 0; k < 3; ++k) a.hi[k] = hi[k];
  a.ranges = ranges;
  a.objs = objs;
  a.rays = rays;
  a.nrays = nrays;
  a.tmax = tmax;
  a.hit_t = hit_t;
  a.hit_obj = hit_obj;
  hipStream_t s = static_cast<hipStream_t>(stream);
  TraceScope ts(s, "raycast");
  raycast_kernel<256><<<static_cast<uint32_t>(ceil_div(nrays, 256)), 256, 0, s>>>(a);
  GB_LAUNCHED();
  return GRID_OK;
}

}  // extern "C"
