// Removal of false intersections: a pair <t, c> of triangle t's cell box is
// kept only when the triangle touches cell c (the fix the Test Results section
// proposes for scenes of long thin diagonal triangles, Hairball, and the
// Conclusions list as future work).  The test is a separating-axis test in
// grid coordinates, u = (p - lo) * inv, where cell (x, y, z) is the unit box
// [x, x+1] x [y, y+1] x [z, z+1]; the axes are the triangle's normal and the
// nine cross products of its edges with the grid axes (the box's own face
// axes cannot separate a cell of the triangle's box).  Every operation is one
// FP32 operation in a fixed order (no contraction), and each cell is widened
// by 1/64 of a cell on every side, so rounding may keep a pair the exact test
// would drop but never drops one it would keep.  A triangle keeps its whole
// box when a vertex lies outside [0, res] on some axis (or is NaN), or when
// its box holds at most two cells (it touches them all).
//
// The culled expansion tests each box pair, keeps the survivors in object
// order (a tile scan plus a decoupled look-back over tiles), and feeds the
// kept count to the radix sort and the ranges.
#pragma once

#include "ranges.hpp"

namespace gb {

constexpr float kOverlapMargin = 1.0f / 64.0f;  // cells

GB_DEV float dot3f(const float a[3], const float b[3]) {
  float s = __fmul_rn(a[0], b[0]);
  s = __fadd_rn(s, __fmul_rn(a[1], b[1]));
  s = __fadd_rn(s, __fmul_rn(a[2], b[2]));
  return s;
}

// The interval [below, above] that the projection c = a . corner of a
// separated cell's lower corner must leave: axis a separates the triangle
// from the widened cell with lower corner b when a . b > above or a . b < below.
GB_DEV void axis_bounds(const float a[3], const float u[3][3], float& above, float& below) {
  const float p0 = dot3f(a, u[0]), p1 = dot3f(a, u[1]), p2 = dot3f(a, u[2]);
  const float tmin = fminf(fminf(p0, p1), p2);
  const float tmax = fmaxf(fmaxf(p0, p1), p2);
  float lo_off = __fadd_rn(fminf(a[0], 0.0f), fminf(a[1], 0.0f));
  lo_off = __fadd_rn(lo_off, fminf(a[2], 0.0f));
  float hi_off = __fadd_rn(fmaxf(a[0], 0.0f), fmaxf(a[1], 0.0f));
  hi_off = __fadd_rn(hi_off, fmaxf(a[2], 0.0f));
  float l1 = __fadd_rn(fabsf(a[0]), fabsf(a[1]));
  l1 = __fadd_rn(l1, fabsf(a[2]));
  const float mg = __fmul_rn(kOverlapMargin, l1);
  above = __fsub_rn(__fadd_rn(tmax, mg), lo_off);
  below = __fsub_rn(__fsub_rn(tmin, mg), hi_off);
}

// A triangle's thirteen axes with their bounds.  The nine edge axes each have
// a zero component, which is left out of their products with a cell corner:
// that changes at most the sign of a zero, and no comparison sees the sign.
struct CullAxes {
  float n[3], n_above, n_below;
  float e[9][2], e_above[9], e_below[9];  // edge axis i * 3 + axis: its two non-zero components
};

GB_DEV void cull_axes(const float u[3][3], CullAxes& c) {
  float e[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int a = 0; a < 3; ++a) e[i][a] = __fsub_rn(u[(i + 1) % 3][a], u[i][a]);
  c.n[0] = __fsub_rn(__fmul_rn(e[0][1], e[1][2]), __fmul_rn(e[0][2], e[1][1]));
  c.n[1] = __fsub_rn(__fmul_rn(e[0][2], e[1][0]), __fmul_rn(e[0][0], e[1][2]));
  c.n[2] = __fsub_rn(__fmul_rn(e[0][0], e[1][1]), __fmul_rn(e[0][1], e[1][0]));
  axis_bounds(c.n, u, c.n_above, c.n_below);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float ax[3] = {0.0f, e[i][2], -e[i][1]};   // e x (1, 0, 0)
    const float ay[3] = {-e[i][2], 0.0f, e[i][0]};   // e x (0, 1, 0)
    const float az[3] = {e[i][1], -e[i][0], 0.0f};   // e x (0, 0, 1)
    axis_bounds(ax, u, c.e_above[3 * i + 0], c.e_below[3 * i + 0]);
    axis_bounds(ay, u, c.e_above[3 * i + 1], c.e_below[3 * i + 1]);
    axis_bounds(az, u, c.e_above[3 * i + 2], c.e_below[3 * i + 2]);
    c.e[3 * i + 0][0] = ax[1]; c.e[3 * i + 0][1] = ax[2];   // (y, z)
    c.e[3 * i + 1][0] = ay[0]; c.e[3 * i + 1][1] = ay[2];   // (x, z)
    c.e[3 * i + 2][0] = az[0]; c.e[3 * i + 2][1] = az[1];   // (x, y)
  }
}

// True when the triangle touches the widened cell with lower corner (x, y, z).
GB_DEV bool cull_touches(const CullAxes& c, float x, float y, float z) {
  const float b[3] = {x, y, z};
  const float cn = dot3f(c.n, b);
  // every axis is evaluated (no early exit): the result is the same, and the
  // wave does not branch per axis
  bool sep = (cn > c.n_above) | (cn < c.n_below);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float cx = __fadd_rn(__fmul_rn(c.e[3 * i + 0][0], y), __fmul_rn(c.e[3 * i + 0][1], z));
    const float cy = __fadd_rn(__fmul_rn(c.e[3 * i + 1][0], x), __fmul_rn(c.e[3 * i + 1][1], z));
    const float cz = __fadd_rn(__fmul_rn(c.e[3 * i + 2][0], x), __fmul_rn(c.e[3 * i + 2][1], y));
    sep = sep | (cx > c.e_above[3 * i + 0]) | (cx < c.e_below[3 * i + 0]);
    sep = sep | (cy > c.e_above[3 * i + 1]) | (cy < c.e_below[3 * i + 1]);
    sep = sep | (cz > c.e_above[3 * i + 2]) | (cz < c.e_below[3 * i + 2]);
  }
  return !sep;
}

// Grid coordinates of triangle t's vertices; true when the test applies (every
// coordinate finite and inside [0, res]).
GB_DEV bool cull_grid_coords(const GridDev& G, uint32_t t, float u[3][3]) {
  const uint32_t* tri = G.tris + 3 * static_cast<uint64_t>(t);
  bool inside = true;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const uint32_t vi = tri[j];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float p = G.verts[static_cast<uint64_t>(a) * G.nverts + vi];
      u[j][a] = __fmul_rn(__fsub_rn(p, G.lo[a]), G.inv[a]);
      inside = inside && u[j][a] >= 0.0f && u[j][a] <= static_cast<float>(G.res[a]);
    }
  }
  return inside;
}

struct CullArgs {
  ExpandOutArgs o;          // the expansion's arguments; cells/objs receive the kept pairs
  uint64_t dest_cap;        // entries cells/objs hold
  uint64_t* status;         // [expansion tiles] look-back words of the kept counts (zeroed)
};

// Digit histograms of the kept keys among a thread's K consecutive items (runs
// of equal digits added once).
template <int K, int RB>
GB_DEV void hist_runs_kept(const SortPlan& plan, const uint32_t (&keys)[K], uint32_t keep, uint32_t* s_hist) {
  constexpr int R = 1 << RB;
  for (uint32_t p = 0; p < plan.passes; ++p) {
    const uint32_t sh = plan.shift[p], dm = (1u << plan.width[p]) - 1u;
    uint32_t cur = 0, cnt = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if ((keep >> k) & 1u) {
        const uint32_t d = (keys[k] >> sh) & dm;
        if (cnt != 0 && d != cur) {
          atomicAdd(&s_hist[p * R + cur], cnt);
          cnt = 0;
        }
        cur = d;
        ++cnt;
      }
    }
    if (cnt != 0) atomicAdd(&s_hist[p * R + cur], cnt);
  }
}

// The culled expansion (plain builds): box pairs of expansion tile e are
// tested and the kept ones written, in object order, at their rank among all
// kept pairs; with RB > 0 also the kept keys' digit histograms and the radix
// passes' cleared look-back words.  The last tile writes the kept total.
template <int Block, int K, int RB>
__global__ __launch_bounds__(Block, 4) void expand_cull_kernel(CullArgs a) {
  constexpr int N = Block * K;
  constexpr int R = RB > 0 ? 1 << RB : 1;
  static_assert(K <= 32, "a thread's keep flags fit one word");
  __shared__ uint32_t s_owner[padded(N)];
  __shared__ uint32_t s_hist[RB > 0 ? 4 * R : 1];
  __shared__ uint32_t s_wtot[Block / kWave];
  __shared__ uint64_t s_prefix;
  __shared__ uint32_t s_tile;
  if (build_failed(a.o.ctl)) return;
  const uint64_t npairs = a.o.ctl->npairs;  // box pairs
  const uint32_t ntiles = static_cast<uint32_t>((npairs + N - 1) / N);
  if constexpr (RB > 0) {
    clear_status<Block>(a.o.clear, npairs);
    for (int i = threadIdx.x; i < 4 * R; i += Block) s_hist[i] = 0;
  }
  const GridDev& G = a.o.ex.gs.one;
  const uint32_t tid = threadIdx.x;
  while (true) {
    const uint32_t tile = next_tile(&a.o.ctl->tile_counter[kCtrExpand], &s_tile);
    if (tile >= ntiles) break;
    uint32_t keys[K], vals[K], xyz[K];
    const uint32_t n =
        expand_tile<Block, K, false, kBlocked, true>(a.o.ex, tile, npairs, ntiles, s_owner, s_wtot, keys, vals, xyz);
    // the overlap test, with the axes of the current object kept across its items
    uint32_t keep = 0;
    uint32_t cur = 0xFFFFFFFFu;
    bool test = false;
    CullAxes ax;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (tid * K + k < n) {
        if (vals[k] != cur) {
          cur = vals[k];
          const Box b = unpack_box(a.o.ex.box[cur]);
          float u[3][3];
          test = b.m[0] * b.m[1] * b.m[2] > 2u && cull_grid_coords(G, cur, u);
          if (test) cull_axes(u, ax);
        }
        const float x = static_cast<float>(xyz[k] & 1023u);
        const float y = static_cast<float>((xyz[k] >> 10) & 1023u);
        const float z = static_cast<float>(xyz[k] >> 20);
        if (!test || cull_touches(ax, x, y, z)) keep |= 1u << k;
      }
    }
    // rank of each kept item among all kept items: thread, then tile, then look-back
    uint32_t ttot;
    const uint32_t texcl = block_exclusive_sum<Block>(static_cast<uint32_t>(__builtin_popcount(keep)), s_wtot, ttot);
    if (tid < kWave) {
      const uint64_t p = lookback_wave(a.status, tile, ttot);
      if (tid == 0) {
        s_prefix = p;
        if (tile == ntiles - 1) a.o.ctl->kept = p + ttot;
      }
    }
    __syncthreads();
    uint64_t pos = s_prefix + texcl;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if ((keep >> k) & 1u) {
        if (pos < a.dest_cap) {
          a.o.cells[pos] = keys[k];
          a.o.objs[pos] = vals[k];
        }
        ++pos;
      }
    }
    if constexpr (RB > 0) hist_runs_kept<K, RB>(a.o.plan, keys, keep, s_hist);
    __syncthreads();  // s_prefix and the tile's LDS are reused by the next tile
  }
  if constexpr (RB > 0) flush_hist<RB, Block>(a.o.plan, a.o.hist, s_hist);
}

// After the culled expansion: the kept count becomes the build's pair count
// (the box count is kept beside it), the capacity is checked against it, and
// the one grid's range plan is sized for it.
struct CullCommitArgs {
  Control* ctl;
  GridRun* run;
  uint64_t out_cap;
  uint64_t ncells;
  uint32_t merge_tile;
};

__global__ void cull_commit_kernel(CullCommitArgs a) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Control* c = a.ctl;
  if (c->error) return;
  const uint64_t box = c->npairs;
  const uint64_t kept = box == 0 ? 0 : c->kept;  // no tile ran when there is no pair
  if (c->cap_flag) {  // the box pairs did not fit: nothing was kept
    c->box_npairs = box;
    return;
  }
  c->box_npairs = box;
  c->npairs = kept;
  if (kept > a.out_cap) c->cap_flag |= 1u;
  a.run[0].npairs = kept;
  const uint32_t mt = static_cast<uint32_t>((a.ncells + 1 + kept + a.merge_tile - 1) / a.merge_tile);
  a.run[0].mtiles = mt;
  a.run[1].mtile_base = mt;
}

}  // namespace gb
