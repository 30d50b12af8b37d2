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
// Each triangle's axes and bounds are computed once, by one thread, into a
// record of the workspace; the culled expansion then tests each box pair
// against its triangle's record, keeps the survivors in object order (a tile
// scan plus a decoupled look-back over tiles), and feeds the kept count to the
// radix sort and the ranges.
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

// A triangle's record in the workspace, in 16-byte groups that the culled
// expansion loads one at a time: the normal axis with its bounds and whether
// the test applies, then per edge its three axes (edge x X, edge x Y, edge x Z:
// their two non-zero components, for (y, z), (x, z) and (x, y)) and bounds.
struct CullEdge {
  float c[3][2];
  float above[3], below[3];
};

struct alignas(16) CullRecord {
  float n[3], n_above;
  float n_below;
  uint32_t test;            // 1: the test applies (else only this word is written)
  float pad[2];
  CullEdge e[3];
};
static_assert(sizeof(CullRecord) == 176, "eleven 16-byte words");
constexpr int kRecWords4 = 11;

// The normal axis separates the widened cell with lower corner (x, y, z).
GB_DEV bool normal_separates(const float n[3], float above, float below, float x, float y, float z) {
  const float b[3] = {x, y, z};
  const float cn = dot3f(n, b);
  return (cn > above) | (cn < below);
}

// One of edge e's three axes separates the widened cell with lower corner (x, y, z).
GB_DEV bool edge_separates(const CullEdge& e, float x, float y, float z) {
  const float cx = __fadd_rn(__fmul_rn(e.c[0][0], y), __fmul_rn(e.c[0][1], z));
  const float cy = __fadd_rn(__fmul_rn(e.c[1][0], x), __fmul_rn(e.c[1][1], z));
  const float cz = __fadd_rn(__fmul_rn(e.c[2][0], x), __fmul_rn(e.c[2][1], y));
  return (cx > e.above[0]) | (cx < e.below[0]) | (cy > e.above[1]) | (cy < e.below[1]) | (cz > e.above[2]) |
         (cz < e.below[2]);
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

struct CullRecordArgs {
  GridDev grid;
  const uint64_t* box;      // [ntris] packed cell boxes of the count
  CullRecord* rec;          // [ntris]
  uint32_t ntris;
  const Control* ctl;
};

// One thread per triangle (after the count, which has checked every vertex index).
template <int Block>
__global__ __launch_bounds__(Block) void cull_record_kernel(CullRecordArgs a) {
  if (build_failed(a.ctl)) return;
  const uint32_t stride = gridDim.x * Block;
  for (uint32_t t = blockIdx.x * Block + threadIdx.x; t < a.ntris; t += stride) {
    const Box b = unpack_box(a.box[t]);
    float u[3][3];
    const bool test = b.m[0] * b.m[1] * b.m[2] > 2u && cull_grid_coords(a.grid, t, u);
    CullRecord& r = a.rec[t];
    if (test) {
      CullAxes ax;
      cull_axes(u, ax);
      r.n[0] = ax.n[0];
      r.n[1] = ax.n[1];
      r.n[2] = ax.n[2];
      r.n_above = ax.n_above;
      r.n_below = ax.n_below;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          r.e[i].c[j][0] = ax.e[3 * i + j][0];
          r.e[i].c[j][1] = ax.e[3 * i + j][1];
          r.e[i].above[j] = ax.e_above[3 * i + j];
          r.e[i].below[j] = ax.e_below[3 * i + j];
        }
    }
    r.test = test ? 1u : 0u;
  }
}

struct CullArgs {
  ExpandOutArgs o;          // the expansion's arguments; cells/objs receive the kept pairs
  const float4* rec;        // [ntris * 11] each triangle's CullRecord
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
// Six waves per SIMD (80 VGPRs; three values spill, reloaded once per tile,
// outside the test) measured fastest: five waves without spills, or eight
// with many, were slower.
template <int Block, int K, int RB>
__global__ __launch_bounds__(Block, 6) void expand_cull_kernel(CullArgs a) {
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
  const uint32_t tid = threadIdx.x;
  while (true) {
    const uint32_t tile = next_tile(&a.o.ctl->tile_counter[kCtrExpand], &s_tile);
    if (tile >= ntiles) break;
    uint32_t keys[K], vals[K], xyz[K];
    const uint32_t n =
        expand_tile<Block, K, false, kBlocked, true>(a.o.ex, tile, npairs, ntiles, s_owner, s_wtot, keys, vals, xyz);
    // the overlap test in four passes over the thread's items (the normal axis,
    // then each edge's three axes), each loading only its part of the current
    // object's record; an item is dropped when some axis separates it
    uint32_t valid = 0, tested = 0, sep = 0;
    {
      uint32_t cur = 0xFFFFFFFFu;
      bool test = false;
      float nv[3] = {0.0f, 0.0f, 0.0f}, na = 0.0f, nb = 0.0f;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (tid * K + k < n) {
          valid |= 1u << k;
          if (vals[k] != cur) {
            cur = vals[k];
            const float4 g0 = a.rec[static_cast<uint64_t>(cur) * kRecWords4];
            const float4 g1 = a.rec[static_cast<uint64_t>(cur) * kRecWords4 + 1];
            nv[0] = g0.x;
            nv[1] = g0.y;
            nv[2] = g0.z;
            na = g0.w;
            nb = g1.x;
            test = __float_as_uint(g1.y) != 0u;
          }
          if (test) {
            tested |= 1u << k;
            if (normal_separates(nv, na, nb, static_cast<float>(xyz[k] & 1023u),
                                 static_cast<float>((xyz[k] >> 10) & 1023u), static_cast<float>(xyz[k] >> 20)))
              sep |= 1u << k;
          }
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      uint32_t cur = 0xFFFFFFFFu;
      CullEdge e{};
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if ((tested >> k) & 1u) {
          if (vals[k] != cur) {
            cur = vals[k];
            const float4* g = a.rec + static_cast<uint64_t>(cur) * kRecWords4 + 2 + 3 * i;
            const float4 g0 = g[0], g1 = g[1], g2 = g[2];
            e.c[0][0] = g0.x;
            e.c[0][1] = g0.y;
            e.c[1][0] = g0.z;
            e.c[1][1] = g0.w;
            e.c[2][0] = g1.x;
            e.c[2][1] = g1.y;
            e.above[0] = g1.z;
            e.above[1] = g1.w;
            e.above[2] = g2.x;
            e.below[0] = g2.y;
            e.below[1] = g2.z;
            e.below[2] = g2.w;
          }
          if (edge_separates(e, static_cast<float>(xyz[k] & 1023u), static_cast<float>((xyz[k] >> 10) & 1023u),
                             static_cast<float>(xyz[k] >> 20)))
            sep |= 1u << k;
        }
      }
    }
    const uint32_t keep = valid & ~sep;
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
