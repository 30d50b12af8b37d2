// The kernels of one build: count+scan, expansion, radix-sort passes and
// per-cell ranges.  Every kernel that runs after the count reads the pair count
// from device memory, so a whole build is a fixed sequence of launches.
#pragma once

#include "common.hpp"
#include "grid.hpp"
#include "tiles.hpp"

namespace gb {

enum CounterSlot : uint32_t {
  kCtrCount = 0, kCtrHist = 1, kCtrExpand = 2, kCtrSort0 = 3,  // sort passes use 3..6
  kCtrSplit = 8, kCtrRanges = 9, kCtrScan = 10, kCtrPlan = 11,
};

// ---------------------------------------------------------------------------
// Grid lookup.  Plain builds carry their one grid in the kernel arguments;
// batched builds read a device table and find the grid of a triangle from the
// grids' first-triangle indices.
// ---------------------------------------------------------------------------
struct GridSet {
  GridDev one;              // plain builds
  const GridDev* table;     // batched builds (device)
  uint32_t ngrids;          // batched: sort key = the grid's cell_base + its local cell id
};

template <bool Batched>
GB_DEV const GridDev& grid_at(const GridSet& s, uint32_t g) {
  if constexpr (Batched) return s.table[g]; else return s.one;
}

// Smallest g with tri_base[g + 1] > t, starting from a lower bound g.
template <bool Batched>
GB_DEV uint32_t grid_of_tri(const GridSet& s, uint32_t t, uint32_t g) {
  if constexpr (Batched) {
    while (g + 1 < s.ngrids && s.table[g + 1].tri_base <= t) ++g;
    return g;
  } else {
    return 0;
  }
}

// The look-back words the radix passes will use, cleared by the kernel that
// runs before them: pass p uses ceil(NO / tile[p]) * radix[p] words from
// status + p * stride.
struct StatusClear {
  uint64_t* status;
  uint64_t stride;
  uint32_t tile[4];
  uint32_t radix[4];
  uint32_t passes;
};

template <int Block>
GB_DEV void clear_status(const StatusClear& c, uint64_t npairs) {
  const uint64_t first = static_cast<uint64_t>(blockIdx.x) * Block + threadIdx.x;
  const uint64_t step = static_cast<uint64_t>(gridDim.x) * Block;
  for (uint32_t p = 0; p < c.passes; ++p) {
    const uint64_t words = ((npairs + c.tile[p] - 1) / c.tile[p]) * c.radix[p];
    uint64_t* st = c.status + p * c.stride;
    for (uint64_t i = first; i < words; i += step) st[i] = 0;
  }
}

// ---------------------------------------------------------------------------
// CountCells + ExclusiveSum (one pass, decoupled look-back).
// ---------------------------------------------------------------------------
struct CountArgs {
  GridSet gs;
  uint32_t ntris;           // total triangles (all grids)
  uint32_t* start;          // [ntris] exclusive pair offsets (global)
  uint64_t* box;            // [ntris] packed cell boxes
  uint32_t* tfo;            // [ntfo] owner of the first pair of each expansion tile
  uint32_t* tfg;            // [ntfo] batched: grid of that owner
  uint32_t ntfo;
  uint32_t tile_shift;      // log2 of the expansion tile size (one tfo entry per expansion tile)
  uint64_t* status;         // [count tiles] look-back words
  uint4* tfo_work;          // [tfo_work_cap] (object, grid, first entry, last entry) runs left for the plan kernel
  uint32_t tfo_work_cap;
  Control* ctl;
};


// Grid of triangle t (largest g with tri_base[g] <= t), found by one whole
// wave: each level probes 64 evenly spaced grids of the remaining range at
// once, so 512 grids take two dependent loads.  Every lane must pass the same
// t; all lanes get the answer.
GB_DEV uint32_t grid_of_tri_wave(const GridSet& s, uint32_t t) {
  uint32_t lo = 0, end = s.ngrids;  // answer in [lo, end); tri_base[0] = 0 <= t
  const uint32_t lane = lane_id();
  while (end - lo > 1) {
    const uint32_t step = (end - lo + kWave - 1) / kWave;
    const uint32_t g = lo + lane * step;
    const bool le = g < end && s.table[g].tri_base <= t;
    const uint32_t c = static_cast<uint32_t>(__popcll(ballot(le)));  // probes are monotone: lanes 0..c-1
    lo += (c - 1) * step;
    end = lo + step < end ? lo + step : end;
  }
  return lo;
}

// Where count_items finds a triangle's grid: the plain build's one grid, the
// one grid of a batched tile (loaded once, held in scalar registers), or a
// per-triangle walk for batched tiles that straddle grids.
enum CountMode : int { kCountPlain = 0, kCountOneGrid = 1, kCountPerItem = 2 };

// CountCells for the tile's triangles base + k * Block + tid: writes each box
// and leaves the counts in s_val (striped order).
template <int Block, int K, int Mode>
GB_DEV void count_items(const CountArgs& a, const GridDev& G0, uint64_t base, uint32_t* s_val, uint32_t g0 = 0) {
  const uint32_t tid = threadIdx.x;
  uint32_t g = g0;  // kCountPerItem: the grid of the tile's first triangle, walked forward per item

  // all index loads, then all vertex loads, then the arithmetic
  uint32_t gi[K], idx[K][3];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint64_t t = base + static_cast<uint64_t>(k) * Block + tid;
    const uint32_t tc = static_cast<uint32_t>(t < a.ntris ? t : a.ntris - 1);
    if constexpr (Mode == kCountPerItem) g = grid_of_tri<true>(a.gs, tc, g);
    gi[k] = g;
    const GridDev& G = Mode == kCountPerItem ? a.gs.table[g] : G0;
    const uint32_t* tri = G.tris + 3 * static_cast<uint64_t>(tc - G.tri_base);
    idx[k][0] = tri[0];
    idx[k][1] = tri[1];
    idx[k][2] = tri[2];
  }
  float p[K][3][3];
  bool bad[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const GridDev& G = Mode == kCountPerItem ? a.gs.table[gi[k]] : G0;
    bad[k] = idx[k][0] >= G.nverts || idx[k][1] >= G.nverts || idx[k][2] >= G.nverts;
    // a triangle of a soup lists three consecutive vertices: each coordinate's
    // three values are then one 12-byte load instead of three (plain builds; the
    // batched count has no registers to spare for it)
    const bool seq = Mode == kCountPlain && !bad[k] && idx[k][1] == idx[k][0] + 1u && idx[k][2] == idx[k][0] + 2u;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const float* v = G.verts + static_cast<uint64_t>(ax) * G.nverts;
      if (seq) {
        const float3 q = *reinterpret_cast<const float3*>(v + idx[k][0]);
        p[k][ax][0] = q.x;
        p[k][ax][1] = q.y;
        p[k][ax][2] = q.z;
      } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) p[k][ax][c] = bad[k] ? 0.0f : v[idx[k][c]];  // no load for a bad index
      }
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint64_t t = base + static_cast<uint64_t>(k) * Block + tid;
    uint32_t cnt = 0;
    if (t < a.ntris) {
      const GridDev& G = Mode == kCountPerItem ? a.gs.table[gi[k]] : G0;
      uint64_t packed = 0;
      cnt = 1;
      if (bad[k]) {
        atomicOr(&a.ctl->error, kErrBadIndex);
      } else {
        uint32_t lo[3], m[3];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          const float pmin = fminf(fminf(p[k][ax][0], p[k][ax][1]), p[k][ax][2]);
          const float pmax = fmaxf(fmaxf(p[k][ax][0], p[k][ax][1]), p[k][ax][2]);
          const uint32_t cl = cell_coord(pmin, G.lo[ax], G.inv[ax], G.res[ax] - 1);
          const uint32_t ch = cell_coord(pmax, G.lo[ax], G.inv[ax], G.res[ax] - 1);
          lo[ax] = cl;
          m[ax] = ch - cl + 1;
        }
        cnt = m[0] * m[1] * m[2];
        packed = pack_box(lo, m);
      }
      a.box[t] = packed;
    }
    s_val[pad32(k * Block + tid)] = cnt;
  }
}

template <int Block, int K, bool Batched>
__global__ __launch_bounds__(Block) void count_kernel(CountArgs a) {
  constexpr int Tile = Block * K;
  __shared__ uint32_t s_val[padded(Tile)];
  __shared__ uint64_t s_wtot[Block / kWave];
  __shared__ uint64_t s_prefix;
  __shared__ uint32_t s_tile;
  const uint32_t tile = next_tile(&a.ctl->tile_counter[kCtrCount], &s_tile);
  const uint32_t tid = threadIdx.x;
  const uint64_t base = static_cast<uint64_t>(tile) * Tile;
  const uint32_t ntiles = (a.ntris + Tile - 1) / Tile;
  // batched: the grid of the tile's first triangle, and whether every
  // triangle of the tile lies in it (the same for the whole workgroup)
  uint32_t gl = 0;
  bool one = true;
  if constexpr (Batched) {
    const uint32_t t0 = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(base < a.ntris ? base : a.ntris - 1));
    const uint64_t e = base + Tile < a.ntris ? base + Tile : a.ntris;
    const uint32_t t1 = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(e - 1));
    gl = __builtin_amdgcn_readfirstlane(grid_of_tri_wave(a.gs, t0));
    one = gl + 1 >= a.gs.ngrids || a.gs.table[gl + 1].tri_base > t1;
    if (one) {
      const GridDev G = a.gs.table[gl];
      count_items<Block, K, kCountOneGrid>(a, G, base, s_val);
    } else {
      count_items<Block, K, kCountPerItem>(a, a.gs.table[gl], base, s_val, gl);
    }
  } else {
    count_items<Block, K, kCountPlain>(a, a.gs.one, base, s_val);
  }
  __syncthreads();

  uint32_t mine[K];
  uint64_t sum = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    mine[k] = s_val[pad32(tid * K + k)];
    sum += mine[k];
  }
  uint64_t total;
  uint64_t excl = block_exclusive_sum64<Block>(sum, s_wtot, total);
  if (tid < kWave) {
    const uint64_t p = lookback_wave(a.status, tile, total);
    if (tid == 0) {
      s_prefix = p;
      if (tile == ntiles - 1) a.ctl->npairs = p + total;
    }
  }
  __syncthreads();
  excl += s_prefix;

#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint64_t t = base + static_cast<uint64_t>(tid) * K + k;
    s_val[pad32(tid * K + k)] = static_cast<uint32_t>(excl);
    if (mine[k] != 0 && t < a.ntris) {
      // expansion tiles whose first pair this object owns
      const OwnedTiles ot = owned_tiles(excl, mine[k], a.tile_shift, a.ntfo);
      if (ot.any) {
        // about one object per expansion tile; its grid is the tile's first
        // or one a few entries after it
        const uint32_t g = one ? gl : grid_of_tri<Batched>(a.gs, static_cast<uint32_t>(t), gl);
        for (uint64_t j = ot.lo; j <= ot.inl; ++j) {
          a.tfo[j] = static_cast<uint32_t>(t);
          if constexpr (Batched) a.tfg[j] = g;
        }
        if (ot.inl < ot.hi) {  // a huge object: the rest of its run goes to the plan kernel
          const uint32_t w = atomicAdd(&a.ctl->tfo_work_n, 1u);
          if (w < a.tfo_work_cap)
            a.tfo_work[w] = make_uint4(static_cast<uint32_t>(t), g, static_cast<uint32_t>(ot.inl + 1),
                                       static_cast<uint32_t>(ot.hi));
          else
            atomicOr(&a.ctl->error, kErrInternal);
        }
      }
    }
    excl += mine[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint64_t t = base + static_cast<uint64_t>(k) * Block + tid;
    if (t < a.ntris) a.start[t] = s_val[pad32(k * Block + tid)];
  }
}

// ---------------------------------------------------------------------------
// Expansion of one tile of N = Block * K pairs (N must be the expansion tile
// the count indexed tfo by): pairs [tile * N, tile * N + n) -> (key, value),
// blocked (item k of thread t is pair tile * N + t * K + k) or wave-striped
// (item k of lane l in wave w is pair tile * N + w * 64 * K + k * 64 + l).
//
// The owner of each pair is found as in the paper's MakeObjectIds +
// InclusiveSum, in its max form: every object writes its id at its first pair
// slot and an inclusive max-scan spreads it over its slots (the tile's first
// slot is seeded with the owner of the tile's first pair).  The relative cell
// offset is the pair index minus the owner's start (the segmented exclusive
// sum of ones), and GlobalCoords maps it into the owner's box.
// ---------------------------------------------------------------------------
struct ExpandArgs {
  GridSet gs;
  const uint32_t* start;    // [ntris] global pair offsets
  const uint64_t* box;      // [ntris]
  const uint32_t* tfo;      // [ntiles + ...] owner of each tile's first pair
  const uint32_t* tfg;      // batched: grid of that owner
  uint32_t ntris;           // total triangles
  Control* ctl;             // for the consistency flag
};

// What the expansion needs of a triangle's grid to form its keys and values.
struct GridKeyParams {
  uint32_t res0, res01, cell_base, tri_base;
};

GB_DEV GridKeyParams key_params(const GridDev& G) {
  return {G.res[0], G.res[0] * G.res[1], static_cast<uint32_t>(G.cell_base), G.tri_base};
}

// The grids of a tile's objects lie in [lo, hi] (batched); most tiles lie in
// one grid, whose parameters are then loaded once for the whole tile.  A
// thread visits its objects in increasing order, so in a tile that straddles
// grids it keeps the parameters of its current grid and the first triangle of
// the next one, and searches again only when an object crosses that boundary.
struct TileGrids {
  uint32_t lo, hi, cur, next_tb;
  GridKeyParams p, q;
};

template <bool Batched>
GB_DEV TileGrids tile_grids(const ExpandArgs& a, uint32_t tile, uint32_t ntiles) {
  TileGrids t{};
  if constexpr (Batched) {
    // the tile is the same for the whole workgroup: made visibly uniform, the
    // grid range and the parameters are scalar loads held in scalar registers
    const uint32_t tu = __builtin_amdgcn_readfirstlane(tile);
    t.lo = __builtin_amdgcn_readfirstlane(a.tfg[tu]);
    t.hi = __builtin_amdgcn_readfirstlane(tu + 1 < ntiles ? a.tfg[tu + 1] : a.gs.ngrids - 1);
    t.cur = t.lo;
    t.p = key_params(a.gs.table[t.lo]);
    t.q = t.p;
    t.next_tb = t.lo + 1 < a.gs.ngrids ? a.gs.table[t.lo + 1].tri_base : 0xFFFFFFFFu;
  } else {
    t.p = key_params(a.gs.one);
  }
  return t;
}

// Parameters of object obj's grid (objects of a thread come in increasing order).
template <bool Batched>
GB_DEV GridKeyParams obj_params(const ExpandArgs& a, TileGrids& t, uint32_t obj) {
  if constexpr (Batched) {
    if (t.lo != t.hi) {
      if (obj >= t.next_tb) {
        t.cur = grid_of_tri<true>(a.gs, obj, t.cur);
        t.q = key_params(a.gs.table[t.cur]);
        t.next_tb = t.cur + 1 < a.gs.ngrids ? a.gs.table[t.cur + 1].tri_base : 0xFFFFFFFFu;
      }
      return t.q;
    }
  }
  return t.p;
}

// Layout of the items a thread holds after expand_tile: wave-striped (item k
// of lane l in wave w is slot w * 64 * K + k * 64 + l; what the radix rank
// needs) or blocked (item k of thread t is slot t * K + k; contiguous stores).
enum ItemLayout : int { kStriped = 0, kBlocked = 1 };

template <int Block, int K, int Layout>
GB_DEV uint32_t item_slot(uint32_t tid, int k) {
  if constexpr (Layout == kBlocked) return tid * K + k;
  else return (tid / kWave) * (kWave * K) + k * kWave + (tid % kWave);
}

// s_slot must hold padded(Block * K) words.  Returns the tile's item count.
// OneGrid: the caller guarantees that the tile's objects lie in one grid.
// coords (optional, blocked single-grid tiles only): each item's cell
// coordinates packed as x | y << 10 | z << 20.
template <int Block, int K, bool Batched, int Layout = kStriped, bool OneGrid = false>
GB_DEV uint32_t expand_tile(const ExpandArgs& a, uint32_t tile, uint64_t npairs, uint32_t ntiles, uint32_t* s_slot,
                            uint32_t* s_wtot, uint32_t (&keys)[K], uint32_t (&vals)[K], uint32_t* coords = nullptr) {
  constexpr int N = Block * K;
  static_assert(N <= 65536, "slot and object offsets are packed in 16 bits");
  constexpr int kHeadBatch = 4;
  const uint32_t tid = threadIdx.x;
  const uint64_t base = static_cast<uint64_t>(tile) * N;
  const uint32_t n = static_cast<uint32_t>(npairs - base < N ? npairs - base : N);
  const uint32_t t0 = a.tfo[tile];
  uint32_t thi = tile + 1 < ntiles ? a.tfo[tile + 1] : a.ntris - 1;
  if (thi < t0) {
    // tile owners must not decrease; if they did, the build reports an internal
    // error and this tile stays within its own first object
    if (threadIdx.x == 0) atomicOr(&a.ctl->error, kErrInternal);
    thi = t0;
  }
  const uint32_t s0 = a.start[t0];  // the carried-in owner starts at or before the tile
#pragma unroll
  for (int k = 0; k < K; ++k) s_slot[pad32(k * Block + tid)] = 0;
  __syncthreads();
  // Each object starting inside the tile marks its first slot with
  // (object offset from t0) << 16 | slot; both fields grow along the tile, so
  // a max-scan hands every slot its owner and the owner's first slot.
  const uint32_t nobj = thi - t0;
  for (uint32_t j0 = 0; j0 < nobj; j0 += Block * kHeadBatch) {
    uint32_t st[kHeadBatch];
#pragma unroll
    for (int u = 0; u < kHeadBatch; ++u) {
      const uint32_t j = j0 + u * Block + tid + 1;
      st[u] = a.start[t0 + (j <= nobj ? j : nobj)];
    }
#pragma unroll
    for (int u = 0; u < kHeadBatch; ++u) {
      const uint32_t j = j0 + u * Block + tid + 1;
      const uint32_t slot = st[u] - static_cast<uint32_t>(base);
      if (j <= nobj && slot < n) s_slot[pad32(slot)] = (j << 16) | slot;
    }
  }
  __syncthreads();
  // inclusive max-scan over the tile's slots, K consecutive slots per thread
  uint32_t sv[K];
  uint32_t run = 0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    sv[k] = s_slot[pad32(tid * K + k)];
    run = run > sv[k] ? run : sv[k];
  }
  run = block_exclusive_max<Block>(run, s_wtot);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    run = run > sv[k] ? run : sv[k];
    sv[k] = run;
  }
  if constexpr (Layout == kStriped) {
#pragma unroll
    for (int k = 0; k < K; ++k) s_slot[pad32(tid * K + k)] = sv[k];
    __syncthreads();
  }
  TileGrids tg = tile_grids<Batched>(a, tile, ntiles);
  // blocked tiles inside one grid step GlobalCoords; blocked tiles that
  // straddle grids (rare) take the chunked path below, which keeps fewer
  // registers live while it looks grids up
  if (Layout == kBlocked && (!Batched || OneGrid || tg.lo == tg.hi)) {
    // A thread's K consecutive slots mostly belong to one object, and an owner
    // that starts inside the run starts at offset 0, so GlobalCoords is only
    // evaluated for the run's first slot and then stepped (x fastest) instead
    // of dividing for every pair.  All K box loads are issued first.
    uint64_t bx[K];
#pragma unroll
    for (int k = 0; k < K; ++k) bx[k] = a.box[t0 + (sv[k] >> 16)];
    uint32_t x = 0, y = 0, z = 0;
    {
      const uint32_t ii = tid * K < n ? tid * K : n - 1;
      const uint32_t v = sv[0];
      const uint32_t rid = (v >> 16) == 0 ? static_cast<uint32_t>(base) + ii - s0 : ii - (v & 0xFFFFu);
      const Box b = unpack_box(bx[0]);
      const uint32_t mxy = b.m[0] * b.m[1];
      z = rid / mxy;
      const uint32_t r2 = rid - z * mxy;
      y = r2 / b.m[0];
      x = r2 - y * b.m[0];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint32_t idx = tid * K + k;
      const uint32_t obj = t0 + (sv[k] >> 16);
      const Box b = unpack_box(bx[k]);
      if (k > 0) {
        if (sv[k] != sv[k - 1]) {
          x = y = z = 0;  // a new owner starts here
        } else {
          ++x;
          const bool cx = x == b.m[0];
          x = cx ? 0u : x;
          y += cx ? 1u : 0u;
          const bool cy = y == b.m[1];
          y = cy ? 0u : y;
          z += cy ? 1u : 0u;
        }
      }
      const GridKeyParams& gp = tg.p;
      const uint32_t cell = (b.lo[0] + x) + gp.res0 * (b.lo[1] + y) + gp.res01 * (b.lo[2] + z);
      if (coords) coords[k] = (b.lo[0] + x) | ((b.lo[1] + y) << 10) | ((b.lo[2] + z) << 20);
      if constexpr (Batched) {
        keys[k] = gp.cell_base + cell;
        vals[k] = obj - gp.tri_base;
      } else {
        keys[k] = cell;
        vals[k] = obj;
      }
      if (idx >= n) {
        keys[k] = 0xFFFFFFFFu;
        vals[k] = 0;
      }
    }
    __syncthreads();
    return n;
  }
  // items in chunks: all box gathers of a chunk are in flight together, while
  // the live registers stay bounded
  constexpr int KC = K >= 8 ? 8 : K;
  static_assert(K % KC == 0, "items per thread must be a multiple of the chunk");
#pragma unroll
  for (int c0 = 0; c0 < K; c0 += KC) {
    uint32_t obj[KC], rid[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      const uint32_t idx = item_slot<Block, K, Layout>(tid, c0 + c);
      const uint32_t ii = idx < n ? idx : n - 1;
      const uint32_t v = Layout == kBlocked ? sv[c0 + c] : s_slot[pad32(ii)];
      const uint32_t r = v >> 16;
      obj[c] = t0 + r;
      rid[c] = r == 0 ? static_cast<uint32_t>(base) + ii - s0 : ii - (v & 0xFFFFu);
    }
    uint64_t bx[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) bx[c] = a.box[obj[c]];
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      const int k = c0 + c;
      const uint32_t idx = item_slot<Block, K, Layout>(tid, k);
      const Box b = unpack_box(bx[c]);
      const GridKeyParams gp = obj_params<Batched>(a, tg, obj[c]);
      const uint32_t cell = cell_of(b, rid[c], gp.res0, gp.res01);
      if constexpr (Batched) {
        keys[k] = gp.cell_base + cell;
        vals[k] = obj[c] - gp.tri_base;
      } else {
        keys[k] = cell;
        vals[k] = obj[c];
      }
      if (idx >= n) {
        keys[k] = 0xFFFFFFFFu;
        vals[k] = 0;
      }
    }
  }
  __syncthreads();
  return n;
}

// ---------------------------------------------------------------------------
// Radix sort plan: up to 4 passes over the low `bits` bits of the key.
// ---------------------------------------------------------------------------
constexpr int kHistCopies = 16;   // global copies of the digit histograms (see flush_hist)

struct SortPlan {
  uint32_t passes;
  uint32_t shift[4];
  uint32_t width[4];
};

constexpr int kRadixMax = 2048;

// Object-order pair lists written out (the expansion on its own).  With
// RB > 0 it also accumulates the digit histograms of every radix pass from
// the keys it holds, and clears the passes' look-back words, so the sort can
// start from these arrays without another read.
struct ExpandOutArgs {
  ExpandArgs ex;
  uint32_t* cells;
  uint32_t* objs;
  SortPlan plan;
  uint32_t* hist;           // [4][kRadixMax]
  StatusClear clear;        // the radix passes' look-back words
  uint32_t vec16;           // cells and objs are 16-byte aligned
  Control* ctl;
};

// Batched tile whose objects lie in more than one grid.
GB_DEV bool tile_straddles(const ExpandArgs& a, uint32_t tile, uint32_t ntiles) {
  const uint32_t hi = tile + 1 < ntiles ? a.tfg[tile + 1] : a.gs.ngrids - 1;
  return a.tfg[tile] != hi;
}

// Digit histograms of every pass for a thread's K consecutive keys (blocked
// layout): consecutive pairs of one object mostly share their upper digits, so
// each run of equal digits is added once.
template <int Block, int K, int RB>
GB_DEV void hist_runs(const SortPlan& plan, const uint32_t (&keys)[K], uint32_t n, uint32_t* s_hist) {
  constexpr int R = 1 << RB;
  const uint32_t first = threadIdx.x * K;
  const uint32_t m = first < n ? (n - first < K ? n - first : K) : 0;
  for (uint32_t p = 0; p < plan.passes; ++p) {
    const uint32_t sh = plan.shift[p], dm = (1u << plan.width[p]) - 1u;
    uint32_t cur = 0, cnt = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (static_cast<uint32_t>(k) < m) {
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

// Store a tile's pairs (a thread's K consecutive pairs, 16-byte stores when
// all are present) and add its digits to the block's histograms.
template <int Block, int K, int RB>
GB_DEV void store_tile(const ExpandOutArgs& a, uint32_t tile, uint32_t n, const uint32_t (&keys)[K],
                       const uint32_t (&vals)[K], uint32_t* s_hist) {
  constexpr int N = Block * K;
  constexpr int R = RB > 0 ? 1 << RB : 1;
  const uint64_t base = static_cast<uint64_t>(tile) * N;
  const uint32_t first = threadIdx.x * K;
  if (a.vec16 && first + K <= n) {
    uint4* ck = reinterpret_cast<uint4*>(a.cells + base + first);
    uint4* ov = reinterpret_cast<uint4*>(a.objs + base + first);
#pragma unroll
    for (int q = 0; q < K / 4; ++q) {
      ck[q] = make_uint4(keys[4 * q], keys[4 * q + 1], keys[4 * q + 2], keys[4 * q + 3]);
      ov[q] = make_uint4(vals[4 * q], vals[4 * q + 1], vals[4 * q + 2], vals[4 * q + 3]);
    }
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (first + k < n) {
        a.cells[base + first + k] = keys[k];
        a.objs[base + first + k] = vals[k];
      }
    }
  }
  if constexpr (RB > 0) hist_runs<Block, K, RB>(a.plan, keys, n, s_hist);
}

// A block's histograms go into one of kHistCopies global copies (chosen by
// block index), so the blocks that finish together do not all add into the
// same words; the first tile of each radix pass sums the copies.
template <int RB, int Block>
GB_DEV void flush_hist(const SortPlan& plan, uint32_t* hist, const uint32_t* s_hist) {
  constexpr int R = 1 << RB;
  uint32_t* h = hist + (blockIdx.x % kHistCopies) * (4 * kRadixMax);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < plan.passes * R; i += Block) {
    const uint32_t v = s_hist[i];
    if (v) atomicAdd(&h[(i / R) * kRadixMax + (i % R)], v);
  }
}

// The expansion written out in object order, with the digit histograms of
// every radix pass and the look-back words of every pass cleared.  Batched
// builds skip the tiles that straddle grids here; expand_straddle_kernel
// writes those.  Bounded to six waves per SIMD (at most 80 VGPRs, no spills):
// at five, the owners' dependent loads were hidden less well (0.186 against
// 0.167 ms on 51M pairs).
template <int Block, int K, int RB, bool Batched>
__global__ __launch_bounds__(Block, 6) void expand_kernel(ExpandOutArgs a) {
  constexpr int N = Block * K;
  constexpr int R = RB > 0 ? 1 << RB : 1;
  static_assert(K % 4 == 0, "items are stored four at a time");
  __shared__ uint32_t s_owner[padded(N)];
  __shared__ uint32_t s_hist[RB > 0 ? 4 * R : 1];
  __shared__ uint32_t s_wtot[Block / kWave];
  __shared__ uint32_t s_tile;
  if (build_failed(a.ctl)) return;
  const uint64_t npairs = a.ctl->npairs;
  const uint32_t ntiles = static_cast<uint32_t>((npairs + N - 1) / N);
  if constexpr (RB > 0) {
    clear_status<Block>(a.clear, npairs);
    for (int i = threadIdx.x; i < 4 * R; i += Block) s_hist[i] = 0;
  }
  while (true) {
    const uint32_t tile = next_tile(&a.ctl->tile_counter[kCtrExpand], &s_tile);
    if (tile >= ntiles) break;
    if constexpr (Batched) {
      if (tile_straddles(a.ex, __builtin_amdgcn_readfirstlane(tile), ntiles)) continue;
    }
    uint32_t keys[K], vals[K];
    const uint32_t n =
        expand_tile<Block, K, Batched, kBlocked, true>(a.ex, tile, npairs, ntiles, s_owner, s_wtot, keys, vals);
    store_tile<Block, K, RB>(a, tile, n, keys, vals, s_hist);
  }
  if constexpr (RB > 0) flush_hist<RB, Block>(a.plan, a.hist, s_hist);
}

// Batched builds: the tiles whose objects lie in more than one grid (about
// one per grid boundary), with the grid looked up per object.
template <int Block, int K, int RB>
__global__ __launch_bounds__(Block, 2) void expand_straddle_kernel(ExpandOutArgs a) {
  constexpr int N = Block * K;
  constexpr int R = RB > 0 ? 1 << RB : 1;
  __shared__ uint32_t s_owner[padded(N)];
  __shared__ uint32_t s_hist[RB > 0 ? 4 * R : 1];
  __shared__ uint32_t s_wtot[Block / kWave];
  if (build_failed(a.ctl)) return;
  const uint64_t npairs = a.ctl->npairs;
  const uint32_t ntiles = static_cast<uint32_t>((npairs + N - 1) / N);
  if constexpr (RB > 0) {
    for (int i = threadIdx.x; i < 4 * R; i += Block) s_hist[i] = 0;
  }
  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    if (!tile_straddles(a.ex, __builtin_amdgcn_readfirstlane(tile), ntiles)) continue;
    __syncthreads();  // the previous tile's readers of s_owner are done
    uint32_t keys[K], vals[K];
    const uint32_t n =
        expand_tile<Block, K, true, kBlocked, false>(a.ex, tile, npairs, ntiles, s_owner, s_wtot, keys, vals);
    store_tile<Block, K, RB>(a, tile, n, keys, vals, s_hist);
  }
  if constexpr (RB > 0) flush_hist<RB, Block>(a.plan, a.hist, s_hist);
}

// The pair generation of sorted-grid builders (Related Work; their MakePairs
// kernel, which the Test Results section finds dominant on architectural
// scenes): one thread per object writes all of that object's pairs, so a
// thread's work is its object's cell count.  Plain builds only; it writes
// what expand_kernel writes: the object-order pairs, the digit histograms of
// every radix pass and the passes' cleared look-back words.
template <int Block, int RB>
__global__ __launch_bounds__(Block) void makepairs_kernel(ExpandOutArgs a) {
  constexpr int R = RB > 0 ? 1 << RB : 1;
  __shared__ uint32_t s_hist[RB > 0 ? 4 * R : 1];
  if (build_failed(a.ctl)) return;
  if constexpr (RB > 0) {
    clear_status<Block>(a.clear, a.ctl->npairs);
    for (int i = threadIdx.x; i < 4 * R; i += Block) s_hist[i] = 0;
    __syncthreads();
  }
  const uint32_t res0 = a.ex.gs.one.res[0];
  const uint32_t res01 = res0 * a.ex.gs.one.res[1];
  // a run of equal digits per pass is added to the histogram once
  uint32_t cur[4] = {0, 0, 0, 0}, cnt[4] = {0, 0, 0, 0};
  const uint64_t step = static_cast<uint64_t>(gridDim.x) * Block;
  for (uint64_t t = static_cast<uint64_t>(blockIdx.x) * Block + threadIdx.x; t < a.ex.ntris; t += step) {
    const Box b = unpack_box(a.ex.box[t]);
    const uint64_t s0 = a.ex.start[t];
    const uint32_t n = b.m[0] * b.m[1] * b.m[2];
    uint32_t x = 0, y = 0, z = 0;  // GlobalCoords stepped along the object's cells
    for (uint32_t r = 0; r < n; ++r) {
      const uint32_t cell = (b.lo[0] + x) + res0 * (b.lo[1] + y) + res01 * (b.lo[2] + z);
      a.cells[s0 + r] = cell;
      a.objs[s0 + r] = static_cast<uint32_t>(t);
      if constexpr (RB > 0) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          if (static_cast<uint32_t>(p) < a.plan.passes) {
            const uint32_t d = (cell >> a.plan.shift[p]) & ((1u << a.plan.width[p]) - 1u);
            if (cnt[p] != 0 && d != cur[p]) {
              atomicAdd(&s_hist[p * R + cur[p]], cnt[p]);
              cnt[p] = 0;
            }
            cur[p] = d;
            ++cnt[p];
          }
        }
      }
      if (++x == b.m[0]) {
        x = 0;
        if (++y == b.m[1]) {
          y = 0;
          ++z;
        }
      }
    }
  }
  if constexpr (RB > 0) {
#pragma unroll
    for (int p = 0; p < 4; ++p)
      if (cnt[p] != 0) atomicAdd(&s_hist[p * R + cur[p]], cnt[p]);
    flush_hist<RB, Block>(a.plan, a.hist, s_hist);
  }
}

// One read of the keys (regenerated from the expansion) for the digit
// histograms of every pass; also clears the look-back words of every pass.
struct HistArgs {
  ExpandArgs ex;
  SortPlan plan;
  uint32_t* hist;           // [4][kRadixMax]
  StatusClear clear;        // the radix passes' look-back words
  Control* ctl;
};

template <int Block, int K, int RB, bool Batched>
__global__ __launch_bounds__(Block) void hist_kernel(HistArgs a) {
  constexpr int N = Block * K;
  constexpr int R = 1 << RB;
  __shared__ uint32_t s_owner[padded(N)];
  __shared__ uint32_t s_hist[4 * R];
  __shared__ uint32_t s_wtot[Block / kWave];
  __shared__ uint32_t s_tile;
  if (build_failed(a.ctl)) return;
  const uint64_t npairs = a.ctl->npairs;
  const uint32_t ntiles = static_cast<uint32_t>((npairs + N - 1) / N);
  clear_status<Block>(a.clear, npairs);
  for (int i = threadIdx.x; i < 4 * R; i += Block) s_hist[i] = 0;
  __syncthreads();
  while (true) {
    const uint32_t tile = next_tile(&a.ctl->tile_counter[kCtrHist], &s_tile);
    if (tile >= ntiles) break;
    // blocked layout: GlobalCoords stepped along each thread's run of slots,
    // and each run of equal digits added once
    uint32_t keys[K], vals[K];
    const uint32_t n = expand_tile<Block, K, Batched, kBlocked>(a.ex, tile, npairs, ntiles, s_owner, s_wtot, keys, vals);
    hist_runs<Block, K, RB>(a.plan, keys, n, s_hist);
  }
  flush_hist<RB, Block>(a.plan, a.hist, s_hist);
}

}  // namespace gb
