// Per-grid bookkeeping after the count, and the per-cell range table
// (RunLengthEncode + NonEmptyCells + ExclusiveSum over the grid, Algorithm 1).
//
// The ranges are produced by a merge-path walk over two sorted sequences: the
// cell events 0..R (event c stands for "cell c begins") and the sorted pair
// cells, with an event ordered before the pairs of its own cell.  When event c
// is reached, the number of pairs consumed so far is exactly the number of
// pairs whose cell is < c, which is G[c].  Tiles split the merged sequence
// evenly, so the work per tile is the same whether the cells are empty or
// full; each event writes the begin of its cell and the end of the cell before
// it, and the writes of a tile are one contiguous stretch of the table.
#pragma once

#include "kernels.hpp"

namespace gb {

struct GridRun {
  uint64_t pair_base;    // first pair of the grid in the batch's pair list
  uint64_t npairs;       // NO of the grid
  uint32_t mtile_base;   // first merge tile of the grid
  uint32_t mtiles;       // merge tiles of the grid
};

// One workgroup: pair bases, pair counts and merge tiles of every grid.
struct PlanArgs {
  GridSet gs;
  const uint32_t* start;   // [ntris]
  uint32_t ntris;
  uint32_t merge_tile;     // items per merge tile
  GridRun* run;            // [ngrids + 1]; run[ngrids].mtile_base = total merge tiles
  uint64_t* npairs_out;    // [ngrids + 1] each grid's NO for the host, then the count's status word
  uint32_t* cap_flag;      // set when a grid's NO exceeds its capacity
  uint64_t cap_total;      // pairs the workspace holds (all grids together)
  uint32_t* tfo;           // tile-owner table of the expansion (and tfg, batched) ...
  uint32_t* tfg;
  const uint4* tfo_work;   // ... and the runs of it the count left for this kernel
  uint32_t tfo_work_cap;
  Control* ctl;
};

template <int Block, bool Batched>
__global__ __launch_bounds__(Block) void plan_kernel(PlanArgs a) {
  __shared__ uint32_t s_wtot[Block / kWave];
  {
    // the tile-owner runs of huge objects, written by the whole workgroup
    const uint32_t nw = a.ctl->tfo_work_n < a.tfo_work_cap ? a.ctl->tfo_work_n : a.tfo_work_cap;
    for (uint32_t w = 0; w < nw; ++w) {
      const uint4 it = a.tfo_work[w];
      for (uint32_t j = it.z + threadIdx.x; j <= it.w; j += Block) {
        a.tfo[j] = it.x;
        if constexpr (Batched) a.tfg[j] = it.y;
      }
    }
  }
  const uint64_t total = a.ctl->npairs;
  const uint32_t G = a.gs.ngrids;
  if (threadIdx.x == 0 && total > 0xFFFFFFFFull) atomicOr(a.cap_flag, 2u);  // 32-bit pair indices overflow
  for (uint32_t g = threadIdx.x; g < G; g += Block) {
    const uint32_t tb = grid_at<Batched>(a.gs, g).tri_base;
    a.run[g].pair_base = tb < a.ntris ? a.start[tb] : total;
  }
  __syncthreads();
  uint32_t carry = 0;
  for (uint32_t g0 = 0; g0 < G; g0 += Block) {
    const uint32_t g = g0 + threadIdx.x;
    uint32_t tiles = 0;
    if (g < G) {
      const GridDev& gd = grid_at<Batched>(a.gs, g);
      const uint64_t pb = a.run[g].pair_base;
      const uint64_t pe = g + 1 < G ? a.run[g + 1].pair_base : total;
      const uint64_t no = pe - pb;
      const uint64_t ncell = static_cast<uint64_t>(gd.res[0]) * gd.res[1] * gd.res[2];
      a.run[g].npairs = no;
      if (a.npairs_out) a.npairs_out[g] = no;
      if (no > gd.cap_pairs) atomicOr(a.cap_flag, 1u);
      const uint64_t len = ncell + 1 + no;
      tiles = static_cast<uint32_t>((len + a.merge_tile - 1) / a.merge_tile);
      a.run[g].mtiles = tiles;
    }
    uint32_t tot;
    const uint32_t ex = block_exclusive_sum<Block>(tiles, s_wtot, tot);
    if (g < G) a.run[g].mtile_base = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    a.run[G].mtile_base = carry;
    if (total > a.cap_total) atomicOr(a.cap_flag, 1u);
  }
  if (a.npairs_out) {
    // the status word: the count's error bits, then the capacity flags shifted by 2
    __syncthreads();
    if (threadIdx.x == 0) a.npairs_out[G] = a.ctl->error | (static_cast<uint64_t>(atomicOr(a.cap_flag, 0u)) << 2);
  }
}

// Where the last radix pass of a batched build writes each grid's pairs: its
// output arrays, its first pair in the batch and its first cell in the batch's
// cell space (32 bytes, read with two vector loads).
struct alignas(16) GridSink {
  uint32_t* cells;
  uint32_t* objs;
  uint64_t pair_base;
  uint32_t cell_base;
  uint32_t straddles;      // in the key map: the bucket holds more than one grid's keys
};

// Sort keys number the cells of all grids of a batch in one space.  Bucket j
// of the key map covers the keys [j << kshift, (j + 1) << kshift) and holds the
// grids of its first and last key, so the grid of a key is one cached load
// away, with a short search only in the few buckets a grid boundary crosses.
struct SinkArgs {
  GridSet gs;
  const GridRun* run;
  uint32_t* cap_flag;      // set when a grid's NO exceeds the capacity of its outputs
  GridSink* sink;          // [ngrids]
  uint2* kmap;             // [nbuckets] grids of the bucket's first and last key
  GridSink* ksink;         // [nbuckets] the sink of the bucket's first grid, straddles set if it has several
  uint32_t nbuckets;
  uint32_t kshift;
  uint64_t ncells;         // cells of the batch: every key is below it
};

// Largest g with cell_base[g] <= key.
GB_DEV uint32_t grid_of_cell(const GridSet& s, uint64_t key) {
  uint32_t lo = 0, hi = s.ngrids;  // answer in [lo, hi)
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (s.table[mid].cell_base <= key) lo = mid; else hi = mid;
  }
  return lo;
}

template <int Block>
__global__ __launch_bounds__(Block) void sink_kernel(SinkArgs a) {
  const uint32_t stride = gridDim.x * Block;
  const uint32_t first = blockIdx.x * Block + threadIdx.x;
  for (uint32_t g = first; g < a.gs.ngrids; g += stride) {
    const GridDev& d = a.gs.table[g];
    // the outputs may have been given after the count (a build resumed from its
    // count): their capacities are checked again here, before any pass writes
    if (a.run[g].npairs > d.cap_pairs) atomicOr(a.cap_flag, 1u);
    GridSink k;
    k.cells = d.out_cells;
    k.objs = d.out_objs;
    k.pair_base = a.run[g].pair_base;
    k.cell_base = static_cast<uint32_t>(d.cell_base);
    k.straddles = 0;
    a.sink[g] = k;
  }
  for (uint32_t j = first; j < a.nbuckets; j += stride) {
    const uint64_t k0 = static_cast<uint64_t>(j) << a.kshift;
    const uint64_t k1e = (static_cast<uint64_t>(j + 1) << a.kshift) - 1;
    const uint64_t k1 = k1e < a.ncells - 1 ? k1e : a.ncells - 1;
    const uint32_t glo = grid_of_cell(a.gs, k0), ghi = grid_of_cell(a.gs, k1);
    a.kmap[j] = make_uint2(glo, ghi);
    // the bucket's own copy of its first grid's sink: one load for most keys
    const GridDev& d = a.gs.table[glo];
    GridSink k;
    k.cells = d.out_cells;
    k.objs = d.out_objs;
    k.pair_base = a.run[glo].pair_base;
    k.cell_base = static_cast<uint32_t>(d.cell_base);
    k.straddles = glo != ghi ? 1u : 0u;
    a.ksink[j] = k;
  }
}

// Grid of key within [lo, hi] (binary search over the sinks, one thread).
GB_DEV uint32_t sink_of_key(const GridSink* sink, uint32_t key, uint32_t lo, uint32_t hi) {
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (sink[mid].cell_base <= key) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Grid of merge tile b: largest g with run[g].mtile_base <= b.
GB_DEV uint32_t grid_of_mtile(const GridRun* run, uint32_t ngrids, uint32_t b) {
  uint32_t lo = 0, hi = ngrids;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (run[mid].mtile_base <= b) lo = mid; else hi = mid;
  }
  return lo;
}

struct RangesArgs {
  GridSet gs;
  const GridRun* run;
  uint32_t* splits;        // [total merge tiles] pair index at each tile's start
  uint32_t* tile_grid;     // [total merge tiles] batched: grid of each tile (written by split_kernel)
  uint32_t merge_tile;
  Control* ctl;
};

// Merge-path split at diagonal d of grid g: the number of pairs among the
// first d merged items = the smallest j with cells[j] + j + 1 >= d.
GB_DEV uint32_t merge_split(const uint32_t* cells, uint64_t npairs, uint64_t nevents, uint64_t d) {
  uint64_t lo = d > nevents ? d - nevents : 0;
  uint64_t hi = d < npairs ? d : npairs;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (static_cast<uint64_t>(cells[mid]) + mid + 1 >= d) hi = mid; else lo = mid + 1;
  }
  return static_cast<uint32_t>(lo);
}

// Plain builds: each workgroup first loads kSplitSamples evenly spaced cells
// into LDS (one round of loads), and each search takes its first levels
// there: it narrows [lo, hi] to the stretch between the two samples around
// the answer, about npairs / kSplitSamples pairs, before it reads HBM.
constexpr uint32_t kSplitSamples = 1024;

template <int Block, bool Batched>
__global__ __launch_bounds__(Block) void split_kernel(RangesArgs a) {
  __shared__ uint32_t s_sample[Batched ? 1 : kSplitSamples];
  if (build_failed(a.ctl)) return;
  const uint32_t G = a.gs.ngrids;
  const uint32_t total = a.run[G].mtile_base;
  if constexpr (!Batched) {
    // sample k is the cell of pair k * npairs / kSplitSamples (< npairs)
    const uint64_t np = a.run[0].npairs;
    for (uint32_t k = threadIdx.x; k < kSplitSamples; k += Block)
      s_sample[k] = np ? a.gs.one.out_cells[static_cast<uint64_t>(k) * np / kSplitSamples] : 0u;
    __syncthreads();
  }
  for (uint32_t b = blockIdx.x * Block + threadIdx.x; b < total; b += gridDim.x * Block) {
    const uint32_t g = Batched ? grid_of_mtile(a.run, G, b) : 0;
    const GridDev& gd = grid_at<Batched>(a.gs, g);
    const uint64_t ncell = static_cast<uint64_t>(gd.res[0]) * gd.res[1] * gd.res[2];
    const uint64_t d = static_cast<uint64_t>(b - a.run[g].mtile_base) * a.merge_tile;
    const uint64_t np = a.run[g].npairs;
    if constexpr (Batched) {
      a.splits[b] = merge_split(gd.out_cells, np, ncell + 1, d);
      a.tile_grid[b] = g;
    } else {
      // the first sample k whose pair p_k = k * np / kSplitSamples already
      // satisfies cells[p] + p + 1 >= d; the answer lies in (p_{k-1}, p_k]
      // (k = kSplitSamples: in (p_{last}, np])
      uint32_t kl = 0, kh = kSplitSamples;
      while (kl < kh) {
        const uint32_t km = (kl + kh) >> 1;
        const uint64_t pm = static_cast<uint64_t>(km) * np / kSplitSamples;
        if (static_cast<uint64_t>(s_sample[km]) + pm + 1 >= d) kh = km; else kl = km + 1;
      }
      const uint64_t L = kl ? static_cast<uint64_t>(kl - 1) * np / kSplitSamples + 1 : 0;
      const uint64_t H = kl < kSplitSamples ? static_cast<uint64_t>(kl) * np / kSplitSamples : np;
      // the search's own bounds, then the stretch (the answer is clamped to them)
      const uint64_t lo0 = d > ncell + 1 ? d - (ncell + 1) : 0;
      const uint64_t hi0 = d < np ? d : np;
      uint64_t lo = L < hi0 ? L : hi0;
      lo = lo > lo0 ? lo : lo0;
      uint64_t hi = H > lo0 ? H : lo0;
      hi = hi < hi0 ? hi : hi0;
      while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (static_cast<uint64_t>(gd.out_cells[mid]) + mid + 1 >= d) hi = mid; else lo = mid + 1;
      }
      a.splits[b] = static_cast<uint32_t>(lo);
    }
  }
}

// Eight waves per SIMD: every block of the persistent grid is resident at once
// (a block that started late would run its whole static share of the tiles
// after the others had finished).
template <int Block, int K, bool Batched>
__global__ __launch_bounds__(Block, 8) void ranges_kernel(RangesArgs a) {
  constexpr int D = Block * K;
  static_assert(D < 65535, "tile-relative cells and pair offsets are held in 16 bits");
  // Within a tile the pairs' cells lie in [i0 - 1, i1 - 1] and the begins in
  // [j0, j1], so both are kept relative to the tile in 16 bits: half the LDS
  // of 32-bit copies, so every persistent block of a CU stays resident.
  __shared__ uint16_t s_cells[D];   // cell + 1 - i0
  __shared__ uint16_t s_begin[D];   // begin - j0
  if (build_failed(a.ctl)) return;
  const uint32_t G = a.gs.ngrids;
  const uint32_t total = a.run[G].mtile_base;
  const uint32_t tid = threadIdx.x;
  // tiles are independent: a static stride over them, no tile counter
  for (uint32_t b = blockIdx.x; b < total; b += gridDim.x) {
    const uint32_t g = Batched ? __builtin_amdgcn_readfirstlane(a.tile_grid[b]) : 0;
    const GridDev& gd = grid_at<Batched>(a.gs, g);
    const GridRun& gr = a.run[g];
    const uint64_t ncell = static_cast<uint64_t>(gd.res[0]) * gd.res[1] * gd.res[2];
    const uint64_t len = ncell + 1 + gr.npairs;
    const uint32_t lb = b - gr.mtile_base;
    const uint64_t d0 = static_cast<uint64_t>(lb) * D;
    const uint64_t d1 = d0 + D < len ? d0 + D : len;
    const uint64_t j0 = a.splits[b];
    const uint64_t j1 = lb + 1 < gr.mtiles ? a.splits[b + 1] : gr.npairs;
    const uint64_t i0 = d0 - j0, i1 = d1 - j1;
    const uint32_t np = static_cast<uint32_t>(j1 - j0), ne = static_cast<uint32_t>(i1 - i0);
    const uint32_t cbase = static_cast<uint32_t>(i0) - 1u;  // cells of the tile's pairs are >= i0 - 1
    // all K loads of a thread in flight at once (np <= D = Block * K), at
    // 32-bit offsets from the tile's first pair
    const uint32_t* cells_t = gd.out_cells + j0;
    uint32_t cv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint32_t p = k * Block + tid;
      cv[k] = p < np ? cells_t[p] : 0u;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint32_t p = k * Block + tid;
      if (p < np) s_cells[p] = static_cast<uint16_t>(cv[k] - cbase);
    }
    __syncthreads();
    // this thread's stretch of the tile's diagonal; in relative terms pair p
    // precedes event e when cell(p) < i0 + e, i.e. s_cells[p] <= e
    const uint32_t dd0 = tid * K;
    const uint32_t nd = np + ne;
    if (dd0 < nd) {
      // first pair index p with cell(p) + (j0 + p) + 1 >= d0 + dd0, i.e. s_cells[p] + p >= dd0
      uint32_t lo = dd0 > ne ? dd0 - ne : 0, hi = dd0 < np ? dd0 : np;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (static_cast<uint32_t>(s_cells[mid]) + mid >= dd0) hi = mid; else lo = mid + 1;
      }
      uint32_t p = lo, e = dd0 - lo;
      const uint32_t dend = dd0 + K < nd ? dd0 + K : nd;
      for (uint32_t dd = dd0; dd < dend; ++dd) {
        if (e < ne && (p >= np || e + 1 <= s_cells[p])) {
          s_begin[e] = static_cast<uint16_t>(p);
          ++e;
        } else {
          ++p;
        }
      }
    }
    __syncthreads();
    // ranges[q] for q in [2 i0 - 1, 2 i1 - 1): q = 2c is begin(c), q = 2c - 1 is end(c - 1) = begin(c).
    // (i1 >= 1: the first merged item is event 0.)  Entry q0 + ql is the
    // begin of cell i0 + (ql + odd) / 2, with odd = 1 only for the first tile
    // (q0 = 0); at most 2 * D entries per tile, at 32-bit offsets from q0.
    const uint64_t q0 = i0 > 0 ? 2 * i0 - 1 : 0;
    const uint64_t q1e = 2 * i1 - 1;
    const uint64_t q1 = q1e < 2 * ncell ? q1e : 2 * ncell;
    const uint32_t nq = static_cast<uint32_t>(q1 > q0 ? q1 - q0 : 0);
    const uint32_t odd = i0 == 0 ? 1u : 0u;
    const uint32_t jb = static_cast<uint32_t>(j0);
    uint32_t* out_t = gd.out_ranges + q0;
    // sixteen LDS reads in flight, then their stores (a read past the tile's
    // entries is clamped into s_begin and stores nothing)
    constexpr int kGroup = 16;
    static_assert((2 * K) % kGroup == 0, "output entries are written in groups");
#pragma unroll
    for (int k0 = 0; k0 < 2 * K; k0 += kGroup) {
      uint32_t v[kGroup];
#pragma unroll
      for (int k = 0; k < kGroup; ++k) {
        const uint32_t e = ((k0 + k) * Block + tid + odd) >> 1;
        v[k] = s_begin[e < static_cast<uint32_t>(D) ? e : D - 1];
      }
#pragma unroll
      for (int k = 0; k < kGroup; ++k) {
        const uint32_t ql = (k0 + k) * Block + tid;
        if (ql < nq) out_t[ql] = jb + v[k];
      }
    }
    __syncthreads();
  }
}

}  // namespace gb
