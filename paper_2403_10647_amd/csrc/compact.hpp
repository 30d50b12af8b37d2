// The compact-grid build (the atomic construction of the Related Work
// section, which the paper compares against and whose combination with its
// own method, chosen by a statistics pass, it lists as future work):
//   1. every <object, cell> pair adds one to its cell's count (atomics);
//   2. an exclusive scan over the cells turns the counts into each cell's
//      first slot, the paper's compact grid G;
//   3. every pair takes the next slot of its cell (atomics) and writes itself
//      there, in an order the atomics leave open;
//   4. each cell's object ids are sorted, so the output is exactly the sorted
//      path's (a cell's pairs are distinct objects, so their order is unique).
// The range table doubles as the counters: ranges[2c + 1] holds cell c's
// count, then its next free slot, and ends as its end.
#pragma once

#include "ranges.hpp"

namespace gb {

constexpr uint32_t kSmallCell = 32;     // cells of at most this many pairs are sorted by one thread
constexpr uint32_t kLdsCell = 8192;     // larger cells up to this size by a workgroup in LDS

struct CompactArgs {
  ExpandArgs ex;
  uint32_t* ranges;         // [2R] the caller's range table
  uint32_t* cells;          // [cap] outputs
  uint32_t* objs;
  uint64_t cap;
  uint64_t ncells;
  uint64_t* status;         // [cell-scan tiles] look-back words (zeroed)
  uint2* big;               // [big_cap] (first slot, size) of cells larger than kSmallCell
  uint32_t big_cap;
  uint32_t* scratch;        // [cap] merge buffer for cells larger than kLdsCell
  Control* ctl;
};

// Pass 1: counts.  Expansion tiles of N = Block * K pairs (the count's tile-owner table).
template <int Block, int K>
__global__ __launch_bounds__(Block, 4) void compact_count_kernel(CompactArgs a) {
  constexpr int N = Block * K;
  __shared__ uint32_t s_owner[padded(N)];
  __shared__ uint32_t s_wtot[Block / kWave];
  __shared__ uint32_t s_tile;
  if (build_failed(a.ctl)) return;
  const uint64_t npairs = a.ctl->npairs;
  const uint32_t ntiles = static_cast<uint32_t>((npairs + N - 1) / N);
  while (true) {
    const uint32_t tile = next_tile(&a.ctl->tile_counter[kCtrExpand], &s_tile);
    if (tile >= ntiles) break;
    uint32_t keys[K], vals[K];
    const uint32_t n = expand_tile<Block, K, false, kBlocked, true>(a.ex, tile, npairs, ntiles, s_owner, s_wtot, keys, vals);
    for (int k = 0; k < K; ++k)  // unrolled by the compiler (constant trip count)
      if (threadIdx.x * K + k < n) atomicAdd(&a.ranges[2 * static_cast<uint64_t>(keys[k]) + 1], 1u);
  }
}

// Pass 2: exclusive scan of the counts over the cells (decoupled look-back);
// each cell's begin and next free slot both become its first slot.
template <int Block, int K>
__global__ __launch_bounds__(Block) void compact_scan_kernel(CompactArgs a) {
  constexpr int N = Block * K;
  __shared__ uint32_t s_wtot[Block / kWave];
  __shared__ uint64_t s_prefix;
  __shared__ uint32_t s_tile;
  if (build_failed(a.ctl)) return;
  const uint32_t ntiles = static_cast<uint32_t>((a.ncells + N - 1) / N);
  uint2* rg = reinterpret_cast<uint2*>(a.ranges);
  while (true) {
    const uint32_t tile = next_tile(&a.ctl->tile_counter[kCtrSort0], &s_tile);
    if (tile >= ntiles) break;
    const uint64_t c0 = static_cast<uint64_t>(tile) * N + threadIdx.x * K;
    uint32_t cnt[K];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      cnt[k] = c0 + k < a.ncells ? rg[c0 + k].y : 0u;
      sum += cnt[k];
    }
    uint32_t total;
    uint32_t excl = block_exclusive_sum<Block>(sum, s_wtot, total);
    if (threadIdx.x < kWave) {
      const uint64_t p = lookback_wave(a.status, tile, total);
      if (threadIdx.x == 0) s_prefix = p;
    }
    __syncthreads();
    excl += static_cast<uint32_t>(s_prefix);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (c0 + k < a.ncells) rg[c0 + k] = make_uint2(excl, excl);
      excl += cnt[k];
    }
    __syncthreads();
  }
}

// Pass 3: every pair takes the next free slot of its cell.
template <int Block, int K>
__global__ __launch_bounds__(Block, 4) void compact_scatter_kernel(CompactArgs a) {
  constexpr int N = Block * K;
  __shared__ uint32_t s_owner[padded(N)];
  __shared__ uint32_t s_wtot[Block / kWave];
  __shared__ uint32_t s_tile;
  if (build_failed(a.ctl)) return;
  const uint64_t npairs = a.ctl->npairs;
  const uint32_t ntiles = static_cast<uint32_t>((npairs + N - 1) / N);
  while (true) {
    const uint32_t tile = next_tile(&a.ctl->tile_counter[kCtrHist], &s_tile);
    if (tile >= ntiles) break;
    uint32_t keys[K], vals[K];
    const uint32_t n = expand_tile<Block, K, false, kBlocked, true>(a.ex, tile, npairs, ntiles, s_owner, s_wtot, keys, vals);
    uint32_t pos[K];
#pragma unroll
    for (int k = 0; k < K; ++k)
      pos[k] = threadIdx.x * K + k < n ? atomicAdd(&a.ranges[2 * static_cast<uint64_t>(keys[k]) + 1], 1u) : 0u;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (threadIdx.x * K + k < n && pos[k] < a.cap) {
        a.cells[pos[k]] = keys[k];
        a.objs[pos[k]] = vals[k];
      }
    }
  }
}

// Pass 4a: cells of at most kSmallCell pairs sorted by one thread each
// (insertion sort in place); larger cells are listed for pass 4b.
template <int Block>
__global__ __launch_bounds__(Block) void compact_sort_small_kernel(CompactArgs a) {
  if (build_failed(a.ctl)) return;
  const uint2* rg = reinterpret_cast<const uint2*>(a.ranges);
  for (uint64_t c = static_cast<uint64_t>(blockIdx.x) * Block + threadIdx.x; c < a.ncells;
       c += static_cast<uint64_t>(gridDim.x) * Block) {
    const uint2 r = rg[c];
    const uint32_t m = r.y - r.x;
    if (m < 2) continue;
    if (m > kSmallCell) {
      const uint32_t w = atomicAdd(&a.ctl->big_n, 1u);
      if (w < a.big_cap) a.big[w] = make_uint2(r.x, m);
      else atomicOr(&a.ctl->error, kErrInternal);
      continue;
    }
    uint32_t* o = a.objs + r.x;
    for (uint32_t i = 1; i < m; ++i) {
      const uint32_t v = o[i];
      uint32_t j = i;
      while (j > 0 && o[j - 1] > v) {
        o[j] = o[j - 1];
        --j;
      }
      o[j] = v;
    }
  }
}

// Bitonic sort of s[0, n2) ascending (n2 a power of two), all threads.
template <int Block>
GB_DEV void lds_bitonic(uint32_t* s, uint32_t n2) {
  for (uint32_t size = 2; size <= n2; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = threadIdx.x; i < n2 / 2; i += Block) {
        const uint32_t lo = 2 * i - (i & (stride - 1));  // lower index of the pair
        const uint32_t hi = lo + stride;
        const bool up = (lo & size) == 0;
        const uint32_t x = s[lo], y = s[hi];
        if ((x > y) == up) {
          s[lo] = y;
          s[hi] = x;
        }
      }
      __syncthreads();
    }
  }
}

// Merge of sorted runs a[0, na) and b[0, nb) into out, all threads of the
// block: each thread finds its stretch of the output by a merge-path search.
template <int Block>
GB_DEV void block_merge(const uint32_t* a, uint32_t na, const uint32_t* b, uint32_t nb, uint32_t* out) {
  const uint32_t total = na + nb;
  const uint32_t per = (total + Block - 1) / Block;
  const uint32_t d0 = threadIdx.x * per < total ? threadIdx.x * per : total;
  const uint32_t d1 = d0 + per < total ? d0 + per : total;
  // smallest i in [max(0, d0 - nb), min(d0, na)] with a[i] > b[d0 - 1 - i] (ties taken from a first)
  uint32_t lo = d0 > nb ? d0 - nb : 0, hi = d0 < na ? d0 : na;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (a[mid] <= b[d0 - 1 - mid]) lo = mid + 1; else hi = mid;
  }
  uint32_t i = lo, j = d0 - lo;
  for (uint32_t d = d0; d < d1; ++d) {
    if (j >= nb || (i < na && a[i] <= b[j])) out[d] = a[i++];
    else out[d] = b[j++];
  }
}

// Pass 4b: one workgroup per listed cell.  Up to kLdsCell pairs: a bitonic
// sort in LDS.  Larger cells: runs of kLdsCell sorted in LDS, then merged
// pairwise through the scratch buffer (the cell's own stretch of it).
template <int Block>
__global__ __launch_bounds__(Block) void compact_sort_big_kernel(CompactArgs a) {
  __shared__ uint32_t s[kLdsCell];
  if (build_failed(a.ctl)) return;
  const uint32_t nbig = a.ctl->big_n < a.big_cap ? a.ctl->big_n : a.big_cap;
  for (uint32_t w = blockIdx.x; w < nbig; w += gridDim.x) {
    const uint2 e = a.big[w];
    uint32_t* o = a.objs + e.x;
    const uint32_t m = e.y;
    for (uint32_t r0 = 0; r0 < m; r0 += kLdsCell) {
      const uint32_t len = m - r0 < kLdsCell ? m - r0 : kLdsCell;
      uint32_t n2 = 64;
      while (n2 < len) n2 <<= 1;
      for (uint32_t i = threadIdx.x; i < n2; i += Block) s[i] = i < len ? o[r0 + i] : 0xFFFFFFFFu;
      __syncthreads();
      lds_bitonic<Block>(s, n2);
      for (uint32_t i = threadIdx.x; i < len; i += Block) o[r0 + i] = s[i];
      __syncthreads();
    }
    if (m > kLdsCell) {
      uint32_t* src = o;
      uint32_t* dst = a.scratch + e.x;
      for (uint32_t width = kLdsCell; width < m; width <<= 1) {
        for (uint32_t r0 = 0; r0 < m; r0 += 2 * width) {
          const uint32_t na = m - r0 < width ? m - r0 : width;
          const uint32_t nb = m - r0 - na < width ? m - r0 - na : width;
          block_merge<Block>(src + r0, na, src + r0 + na, nb, dst + r0);
        }
        __syncthreads();
        uint32_t* t = src;
        src = dst;
        dst = t;
      }
      if (src != o)
        for (uint32_t i = threadIdx.x; i < m; i += Block) o[i] = src[i];
      __syncthreads();
    }
  }
}

}  // namespace gb
