// One pass of the LSD radix sort (RadixSort of Algorithm 1), in the
// single-pass "onesweep" form (Adinets & Merrill): each tile ranks its keys by
// one digit in LDS, obtains every digit's global offset by a decoupled
// look-back over the tiles before it, and scatters through an LDS staging
// buffer so each digit's run is written contiguously.
#pragma once

#include <type_traits>

#include "ranges.hpp"

namespace gb {

enum SortSource : int { kFromArrays = 0, kFromExpansion = 1 };
enum SortSink : int { kToArrays = 0, kToGrids = 1 };

struct SortPassArgs {
  const uint32_t* keys_in;  // kFromArrays
  const uint32_t* vals_in;
  uint32_t* keys_out;       // kToArrays
  uint32_t* vals_out;
  ExpandArgs ex;            // kFromExpansion (and grid table for kToGrids)
  const uint32_t* hist;     // global digit histogram of this pass [radix]
  uint64_t* status;         // [ntiles][radix] look-back words (zeroed)
  uint32_t narrow;          // 1: launch the 32-bit look-back word kernel (every pass value below 2^30)
  uint64_t n;               // pairs, when not read from the control block
  uint32_t n_from_ctl;      // 1: n = ctl->npairs
  uint32_t hist_copies;     // the pass's digit histogram is the sum of this many copies ...
  uint32_t hist_stride;     // ... hist_stride words apart
  uint32_t shift;
  uint32_t width;           // digit width of this pass (<= RB)
  uint32_t counter;         // tile-counter slot
  const GridSink* sink;     // kToGrids: each grid's outputs, first pair and first cell
  const uint2* kmap;        // kToGrids: key bucket -> (first, last) grid
  const GridSink* ksink;    // kToGrids: key bucket -> its first grid's sink (straddles: search)
  uint32_t kshift;          // kToGrids: key bucket = key >> kshift
  Control* ctl;
};

// Waves per SIMD asked of the register allocator: four (at most 128 VGPRs)
// when the keys come from arrays, except for the 16-key shapes with the widest
// digits, whose rank needs more registers (three waves at 256 threads, two at
// 512 with 11-bit digits); the regenerating variant runs two.
constexpr int onesweep_waves(int Block, int K, int RB, int Source) {
  return Source != kFromArrays ? 2
         : (Block == 256 && K == 16 && RB >= 10) ? 3
         : (Block == 512 && K == 16 && RB >= 11) ? 2
         : 4;
}

// Narrow: 32-bit look-back words (flag and a 30-bit value), for passes of
// fewer than 2^30 pairs; 64-bit words otherwise.
template <int Block, int K, int RB, int Source, int Sink, bool Batched, bool Narrow = false>
__global__ __launch_bounds__(Block, onesweep_waves(Block, K, RB, Source)) void onesweep_kernel(SortPassArgs a) {
  using SW = typename std::conditional<Narrow, uint32_t, uint64_t>::type;
  SW* const status = reinterpret_cast<SW*>(a.status);
  constexpr int N = Block * K;
  constexpr int R = 1 << RB;
  constexpr int W = Block / kWave;
  constexpr int DPT = R > Block ? R / Block : 1;        // digits per thread
  // staging (keys then values) doubles as the per-wave digit counters and the
  // expansion's owner slots
  constexpr int kStage0 = 2 * N > W * R ? 2 * N : W * R;
  // also the expansion's padded slots and, when regenerating, its padded transpose
  constexpr int kStage1 = Source == kFromExpansion ? 2 * padded(N) : padded(N);
  constexpr int kStage = kStage0 > kStage1 ? kStage0 : kStage1;
  __shared__ uint32_t s_stage[kStage];
  __shared__ uint32_t s_tile_excl[R];
  __shared__ uint32_t s_dst[R];
  __shared__ uint32_t s_wtot[W];
  __shared__ uint32_t s_tile;

  if (a.n_from_ctl && build_failed(a.ctl)) return;
  const uint64_t n = a.n_from_ctl ? a.ctl->npairs : a.n;
  const uint32_t ntiles = static_cast<uint32_t>((n + N - 1) / N);
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = lane_id();
  const uint32_t w = tid / kWave;
  const uint32_t dmask = (1u << a.width) - 1u;

  while (true) {
    const uint32_t tile = next_tile(&a.ctl->tile_counter[a.counter], &s_tile);
    if (tile >= ntiles) break;
    const uint64_t base = static_cast<uint64_t>(tile) * N;
    const uint32_t nt = static_cast<uint32_t>(n - base < N ? n - base : N);

    uint32_t keys[K], vals[K];
    if constexpr (Source == kFromExpansion) {
      // blocked expansion (GlobalCoords stepped along each thread's slots),
      // then through LDS into the wave-striped order the stable rank needs
      expand_tile<Block, K, Batched, kBlocked>(a.ex, tile, n, ntiles, s_stage, s_wtot, keys, vals);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        s_stage[pad32(tid * K + k)] = keys[k];
        s_stage[padded(N) + pad32(tid * K + k)] = vals[k];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const uint32_t slot = w * (kWave * K) + k * kWave + lane;
        keys[k] = s_stage[pad32(slot)];
        vals[k] = s_stage[padded(N) + pad32(slot)];
      }
      __syncthreads();  // s_stage becomes the rank's counters
    } else {
      // branch-free loads (the tail re-reads the last element) keep all of
      // them in flight at once; the values are loaded after the rank, which
      // does not need them
      const uint32_t* kin = a.keys_in + base + w * (kWave * K) + lane;
      if (nt == static_cast<uint32_t>(N)) {
#pragma unroll
        for (int k = 0; k < K; ++k) keys[k] = kin[k * kWave];  // full tile: constant offsets
      } else {
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const uint32_t idx = w * (kWave * K) + k * kWave + lane;
          keys[k] = a.keys_in[base + (idx < nt ? idx : nt - 1)];
        }
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const uint32_t idx = w * (kWave * K) + k * kWave + lane;
        if (idx >= nt) keys[k] = 0xFFFFFFFFu;
      }
    }

    // ---- rank: per-wave digit counters, items of a wave taken in order ----
    uint32_t* s_cnt = s_stage;  // [W][R]
    for (int i = lane; i < R; i += kWave) s_cnt[w * R + i] = 0;
    __builtin_amdgcn_wave_barrier();
    uint32_t rank[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint32_t idx = w * (kWave * K) + k * kWave + lane;
      const bool valid = idx < nt;
      const uint32_t d = (keys[k] >> a.shift) & dmask;
      const uint64_t peers = match_digit<RB>(d, valid);
      const uint32_t below = mbcnt(peers);
      const uint32_t c = valid ? s_cnt[w * R + d] : 0u;
      __builtin_amdgcn_wave_barrier();
      if (valid && below == 0) s_cnt[w * R + d] = c + static_cast<uint32_t>(__builtin_popcountll(peers));
      __builtin_amdgcn_wave_barrier();
      rank[k] = c + below;
    }
    if constexpr (Source == kFromArrays) {
      const uint32_t* vin = a.vals_in + base + w * (kWave * K) + lane;
      if (nt == static_cast<uint32_t>(N)) {
#pragma unroll
        for (int k = 0; k < K; ++k) vals[k] = vin[k * kWave];
      } else {
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const uint32_t idx = w * (kWave * K) + k * kWave + lane;
          vals[k] = a.vals_in[base + (idx < nt ? idx : nt - 1)];
        }
      }
    }
    __syncthreads();

    // ---- per digit: prefix over waves, tile total, publish aggregate ----
    uint32_t dcount[DPT];
    uint32_t tsum = 0;
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
      const uint32_t d = tid * DPT + j;
      uint32_t run = 0;
      if (d < static_cast<uint32_t>(R)) {
#pragma unroll
        for (int ww = 0; ww < W; ++ww) {
          const uint32_t c = s_cnt[ww * R + d];
          s_cnt[ww * R + d] = run;
          run += c;
        }
        if (tile == 0) {
          // tile 0 starts each digit at the digit's global offset
        } else {
          status_put(status + static_cast<uint64_t>(tile) * R + d, kFlagAggregate, run);
        }
      }
      dcount[j] = run;
      tsum += run;
    }
    uint32_t ttot;
    const uint32_t texcl0 = block_exclusive_sum<Block>(tsum, s_wtot, ttot);
    {
      uint32_t texcl = texcl0;
#pragma unroll
      for (int j = 0; j < DPT; ++j) {
        const uint32_t d = tid * DPT + j;
        if (d < static_cast<uint32_t>(R)) s_tile_excl[d] = texcl;
        texcl += dcount[j];
      }
    }
    __syncthreads();

    // ---- local positions, then stage keys and values in digit order ----
    uint32_t pos[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint32_t d = (keys[k] >> a.shift) & dmask;
      pos[k] = s_tile_excl[d] + s_cnt[w * R + d] + rank[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint32_t idx = w * (kWave * K) + k * kWave + lane;
      if (idx < nt) {
        s_stage[pos[k]] = keys[k];
        s_stage[N + pos[k]] = vals[k];
      }
    }

    // ---- global digit offsets: tile 0 from the histogram, others by look-back ----
    if (tile == 0) {
      uint32_t hsum = 0, hv[DPT];
#pragma unroll
      for (int j = 0; j < DPT; ++j) {
        const uint32_t d = tid * DPT + j;
        uint32_t h = 0;
        if (d < static_cast<uint32_t>(R))
          for (uint32_t c = 0; c < a.hist_copies; ++c) h += a.hist[c * a.hist_stride + d];
        hv[j] = h;
        hsum += hv[j];
      }
      uint32_t htot;
      uint32_t hex = block_exclusive_sum<Block>(hsum, s_wtot, htot);
      uint32_t texcl = texcl0;
#pragma unroll
      for (int j = 0; j < DPT; ++j) {
        const uint32_t d = tid * DPT + j;
        if (d < static_cast<uint32_t>(R)) {
          status_put(status + d, kFlagPrefix, static_cast<uint64_t>(hex) + dcount[j]);
          s_dst[d] = hex - texcl;
        }
        hex += hv[j];
        texcl += dcount[j];
      }
    } else {
      uint32_t texcl = texcl0;
#pragma unroll
      for (int j = 0; j < DPT; ++j) {
        const uint32_t d = tid * DPT + j;
        if (d < static_cast<uint32_t>(R)) {
          const uint64_t ex = lookback_thread(status, R, d, tile);
          status_put(status + static_cast<uint64_t>(tile) * R + d, kFlagPrefix, ex + dcount[j]);
          s_dst[d] = static_cast<uint32_t>(ex) - texcl;
        }
        texcl += dcount[j];
      }
    }
    __syncthreads();

    // ---- scatter: consecutive threads write consecutive slots of a digit run ----
    if constexpr (Sink == kToArrays) {
      for (uint32_t i = tid; i < nt; i += Block) {
        const uint32_t key = s_stage[i];
        const uint32_t val = s_stage[N + i];
        const uint32_t d = (key >> a.shift) & dmask;
        const uint32_t dst = s_dst[d] + i;
        a.keys_out[dst] = key;
        a.vals_out[dst] = val;
      }
    } else {
      // batched: each slot's grid comes from the key map and the grid's
      // output descriptor; the lookups of C slots are in flight together
      constexpr int C = 4;
      for (uint32_t i0 = tid; i0 < nt; i0 += C * Block) {
        uint32_t kk[C], vv[C];
        GridSink sk[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const uint32_t i = i0 + c * Block;
          const uint32_t ii = i < nt ? i : nt - 1;  // past the tail: a valid slot, nothing stored
          kk[c] = s_stage[ii];
          vv[c] = s_stage[N + ii];
          sk[c] = a.ksink[kk[c] >> a.kshift];
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
          if (sk[c].straddles) {  // a bucket a grid boundary crosses (rare)
            const uint2 km = a.kmap[kk[c] >> a.kshift];
            sk[c] = a.sink[sink_of_key(a.sink, kk[c], km.x, km.y)];
          }
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
          const uint32_t i = i0 + c * Block;
          if (i < nt) {
            const uint32_t dst = s_dst[(kk[c] >> a.shift) & dmask] + i;
            const uint64_t local = dst - sk[c].pair_base;
            sk[c].cells[local] = kk[c] - sk[c].cell_base;
            sk[c].objs[local] = vv[c];
          }
        }
      }
    }
    __syncthreads();
  }
}

// Digit histograms of every pass from keys held in an array (one read).
struct HistArrayArgs {
  const uint32_t* keys;
  uint64_t n;
  SortPlan plan;
  uint32_t* hist;           // [4][kRadixMax]
  uint64_t* sort_status;    // [passes][status_stride], cleared here
  uint64_t status_stride;
  Control* ctl;
};

template <int Block, int K, int RB>
__global__ __launch_bounds__(Block) void hist_array_kernel(HistArrayArgs a) {
  constexpr int N = Block * K;
  constexpr int R = 1 << RB;
  __shared__ uint32_t s_hist[4 * R];
  __shared__ uint32_t s_tile;
  const uint32_t ntiles = static_cast<uint32_t>((a.n + N - 1) / N);
  {
    const uint64_t per_pass = static_cast<uint64_t>(ntiles) * R;
    const uint64_t nwords = static_cast<uint64_t>(a.plan.passes) * per_pass;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * Block + threadIdx.x; i < nwords;
         i += static_cast<uint64_t>(gridDim.x) * Block)
      a.sort_status[(i / per_pass) * a.status_stride + i % per_pass] = 0;
  }
  for (int i = threadIdx.x; i < 4 * R; i += Block) s_hist[i] = 0;
  __syncthreads();
  while (true) {
    const uint32_t tile = next_tile(&a.ctl->tile_counter[kCtrHist], &s_tile);
    if (tile >= ntiles) break;
    const uint64_t base = static_cast<uint64_t>(tile) * N;
    for (int k = 0; k < K; ++k) {
      const uint64_t i = base + static_cast<uint64_t>(k) * Block + threadIdx.x;
      if (i < a.n) {
        const uint32_t key = a.keys[i];
        for (uint32_t p = 0; p < a.plan.passes; ++p)
          atomicAdd(&s_hist[p * R + ((key >> a.plan.shift[p]) & ((1u << a.plan.width[p]) - 1u))], 1u);
      }
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < a.plan.passes * R; i += Block) {
    const uint32_t v = s_hist[i];
    if (v) atomicAdd(&a.hist[(i / R) * kRadixMax + (i % R)], v);
  }
}

}  // namespace gb
