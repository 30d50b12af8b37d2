// Single-pass scans over uint32 arrays with decoupled look-back: exclusive
// sum, inclusive max and segmented exclusive sum (the ExclusiveSum,
// InclusiveSum and SegmentedExclusiveSum steps of Algorithm 1).
#pragma once

#include "kernels.hpp"

namespace gb {

// Scan element: 62-bit payload of a look-back word.  For the segmented sum
// bit 61 is "a segment head lies in this range" and bits 0..60 the sum since
// the last head.
struct ScanSum {
  GB_DEV static uint64_t lift(uint32_t v, uint32_t) { return v; }
  GB_DEV static uint64_t op(uint64_t a, uint64_t b) { return (a + b) & kValueMask; }
};
struct ScanMax {
  GB_DEV static uint64_t lift(uint32_t v, uint32_t) { return v; }
  GB_DEV static uint64_t op(uint64_t a, uint64_t b) { return a > b ? a : b; }
};
struct ScanSeg {
  static constexpr uint64_t kHead = uint64_t{1} << 61;
  static constexpr uint64_t kSum = kHead - 1;
  GB_DEV static uint64_t lift(uint32_t v, uint32_t f) { return (f ? kHead : 0) | v; }
  GB_DEV static uint64_t op(uint64_t a, uint64_t b) {
    return (b & kHead) ? b : ((a & kHead) | (((a & kSum) + (b & kSum)) & kSum));
  }
};

// Inclusive scan of a 64-bit payload across a wave, in lane order.
template <class Op>
GB_DEV uint64_t wave_scan_op(uint64_t v) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint64_t o = __shfl_up(v, d, kWave);
    if (lane >= static_cast<uint32_t>(d)) v = Op::op(o, v);
  }
  return v;
}

struct ScanArgs {
  const uint32_t* in;
  const uint32_t* flags;
  uint32_t* out;
  uint64_t n;
  uint64_t* status;
  Control* ctl;
};

// mode: 0 exclusive sum, 1 inclusive max, 2 segmented exclusive sum
template <int Block, int K, class Op, int Mode>
__global__ __launch_bounds__(Block) void scan_kernel(ScanArgs a) {
  constexpr int N = Block * K;
  constexpr int W = Block / kWave;
  __shared__ uint32_t s_v[padded(N)];
  __shared__ uint32_t s_f[Mode == 2 ? padded(N) : 1];
  __shared__ uint64_t s_wave[W];
  __shared__ uint64_t s_prefix;
  __shared__ uint32_t s_tile;
  const uint32_t tile = next_tile(&a.ctl->tile_counter[kCtrScan], &s_tile);
  const uint32_t tid = threadIdx.x;
  const uint64_t base = static_cast<uint64_t>(tile) * N;
  const uint32_t ntiles = static_cast<uint32_t>((a.n + N - 1) / N);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint64_t i = base + k * Block + tid;
    s_v[pad32(k * Block + tid)] = i < a.n ? a.in[i] : 0u;
    if constexpr (Mode == 2) s_f[pad32(k * Block + tid)] = i < a.n ? a.flags[i] : 0u;
  }
  __syncthreads();
  uint64_t agg = Mode == 1 ? 0 : 0;
  uint64_t elem[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    elem[k] = Op::lift(s_v[pad32(tid * K + k)], Mode == 2 ? s_f[Mode == 2 ? pad32(tid * K + k) : 0] : 0u);
    agg = k == 0 ? elem[k] : Op::op(agg, elem[k]);
  }
  // block scan of the per-thread aggregates, in thread order
  const uint64_t winc = wave_scan_op<Op>(agg);
  const uint32_t lane = lane_id(), w = tid / kWave;
  if (lane == kWave - 1) s_wave[w] = winc;
  __syncthreads();
  uint64_t before = 0;
  bool have = false;
  for (uint32_t i = 0; i < w; ++i) {
    before = have ? Op::op(before, s_wave[i]) : s_wave[i];
    have = true;
  }
  uint64_t tile_agg = s_wave[0];
  for (int i = 1; i < W; ++i) tile_agg = Op::op(tile_agg, s_wave[i]);
  uint64_t wex = __shfl_up(winc, 1, kWave);
  // exclusive prefix of this thread inside the tile
  bool has_ex = have || lane > 0;
  uint64_t ex = lane > 0 ? (have ? Op::op(before, wex) : wex) : before;
  __syncthreads();
  if (tid == 0) {
    // serial look-back, oldest contributions combined first
    uint64_t p = 0;
    bool hp = false;
    if (tile == 0) {
      status_store(a.status, kFlagPrefix, tile_agg);
    } else {
      status_store(a.status + tile, kFlagAggregate, tile_agg);
      int64_t j = static_cast<int64_t>(tile) - 1;
      while (j >= 0) {
        const uint64_t s = status_load(a.status + j);
        const uint64_t f = s >> 62;
        if (f == kFlagInvalid) {
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        const uint64_t v = s & kValueMask;
        p = hp ? Op::op(v, p) : v;
        hp = true;
        if (f == kFlagPrefix) break;
        --j;
      }
      status_store(a.status + tile, kFlagPrefix, Op::op(p, tile_agg));
    }
    s_prefix = hp ? p : 0;
    s_tile = hp ? 1u : 0u;
    if (tile == ntiles - 1) a.ctl->scratch[0] = hp ? Op::op(p, tile_agg) : tile_agg;
  }
  __syncthreads();
  const bool hp = s_tile != 0;
  uint64_t run;
  bool hrun;
  if (hp) {
    run = has_ex ? Op::op(s_prefix, ex) : s_prefix;
    hrun = true;
  } else {
    run = ex;
    hrun = has_ex;
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint64_t inc = hrun ? Op::op(run, elem[k]) : elem[k];
    uint32_t o;
    if constexpr (Mode == 0) o = static_cast<uint32_t>(inc - elem[k]);
    else if constexpr (Mode == 1) o = static_cast<uint32_t>(inc);
    else o = static_cast<uint32_t>((inc & ScanSeg::kSum) - (elem[k] & ScanSeg::kSum));
    s_v[pad32(tid * K + k)] = o;
    run = inc;
    hrun = true;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint64_t i = base + k * Block + tid;
    if (i < a.n) a.out[i] = s_v[pad32(k * Block + tid)];
  }
}

}  // namespace gb
