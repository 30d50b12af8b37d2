// Shared device building blocks for the gfx950 grid builder: wave64 scans on
// DPP, match-by-ballot, block scans through LDS and decoupled look-back status
// words (Merrill & Garland's single-pass scan).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define GB_DEV __device__ __forceinline__

namespace gb {

constexpr int kWave = 64;

// Look-back status word: flag in the top two bits, value in the low 62.
constexpr uint64_t kFlagInvalid = 0;
constexpr uint64_t kFlagAggregate = 1;
constexpr uint64_t kFlagPrefix = 2;
constexpr uint64_t kValueMask = (uint64_t{1} << 62) - 1;

// Device-side control block at the head of every workspace.
struct Control {
  uint32_t tile_counter[16];   // dynamic tile ids, one per kernel of the sequence
  uint64_t npairs;             // NO, written by the last count tile
  uint32_t error;              // bit 0: bad vertex index
  uint32_t cap_flag;           // set when some grid's NO exceeds its capacity
  uint64_t scratch[4];
  uint64_t kept;               // culled builds: pairs that survive the overlap test
  uint64_t box_npairs;         // culled builds: the box pair count (npairs then holds the kept count)
  uint32_t tfo_work_n;         // tile-owner runs left for the plan kernel to write
  uint32_t big_n;              // compact builds: cells listed for the workgroup sort
};
constexpr uint32_t kErrBadIndex = 1u;
constexpr uint32_t kErrInternal = 2u;  // an internal consistency check failed (the build's output is invalid)

// After the count, a build whose inputs were rejected on the device (a bad
// vertex index, a pair count above capacity) writes nothing more: every later
// kernel checks this first.  Host-synchronised builds never get here with an
// error; builds launched without a readback rely on it.
GB_DEV bool build_failed(const Control* c) { return (c->error | c->cap_flag) != 0; }

GB_DEV uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// Number of set bits of m at lanes below this one.
GB_DEV uint32_t mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
}

GB_DEV uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// LDS index with one padding word per 32, so blocked accesses (each thread a
// run of K consecutive words, K a power of two) spread over all 32 banks.
GB_DEV uint32_t pad32(uint32_t i) { return i + (i >> 5); }
constexpr int padded(int n) { return n + n / 32; }

template <int Ctrl, int RowMask = 0xf, int BankMask = 0xf>
GB_DEV uint32_t dpp(uint32_t old, uint32_t v) {
  return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(static_cast<int>(old), static_cast<int>(v), Ctrl,
                                                           RowMask, BankMask, false));
}

struct OpAdd {
  static constexpr uint32_t identity = 0;
  GB_DEV uint32_t operator()(uint32_t a, uint32_t b) const { return a + b; }
};
struct OpMax {
  static constexpr uint32_t identity = 0;
  GB_DEV uint32_t operator()(uint32_t a, uint32_t b) const { return a > b ? a : b; }
};

// Inclusive scan across the 64 lanes of a wave (all lanes must be active).
// row_shr 1/2/4/8 scans each row of 16 lanes; row_bcast 15/31 carries row
// totals into the rows above.
template <class Op>
GB_DEV uint32_t wave_inclusive(uint32_t v, Op op) {
  const uint32_t id = Op::identity;
  v = op(v, dpp<0x111>(id, v));
  v = op(v, dpp<0x112>(id, v));
  v = op(v, dpp<0x114>(id, v));
  v = op(v, dpp<0x118>(id, v));
  v = op(v, dpp<0x142, 0xa>(id, v));
  v = op(v, dpp<0x143, 0xc>(id, v));
  return v;
}

GB_DEV uint32_t wave_readlane(uint32_t v, int lane) {
  return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), lane));
}

// 64-bit inclusive sum across a wave, through ds_bpermute (not a hot loop).
GB_DEV uint64_t wave_inclusive_sum64(uint64_t v) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    uint64_t o = __shfl_up(v, d, kWave);
    if (lane >= static_cast<uint32_t>(d)) v += o;
  }
  return v;
}

GB_DEV uint64_t wave_sum64(uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// Lanes of the wave whose digit equals this lane's (and that are valid).
// Per bit: a signed one-bit extract gives 0 or all ones, its ballot gives the
// lanes with the bit set, and each lane collects the lanes that disagree with
// it, n |= ballot ^ bit (a three-input bitwise op per 32-lane half); the
// match is the valid lanes outside n.
template <int Bits>
GB_DEV uint64_t match_digit(uint32_t d, bool valid) {
  const uint64_t vm = ballot(valid);
  // lanes that differ from this one in some bit: n |= ballot ^ bit
  uint32_t nlo = 0, nhi = 0;
#pragma unroll
  for (int b = 0; b < Bits; ++b) {
    // the bit as 0 / all ones, and the wave's lanes that have it set
    uint32_t bit;
    uint64_t bb;
    asm("v_bfe_i32 %0, %1, %2, 1" : "=v"(bit) : "v"(d), "i"(b));
    asm("v_cmp_ne_u32 %0, 0, %1" : "=s"(bb) : "v"(bit));
    // n |= ballot ^ bit: table 0xF6 over (n, ballot, bit), index n * 4 + ballot * 2 + bit
    asm("v_bitop3_b32 %0, %0, %1, %2 bitop3:0xf6" : "+v"(nlo) : "s"(static_cast<uint32_t>(bb)), "v"(bit));
    asm("v_bitop3_b32 %0, %0, %1, %2 bitop3:0xf6" : "+v"(nhi) : "s"(static_cast<uint32_t>(bb >> 32)), "v"(bit));
  }
  return vm & ~((static_cast<uint64_t>(nhi) << 32) | nlo);
}

GB_DEV void status_store(uint64_t* p, uint64_t flag, uint64_t value) {
  __hip_atomic_store(p, (flag << 62) | (value & kValueMask), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
GB_DEV uint64_t status_load(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Decoupled look-back by one full wave over status[tile - 1], status[tile - 2],
// ... (stride apart).  Publishes the tile's aggregate, returns the exclusive
// prefix (the sum of every earlier tile) and publishes the inclusive prefix.
// Every lane returns the same value.
GB_DEV uint64_t lookback_wave(uint64_t* status, uint32_t tile, uint64_t aggregate) {
  const uint32_t lane = lane_id();
  if (tile == 0) {
    if (lane == 0) status_store(status, kFlagPrefix, aggregate);
    return 0;
  }
  if (lane == 0) status_store(status + tile, kFlagAggregate, aggregate);
  uint64_t excl = 0;
  int64_t top = static_cast<int64_t>(tile) - 1;
  while (true) {
    const int64_t idx = top - lane;
    uint64_t s = idx >= 0 ? status_load(status + idx) : (kFlagPrefix << 62);
    const uint64_t flag = s >> 62;
    const uint64_t inval = ballot(flag == kFlagInvalid);
    const uint64_t pref = ballot(flag == kFlagPrefix);
    const uint64_t need = pref ? ((pref & (~pref + 1)) << 1) - 1 : ~uint64_t{0};  // lanes up to first prefix
    if (inval & need) {
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    const uint64_t v = ((need >> lane) & 1u) ? (s & kValueMask) : 0;
    excl += wave_sum64(v);
    if (pref) break;
    top -= kWave;
  }
  if (lane == 0) status_store(status + tile, kFlagPrefix, excl + aggregate);
  return excl;
}

// Look-back words of W bits (64, or 32 while every value fits in 30 bits):
// the flag in the top two bits, the value below.  Half-width words halve
// the look-back's stores and polls.
template <typename W>
GB_DEV void status_put(W* p, uint64_t flag, uint64_t value) {
  constexpr int S = sizeof(W) * 8 - 2;
  const W w = static_cast<W>((flag << S) | (value & ((uint64_t{1} << S) - 1)));
  __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename W>
GB_DEV W status_get(const W* p) {
  return __hip_atomic_load(const_cast<W*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Look-back by one thread along status[(tile - 1) * stride + col], ....
// The nearest predecessor usually holds its inclusive prefix already, so it
// is read alone first; a chain of aggregates is then read four tiles per
// round, one memory latency per four tiles.
template <typename W>
GB_DEV uint64_t lookback_thread(W* status, uint32_t stride, uint32_t col, uint32_t tile) {
  constexpr int kAhead = 4;
  constexpr int S = sizeof(W) * 8 - 2;
  constexpr W kMask = static_cast<W>((uint64_t{1} << S) - 1);
  uint64_t excl = 0;
  int64_t j = static_cast<int64_t>(tile) - 1;
  if (j < 0) return 0;
  {
    const W s = status_get(status + static_cast<uint64_t>(j) * stride + col);
    const W flag = s >> S;
    if (flag == kFlagPrefix) return s & kMask;
    if (flag == kFlagAggregate) {
      excl = s & kMask;
      --j;
    }
  }
  while (j >= 0) {
    W s[kAhead];
#pragma unroll
    for (int u = 0; u < kAhead; ++u)
      s[u] = j - u >= 0 ? status_get(status + static_cast<uint64_t>(j - u) * stride + col)
                        : static_cast<W>(static_cast<W>(kFlagPrefix) << S);
    bool done = false, stalled = false;
#pragma unroll
    for (int u = 0; u < kAhead; ++u) {
      if (done || stalled) continue;
      const W flag = s[u] >> S;
      if (flag == kFlagInvalid) {
        stalled = true;
      } else {
        excl += s[u] & kMask;
        --j;
        if (flag == kFlagPrefix) done = true;
      }
    }
    if (done) break;
    if (stalled) __builtin_amdgcn_s_sleep(1);
  }
  return excl;
}

// Dynamic tile id: tiles are handed out in launch order, so every tile a
// look-back waits for already belongs to a running workgroup.
GB_DEV uint32_t next_tile(uint32_t* counter, uint32_t* lds_slot) {
  if (threadIdx.x == 0) *lds_slot = atomicAdd(counter, 1u);
  __syncthreads();
  const uint32_t t = *lds_slot;
  __syncthreads();
  return t;
}

// Exclusive block-wide sum of one uint32 per thread; also returns the total.
// wave_tot must hold Block / 64 entries of LDS.
template <int Block>
GB_DEV uint32_t block_exclusive_sum(uint32_t v, uint32_t* wave_tot, uint32_t& total) {
  constexpr int kWaves = Block / kWave;
  const uint32_t lane = lane_id();
  const uint32_t w = threadIdx.x / kWave;
  const uint32_t inc = wave_inclusive(v, OpAdd{});
  if (lane == kWave - 1) wave_tot[w] = inc;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    const uint32_t x = wave_tot[i];
    before += (static_cast<uint32_t>(i) < w) ? x : 0u;
    tot += x;
  }
  __syncthreads();
  total = tot;
  return before + inc - v;
}

// Inclusive block-wide max of one uint32 per thread (wave_tot: Block / 64 LDS).
template <int Block>
GB_DEV uint32_t block_inclusive_max(uint32_t v, uint32_t* wave_tot) {
  constexpr int kWaves = Block / kWave;
  const uint32_t lane = lane_id();
  const uint32_t w = threadIdx.x / kWave;
  const uint32_t inc = wave_inclusive(v, OpMax{});
  if (lane == kWave - 1) wave_tot[w] = inc;
  __syncthreads();
  uint32_t before = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    const uint32_t x = wave_tot[i];
    if (static_cast<uint32_t>(i) < w) before = before > x ? before : x;
  }
  __syncthreads();
  return before > inc ? before : inc;
}

// Exclusive block-wide max of one uint32 per thread (0 for thread 0).
template <int Block>
GB_DEV uint32_t block_exclusive_max(uint32_t v, uint32_t* wave_tot) {
  constexpr int kWaves = Block / kWave;
  const uint32_t lane = lane_id();
  const uint32_t w = threadIdx.x / kWave;
  const uint32_t inc = wave_inclusive(v, OpMax{});
  uint32_t ex = __shfl_up(inc, 1, kWave);
  if (lane == 0) ex = 0;
  if (lane == kWave - 1) wave_tot[w] = inc;
  __syncthreads();
  uint32_t before = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    const uint32_t x = wave_tot[i];
    if (static_cast<uint32_t>(i) < w) before = before > x ? before : x;
  }
  __syncthreads();
  return before > ex ? before : ex;
}

// Exclusive block-wide sum of one uint64 per thread; also returns the total.
template <int Block>
GB_DEV uint64_t block_exclusive_sum64(uint64_t v, uint64_t* wave_tot, uint64_t& total) {
  constexpr int kWaves = Block / kWave;
  const uint32_t lane = lane_id();
  const uint32_t w = threadIdx.x / kWave;
  const uint64_t inc = wave_inclusive_sum64(v);
  if (lane == kWave - 1) wave_tot[w] = inc;
  __syncthreads();
  uint64_t before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    const uint64_t x = wave_tot[i];
    before += (static_cast<uint32_t>(i) < w) ? x : 0u;
    tot += x;
  }
  __syncthreads();
  total = tot;
  return before + inc - v;
}

}  // namespace gb
