// Which entries of the expansion's tile-owner table an object writes (host
// and device: the count kernel runs it, and a host test checks it against
// brute force).  Entry j of the table is the object that owns pair j * 2^shift,
// the first pair of expansion tile j.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gb {

// Table entries the count writes itself for one object; the rest of a longer
// run is left to the plan kernel, whose whole workgroup fills it.
constexpr uint32_t kTfoInline = 32;

// An object whose pairs are [first, first + count) owns the first pair of the
// expansion tiles ceil(first / 2^shift) .. floor((first + count - 1) / 2^shift);
// the table holds those below ntfo.  The count writes entries [lo, inl] and
// leaves (inl, hi] as one run for the plan kernel.
struct OwnedTiles {
  uint64_t lo, inl, hi;
  bool any;
};

__host__ __device__ inline OwnedTiles owned_tiles(uint64_t first, uint64_t count, uint32_t shift, uint64_t ntfo) {
  OwnedTiles r{0, 0, 0, false};
  if (count == 0 || ntfo == 0) return r;
  const uint64_t mask = (uint64_t{1} << shift) - 1;
  const uint64_t lo = (first + mask) >> shift;
  const uint64_t last = (first + count - 1) >> shift;
  if (lo > last || lo >= ntfo) return r;
  r.any = true;
  r.lo = lo;
  r.hi = last < ntfo ? last : ntfo - 1;
  r.inl = lo + kTfoInline - 1 < r.hi ? lo + kTfoInline - 1 : r.hi;
  return r;
}

// Runs left for the plan kernel: only objects that own more than kTfoInline
// tiles leave one, and objects own disjoint tiles, so fewer than
// ntfo / kTfoInline of them.
__host__ __device__ inline uint32_t tfo_work_cap(uint32_t ntfo) { return ntfo / kTfoInline + 2; }

}  // namespace gb
