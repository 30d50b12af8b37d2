/* The tile-owner table the count and the plan kernel write together, rebuilt on
 * the host from the same index function (owned_tiles) and compared with brute
 * force: entry j must be the object whose pairs hold pair j * 2^shift, for
 * every expansion tile, however large an object is; and the runs left for the
 * plan kernel must stay within tfo_work_cap.  Exits 0 and prints "ok" on success. */
#include <stdint.h>
#include <stdio.h>

#include <algorithm>
#include <vector>

#include "tiles.hpp"

#define CHECK(c, msg) do { if (!(c)) { fprintf(stderr, "FAIL: %s (trial %d)\n", msg, trial); return 1; } } while (0)

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t next_u64() {  // splitmix64
  uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

int main() {
  const uint32_t shifts[] = {2, 5, 12};
  for (int trial = 0; trial < 300; ++trial) {
    const uint32_t shift = shifts[trial % 3];
    const uint64_t tile = uint64_t{1} << shift;
    const uint32_t nobj = 1 + static_cast<uint32_t>(next_u64() % 3000);
    std::vector<uint64_t> count(nobj), start(nobj);
    uint64_t total = 0;
    for (uint32_t t = 0; t < nobj; ++t) {
      const uint64_t r = next_u64() % 100;
      // mostly small boxes, some spanning many tiles (beyond the inline entries)
      count[t] = r < 90 ? 1 + next_u64() % 12 : r < 98 ? 1 + next_u64() % (8 * tile) : 1 + next_u64() % (200 * tile);
      start[t] = total;
      total += count[t];
    }
    const uint64_t ntiles = (total + tile - 1) / tile;
    const uint32_t ntfo = static_cast<uint32_t>(ntiles + 1 + (trial % 2) * 7);  // the layout keeps at least one spare entry
    std::vector<int64_t> tfo(ntfo, -1);
    struct Run { uint32_t t; uint64_t lo, hi; };
    std::vector<Run> runs;
    for (uint32_t t = 0; t < nobj; ++t) {
      const gb::OwnedTiles o = gb::owned_tiles(start[t], count[t], shift, ntfo);
      if (!o.any) continue;
      CHECK(o.lo <= o.inl && o.inl <= o.hi && o.hi < ntfo, "run bounds");
      CHECK(o.inl - o.lo + 1 <= gb::kTfoInline, "inline entries");
      for (uint64_t j = o.lo; j <= o.inl; ++j) {
        CHECK(tfo[j] == -1, "entry written twice");
        tfo[j] = t;
      }
      if (o.inl < o.hi) runs.push_back({t, o.inl + 1, o.hi});
    }
    CHECK(runs.size() <= gb::tfo_work_cap(ntfo), "runs beyond the work list");
    for (const Run& r : runs)
      for (uint64_t j = r.lo; j <= r.hi; ++j) {
        CHECK(tfo[j] == -1, "run entry written twice");
        tfo[j] = r.t;
      }
    for (uint64_t j = 0; j < ntiles; ++j) {
      const uint64_t p = j * tile;  // owner of pair p: the last object starting at or before it
      const uint64_t owner = static_cast<uint64_t>(std::upper_bound(start.begin(), start.end(), p) - start.begin()) - 1;
      CHECK(tfo[j] == static_cast<int64_t>(owner), "tile owner");
    }
    for (uint64_t j = ntiles; j < ntfo; ++j) CHECK(tfo[j] == -1, "entry past the last tile");
    // an empty object owns nothing, and nothing is owned past the table
    CHECK(!gb::owned_tiles(5 * tile, 0, shift, ntfo).any, "empty object");
    CHECK(!gb::owned_tiles(uint64_t{ntfo} * tile, 3 * tile, shift, ntfo).any, "past the table");
  }
  printf("ok\n");
  return 0;
}
