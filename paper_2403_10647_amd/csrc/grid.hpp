// Per-grid parameters as the kernels see them, and the FP32 world -> cell map.
#pragma once

#include "common.hpp"

namespace gb {

struct GridDev {
  const float* verts;      // FP32 [3][nverts]
  const uint32_t* tris;    // uint32 [ntris][3]
  uint32_t* out_cells;     // [cap_pairs]
  uint32_t* out_objs;      // [cap_pairs]
  uint32_t* out_ranges;    // [2 * R]
  uint64_t cap_pairs;
  uint64_t cell_base;      // first cell of this grid in the batch's cell space
  uint32_t nverts;
  uint32_t ntris;
  uint32_t tri_base;       // first triangle of this grid in the batch
  uint32_t res[3];
  float lo[3];
  float inv[3];
};

// Packed cell box of a triangle: lo corner (3 x 10 bits) and extent - 1
// (3 x 10 bits), so one 64-bit word per triangle.
GB_DEV uint64_t pack_box(const uint32_t lo[3], const uint32_t m[3]) {
  return static_cast<uint64_t>(lo[0]) | (static_cast<uint64_t>(lo[1]) << 10) | (static_cast<uint64_t>(lo[2]) << 20) |
         (static_cast<uint64_t>(m[0] - 1) << 30) | (static_cast<uint64_t>(m[1] - 1) << 40) |
         (static_cast<uint64_t>(m[2] - 1) << 50);
}

struct Box {
  uint32_t lo[3];
  uint32_t m[3];
};

GB_DEV Box unpack_box(uint64_t b) {
  Box r;
  r.lo[0] = static_cast<uint32_t>(b) & 1023u;
  r.lo[1] = static_cast<uint32_t>(b >> 10) & 1023u;
  r.lo[2] = static_cast<uint32_t>(b >> 20) & 1023u;
  r.m[0] = (static_cast<uint32_t>(b >> 30) & 1023u) + 1u;
  r.m[1] = (static_cast<uint32_t>(b >> 40) & 1023u) + 1u;
  r.m[2] = (static_cast<uint32_t>(b >> 50) & 1023u) + 1u;
  return r;
}

// One axis of the world -> cell map: min(max(floor((p - lo) * inv), 0), res - 1),
// each step one IEEE FP32 operation (the library is built without contraction).
GB_DEV uint32_t cell_coord(float p, float lo, float inv, uint32_t res_minus_1) {
  const float s = __fsub_rn(p, lo);
  const float u = __fmul_rn(s, inv);
  float f = floorf(u);
  f = fmaxf(f, 0.0f);
  f = fminf(f, static_cast<float>(res_minus_1));
  return static_cast<uint32_t>(f);
}

// GlobalCoords (Section 3) followed by the x-fastest linear cell id.
GB_DEV uint32_t cell_of(const Box& b, uint32_t rid, uint32_t rx, uint32_t rxy) {
  const uint32_t mxy = b.m[0] * b.m[1];
  const uint32_t z = rid / mxy;
  const uint32_t r2 = rid - z * mxy;
  const uint32_t y = r2 / b.m[0];
  const uint32_t x = r2 - y * b.m[0];
  return (b.lo[0] + x) + rx * (b.lo[1] + y) + rxy * (b.lo[2] + z);
}

}  // namespace gb
