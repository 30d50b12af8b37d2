// Ray casting over a built grid, the use the grid is made for (Introduction;
// Related Work): each ray's closest triangle, found by walking the cells the
// ray crosses and testing the objects each cell lists (objs[ranges[2c] ..
// ranges[2c + 1])).
//
// Contract (the same result as testing every triangle):
//  * a ray is o + t d, t in [t0, t1]: [0, tmax] clipped to the grid box by
//    the slab test; only hits inside the box count;
//  * the hit test is Moller and Trumbore's in a fixed order of FP32
//    operations (no contraction, IEEE division); a grazing ray
//    (det^2 < 1e-8 |e1|^2 |e2|^2 |d|^2) or a degenerate triangle misses; edges
//    count;
//  * the result is the smallest hit t, then the smallest object id; no hit:
//    t = +inf, id 0xFFFFFFFF.
// The walk goes slab by slab along the ray's dominant axis; in each slab it
// visits every cell the ray can touch there, with the slab's t-interval and
// the cross-section widened by 1/32 of a cell, so rounding in the walk never
// skips a cell the ray passes through.  It stops after the slab in which the
// best hit lies (by the same margin) before the slab's far face: every later
// cell lies beyond that hit.
#pragma once

#include "grid.hpp"

namespace gb {

constexpr float kGrazingRay = 1e-8f;
constexpr float kWalkPad = 1.0f / 32.0f;   // cells

GB_DEV float dot3r(const float a[3], const float b[3]) {
  float s = __fmul_rn(a[0], b[0]);
  s = __fadd_rn(s, __fmul_rn(a[1], b[1]));
  return __fadd_rn(s, __fmul_rn(a[2], b[2]));
}

GB_DEV void cross3r(const float a[3], const float b[3], float r[3]) {
  r[0] = __fsub_rn(__fmul_rn(a[1], b[2]), __fmul_rn(a[2], b[1]));
  r[1] = __fsub_rn(__fmul_rn(a[2], b[0]), __fmul_rn(a[0], b[2]));
  r[2] = __fsub_rn(__fmul_rn(a[0], b[1]), __fmul_rn(a[1], b[0]));
}

// Hit parameter of ray (o, d) with triangle (v0, v1, v2), or +inf.
GB_DEV float ray_tri(const float o[3], const float d[3], const float v0[3], const float v1[3], const float v2[3]) {
  float e1[3], e2[3], s[3], p[3], q[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    e1[a] = __fsub_rn(v1[a], v0[a]);
    e2[a] = __fsub_rn(v2[a], v0[a]);
    s[a] = __fsub_rn(o[a], v0[a]);
  }
  cross3r(d, e2, p);
  float det = dot3r(e1, p);
  const float lim = __fmul_rn(__fmul_rn(__fmul_rn(dot3r(e1, e1), dot3r(e2, e2)), dot3r(d, d)), kGrazingRay);
  if (!(__fmul_rn(det, det) >= lim) || det == 0.0f) return __builtin_inff();
  float u = dot3r(s, p);
  cross3r(s, e1, q);
  float v = dot3r(d, q);
  float tn = dot3r(e2, q);
  if (det < 0.0f) {
    det = -det;
    u = -u;
    v = -v;
    tn = -tn;
  }
  if (!(u >= 0.0f && v >= 0.0f && __fadd_rn(u, v) <= det)) return __builtin_inff();
  return __fdiv_rn(tn, det);
}

// Triangles of a cell loaded together (two: 74 VGPRs, six waves per SIMD;
// four measured no faster with five).
constexpr int kRayGroup = 2;

struct RaycastArgs {
  GridDev g;                // verts, tris, nverts, lo, inv, res
  float hi[3];
  const uint32_t* ranges;   // [2R]
  const uint32_t* objs;     // [NO]
  const float* rays;        // [6][nrays]
  uint32_t nrays;
  float tmax;
  float* hit_t;             // [nrays]
  uint32_t* hit_obj;        // [nrays]
};

template <int Block>
__global__ __launch_bounds__(Block) void raycast_kernel(RaycastArgs a) {
  const uint32_t r = blockIdx.x * Block + threadIdx.x;
  if (r >= a.nrays) return;
  const GridDev& G = a.g;
  float o[3], d[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    o[k] = a.rays[static_cast<uint64_t>(k) * a.nrays + r];
    d[k] = a.rays[static_cast<uint64_t>(3 + k) * a.nrays + r];
  }
  float best = __builtin_inff();
  uint32_t best_id = 0xFFFFFFFFu;
  // [t0, t1]: [0, tmax] clipped to the box (the contract's slab test)
  float t0 = 0.0f, t1 = a.tmax;
  bool live = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (d[k] != 0.0f) {
      const float ta = __fdiv_rn(__fsub_rn(G.lo[k], o[k]), d[k]);
      const float tb = __fdiv_rn(__fsub_rn(a.hi[k], o[k]), d[k]);
      t0 = fmaxf(t0, fminf(ta, tb));
      t1 = fminf(t1, fmaxf(ta, tb));
    } else if (!(o[k] >= G.lo[k] && o[k] <= a.hi[k])) {
      live = false;
    }
  }
  live = live && t0 <= t1;
  // the dominant axis m and the two others
  const float ad0 = fabsf(d[0]), ad1 = fabsf(d[1]), ad2 = fabsf(d[2]);
  const int m = (ad0 >= ad1 && ad0 >= ad2) ? 0 : (ad1 >= ad2 ? 1 : 2);
  live = live && d[m] != 0.0f;
  if (live) {
    const int a1 = m == 0 ? 1 : 0, a2 = m == 2 ? 1 : 2;
    const float w = __fdiv_rn(__fsub_rn(a.hi[m], G.lo[m]), static_cast<float>(G.res[m]));  // slab width
    const float wt = fabsf(w / d[m]);                                                         // in t
    const int rm = static_cast<int>(G.res[m]) - 1;
    auto slab_of = [&](float t) {
      const float c = floorf((o[m] + t * d[m] - G.lo[m]) * G.inv[m]);
      return static_cast<int>(fminf(fmaxf(c, 0.0f), static_cast<float>(rm)));
    };
    const int step = d[m] > 0.0f ? 1 : -1;
    int k = slab_of(t0) - step;                 // one slab early: rounding may misplace the entry
    k = k < 0 ? 0 : (k > rm ? rm : k);
    int kend = slab_of(t1) + step;
    kend = kend < 0 ? 0 : (kend > rm ? rm : kend);
    const uint32_t rx = G.res[0], rxy = G.res[0] * G.res[1];
    while (true) {
      const float pa = G.lo[m] + static_cast<float>(k) * w;
      const float ta = (pa - o[m]) / d[m], tb = (pa + w - o[m]) / d[m];
      const float te = fmaxf(ta, tb);
      const float ps = fmaxf(t0, fminf(ta, tb) - kWalkPad * wt);
      const float pe = fminf(t1, te + kWalkPad * wt);
      if (ps <= pe) {
        int lo1, hi1, lo2, hi2;
        {
          const float c0 = o[a1] + ps * d[a1], c1 = o[a1] + pe * d[a1];
          const float f0 = floorf((fminf(c0, c1) - G.lo[a1]) * G.inv[a1] - kWalkPad);
          const float f1 = floorf((fmaxf(c0, c1) - G.lo[a1]) * G.inv[a1] + kWalkPad);
          const float r1 = static_cast<float>(G.res[a1] - 1);
          lo1 = static_cast<int>(fminf(fmaxf(f0, 0.0f), r1));
          hi1 = static_cast<int>(fminf(fmaxf(f1, 0.0f), r1));
        }
        {
          const float c0 = o[a2] + ps * d[a2], c1 = o[a2] + pe * d[a2];
          const float f0 = floorf((fminf(c0, c1) - G.lo[a2]) * G.inv[a2] - kWalkPad);
          const float f1 = floorf((fmaxf(c0, c1) - G.lo[a2]) * G.inv[a2] + kWalkPad);
          const float r2 = static_cast<float>(G.res[a2] - 1);
          lo2 = static_cast<int>(fminf(fmaxf(f0, 0.0f), r2));
          hi2 = static_cast<int>(fminf(fmaxf(f1, 0.0f), r2));
        }
        for (int j2 = lo2; j2 <= hi2; ++j2) {
          for (int j1 = lo1; j1 <= hi1; ++j1) {
            uint32_t xyz[3];
            xyz[m] = static_cast<uint32_t>(k);
            xyz[a1] = static_cast<uint32_t>(j1);
            xyz[a2] = static_cast<uint32_t>(j2);
            const uint64_t c = xyz[0] + rx * xyz[1] + static_cast<uint64_t>(rxy) * xyz[2];
            const uint32_t b = a.ranges[2 * c], e = a.ranges[2 * c + 1];
            // the cell's triangles kRayGroup at a time: their ids, then their vertex
            // indices, then their vertices are each loaded together (the closest
            // hit, by t and then id, does not depend on the order of the tests)
            for (uint32_t i0 = b; i0 < e; i0 += kRayGroup) {
              uint32_t tt[kRayGroup], vi[kRayGroup][3];
              bool ok[kRayGroup];
#pragma unroll
              for (int u = 0; u < kRayGroup; ++u) {
                ok[u] = i0 + u < e;
                tt[u] = ok[u] ? a.objs[i0 + u] : 0u;
                ok[u] = ok[u] && tt[u] < G.ntris;  // an object id this scene does not have: never hit
              }
#pragma unroll
              for (int u = 0; u < kRayGroup; ++u) {
                const uint32_t* tri = G.tris + 3 * static_cast<uint64_t>(ok[u] ? tt[u] : 0u);
#pragma unroll
                for (int jj = 0; jj < 3; ++jj) vi[u][jj] = ok[u] ? tri[jj] : 0u;
                ok[u] = ok[u] && vi[u][0] < G.nverts && vi[u][1] < G.nverts && vi[u][2] < G.nverts;
              }
              float v[kRayGroup][3][3];
#pragma unroll
              for (int u = 0; u < kRayGroup; ++u)
#pragma unroll
                for (int jj = 0; jj < 3; ++jj)
#pragma unroll
                  for (int q = 0; q < 3; ++q)
                    v[u][jj][q] = ok[u] ? G.verts[static_cast<uint64_t>(q) * G.nverts + vi[u][jj]] : 0.0f;
#pragma unroll
              for (int u = 0; u < kRayGroup; ++u) {
                if (!ok[u]) continue;
                const float th = ray_tri(o, d, v[u][0], v[u][1], v[u][2]);
                const uint32_t t = tt[u];
                if (th >= t0 && th <= t1 && (th < best || (th == best && t < best_id))) {
                  best = th;
                  best_id = t;
                }
              }
            }
          }
        }
      }
      // a hit before this slab's far face (by the walk's margin) ends the walk
      if (best <= te - kWalkPad * wt || k == kend) break;
      k += step;
    }
  }
  a.hit_t[r] = best;
  a.hit_obj[r] = best_id;
}

}  // namespace gb
