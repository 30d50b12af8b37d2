/* A C caller of the grid library: no Python, no torch.  It builds a grid of a
 * small random triangle soup through the C ABI (gridbuild.h) with device
 * memory it allocates itself, then checks the result against what the grid
 * contract fixes: cells sorted, objects ascending within a cell, every pair's
 * cell inside its triangle's cell box (recomputed here on the host from the
 * same FP32 map), each triangle present exactly box-size times, and the
 * ranges tiling [0, NO).  Prints "ok <NO>" and exits 0 on success. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "gridbuild.h"

#define CHECK(c, msg) do { if (!(c)) { fprintf(stderr, "FAIL: %s\n", msg); return 1; } } while (0)
#define HIPCHK(x) do { if ((x) != hipSuccess) { fprintf(stderr, "HIP error at %s:%d\n", __FILE__, __LINE__); return 2; } } while (0)

static uint32_t lcg(uint64_t* s) { *s = *s * 6364136223846793005ull + 1442695040888963407ull; return (uint32_t)(*s >> 33); }
static float unif(uint64_t* s) { return (float)(lcg(s) & 0xFFFFFF) / 16777216.0f; }

/* the contract's world-to-cell map, FP32, no contraction */
static uint32_t cell_of(float p, float lo, float inv, uint32_t res) {
  volatile float s = p - lo;
  volatile float u = s * inv;
  float f = floorf(u);
  f = fmaxf(f, 0.0f);
  f = fminf(f, (float)(res - 1));
  return (uint32_t)f;
}

int main(void) {
  const uint32_t T = 5000, V = 3 * T;
  const uint32_t res[3] = {37, 21, 29};
  const float lo[3] = {0.f, 0.f, 0.f}, hi[3] = {1.f, 1.f, 1.f};
  float* hv = (float*)malloc(sizeof(float) * 3 * V);
  uint32_t* ht = (uint32_t*)malloc(sizeof(uint32_t) * 3 * T);
  uint64_t seed = 12345;
  for (uint32_t t = 0; t < T; ++t) {
    const float big = (t % 50 == 0) ? 0.3f : 0.02f;
    float c[3] = {unif(&seed), unif(&seed), unif(&seed)};
    for (int k = 0; k < 3; ++k) {
      for (int a = 0; a < 3; ++a) hv[(size_t)a * V + 3 * t + k] = c[a] + (unif(&seed) - 0.5f) * big;
      ht[3 * t + k] = 3 * t + k;
    }
  }
  float *dv; uint32_t *dt, *cells, *objs, *ranges; void* ws;
  HIPCHK(hipMalloc((void**)&dv, sizeof(float) * 3 * V));
  HIPCHK(hipMalloc((void**)&dt, sizeof(uint32_t) * 3 * T));
  HIPCHK(hipMemcpy(dv, hv, sizeof(float) * 3 * V, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(dt, ht, sizeof(uint32_t) * 3 * T, hipMemcpyHostToDevice));
  const uint64_t R = (uint64_t)res[0] * res[1] * res[2];

  /* count first to size the outputs, as a caller without an estimate would */
  size_t wsz = grid_workspace_size(T, 0, res);
  HIPCHK(hipMalloc(&ws, wsz));
  uint64_t no = 0;
  CHECK(grid_count(dv, V, dt, T, lo, hi, res, ws, wsz, NULL, &no, NULL) == GRID_OK, "grid_count");
  HIPCHK(hipFree(ws));
  wsz = grid_workspace_size(T, no, res);
  HIPCHK(hipMalloc(&ws, wsz));
  HIPCHK(hipMalloc((void**)&cells, sizeof(uint32_t) * (no ? no : 1)));
  HIPCHK(hipMalloc((void**)&objs, sizeof(uint32_t) * (no ? no : 1)));
  HIPCHK(hipMalloc((void**)&ranges, sizeof(uint32_t) * 2 * R));
  grid_out out = {cells, objs, ranges, no, 0};
  int st = grid_build(dv, V, dt, T, lo, hi, res, ws, wsz, &out, NULL);
  CHECK(st == GRID_OK, grid_strerror(st));
  CHECK(out.npairs == no, "npairs");

  uint32_t* hc = (uint32_t*)malloc(sizeof(uint32_t) * no);
  uint32_t* ho = (uint32_t*)malloc(sizeof(uint32_t) * no);
  uint32_t* hr = (uint32_t*)malloc(sizeof(uint32_t) * 2 * R);
  HIPCHK(hipMemcpy(hc, cells, sizeof(uint32_t) * no, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(ho, objs, sizeof(uint32_t) * no, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(hr, ranges, sizeof(uint32_t) * 2 * R, hipMemcpyDeviceToHost));

  float inv[3];
  for (int a = 0; a < 3; ++a) inv[a] = (float)res[a] / (hi[a] - lo[a]);
  uint32_t* seen = (uint32_t*)calloc(T, sizeof(uint32_t));
  for (uint64_t i = 0; i < no; ++i) {
    if (i > 0) {
      CHECK(hc[i] >= hc[i - 1], "cells sorted");
      if (hc[i] == hc[i - 1]) CHECK(ho[i] > ho[i - 1], "objects ascend within a cell");
    }
    const uint32_t t = ho[i];
    CHECK(t < T, "object id in range");
    seen[t]++;
    const uint32_t c = hc[i];
    const uint32_t xyz[3] = {c % res[0], (c / res[0]) % res[1], c / (res[0] * res[1])};
    for (int a = 0; a < 3; ++a) {
      float mn = hv[(size_t)a * V + 3 * t], mx = mn;
      for (int k = 1; k < 3; ++k) {
        const float p = hv[(size_t)a * V + 3 * t + k];
        mn = fminf(mn, p);
        mx = fmaxf(mx, p);
      }
      CHECK(xyz[a] >= cell_of(mn, lo[a], inv[a], res[a]) && xyz[a] <= cell_of(mx, lo[a], inv[a], res[a]),
            "pair inside its triangle's cell box");
    }
  }
  uint64_t total = 0;
  for (uint32_t t = 0; t < T; ++t) {
    uint64_t m = 1;
    for (int a = 0; a < 3; ++a) {
      float mn = hv[(size_t)a * V + 3 * t], mx = mn;
      for (int k = 1; k < 3; ++k) {
        const float p = hv[(size_t)a * V + 3 * t + k];
        mn = fminf(mn, p);
        mx = fmaxf(mx, p);
      }
      m *= cell_of(mx, lo[a], inv[a], res[a]) - cell_of(mn, lo[a], inv[a], res[a]) + 1;
    }
    CHECK(seen[t] == m, "each triangle appears box-size times");
    total += m;
  }
  CHECK(total == no, "NO is the sum of the box sizes");
  CHECK(hr[0] == 0 && hr[2 * R - 1] == no, "ranges start at 0 and end at NO");
  for (uint64_t c = 0; c < R; ++c) {
    CHECK(hr[2 * c] <= hr[2 * c + 1], "begin <= end");
    if (c + 1 < R) CHECK(hr[2 * c + 1] == hr[2 * c + 2], "ranges tile");
    for (uint32_t i = hr[2 * c]; i < hr[2 * c + 1]; ++i) CHECK(hc[i] == c, "range holds its cell's pairs");
  }
  printf("ok %llu\n", (unsigned long long)no);
  hipFree(dv); hipFree(dt); hipFree(cells); hipFree(objs); hipFree(ranges); hipFree(ws);
  free(hv); free(ht); free(hc); free(ho); free(hr); free(seen);
  return 0;
}
