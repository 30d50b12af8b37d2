/* The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer: plain
 * builds and culled builds of seeded soups that include huge triangles,
 * vertices outside the bounds, NaN vertices, a bad vertex index and too small
 * a capacity, through the oracle's C entry points.  Checks what the grid
 * contract fixes (sorted cells, ascending objects within a cell, ranges tiling
 * [0, NO), kept pairs a subset of the box pairs) and exits 0 on success. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_build(const float* verts_soa, uint32_t nverts, const uint32_t* tris, uint32_t ntris, const float lo[3],
                 const float hi[3], const uint32_t res[3], uint32_t* cells, uint32_t* objs, uint32_t* ranges,
                 uint64_t cap_pairs, uint64_t* npairs);
int oracle_build_culled(const float* verts_soa, uint32_t nverts, const uint32_t* tris, uint32_t ntris,
                        const float lo[3], const float hi[3], const uint32_t res[3], uint32_t* cells, uint32_t* objs,
                        uint32_t* ranges, uint64_t cap_pairs, uint64_t* npairs, uint64_t* box_npairs);

#define CHECK(c, msg) do { if (!(c)) { fprintf(stderr, "FAIL: %s\n", msg); return 1; } } while (0)

static uint64_t s_state = 42;
static float unif(void) {
  s_state = s_state * 6364136223846793005ull + 1442695040888963407ull;
  return (float)((s_state >> 40) & 0xFFFFFF) / 16777216.0f;
}

static int check_grid(const uint32_t* cells, const uint32_t* objs, const uint32_t* ranges, uint64_t no,
                      uint64_t ncells) {
  for (uint64_t i = 1; i < no; ++i) {
    CHECK(cells[i - 1] <= cells[i], "cells sorted");
    CHECK(cells[i - 1] < cells[i] || objs[i - 1] < objs[i], "objects ascending within a cell");
  }
  CHECK(ranges[0] == 0 && ranges[2 * ncells - 1] == no, "ranges span [0, NO)");
  for (uint64_t c = 0; c < ncells; ++c) {
    CHECK(ranges[2 * c] <= ranges[2 * c + 1], "begin <= end");
    if (c + 1 < ncells) CHECK(ranges[2 * c + 1] == ranges[2 * c + 2], "ranges tile");
    for (uint32_t i = ranges[2 * c]; i < ranges[2 * c + 1]; ++i) CHECK(cells[i] == c, "range holds its cell");
  }
  return 0;
}

int main(void) {
  const uint32_t T = 3000, V = 3 * T;
  const uint32_t res[3] = {23, 17, 31};
  const float lo[3] = {0.f, 0.f, 0.f}, hi[3] = {1.f, 1.f, 1.f};
  const uint64_t ncells = (uint64_t)res[0] * res[1] * res[2];
  float* v = (float*)malloc(sizeof(float) * 3 * V);
  uint32_t* t = (uint32_t*)malloc(sizeof(uint32_t) * 3 * T);
  for (uint32_t i = 0; i < T; ++i) {
    const float spread = (i % 97 == 0) ? 0.6f : 0.03f;  /* a few huge triangles */
    float c[3] = {unif(), unif(), unif()};
    for (int j = 0; j < 3; ++j)
      for (int a = 0; a < 3; ++a) v[(size_t)a * V + 3 * i + j] = c[a] + (unif() - 0.5f) * spread;
    for (int j = 0; j < 3; ++j) t[3 * i + j] = 3 * i + j;
  }
  v[0] = -2.0f;                   /* outside the bounds */
  v[(size_t)1 * V + 7] = 3.5f;
  v[(size_t)2 * V + 11] = NAN;    /* NaN maps to cell 0 */
  uint64_t no = 0, box = 0;
  CHECK(oracle_build(v, V, t, T, lo, hi, res, NULL, NULL, NULL, 0, &no) == 0, "sizing probe");
  uint32_t* cells = (uint32_t*)malloc(sizeof(uint32_t) * no);
  uint32_t* objs = (uint32_t*)malloc(sizeof(uint32_t) * no);
  uint32_t* ranges = (uint32_t*)malloc(sizeof(uint32_t) * 2 * ncells);
  CHECK(oracle_build(v, V, t, T, lo, hi, res, cells, objs, ranges, no - 1, &no) == -4, "capacity error");
  CHECK(oracle_build(v, V, t, T, lo, hi, res, cells, objs, ranges, no, &no) == 0, "plain build");
  if (check_grid(cells, objs, ranges, no, ncells)) return 1;
  uint64_t kept = 0;
  CHECK(oracle_build_culled(v, V, t, T, lo, hi, res, NULL, NULL, NULL, 0, &kept, &box) == 0, "culled probe");
  CHECK(box == no && kept <= no && kept >= T, "kept pairs within the box pairs, one per triangle at least");
  CHECK(oracle_build_culled(v, V, t, T, lo, hi, res, cells, objs, ranges, kept, &kept, &box) == 0, "culled build");
  if (check_grid(cells, objs, ranges, kept, ncells)) return 1;
  t[5] = V;                       /* a bad vertex index */
  CHECK(oracle_build(v, V, t, T, lo, hi, res, NULL, NULL, NULL, 0, &no) == -5, "bad index");
  CHECK(oracle_build(v, V, t, 0, lo, hi, res, cells, objs, ranges, 0, &no) == 0 && no == 0, "empty scene");
  free(v); free(t); free(cells); free(objs); free(ranges);
  printf("ok %llu %llu\n", (unsigned long long)box, (unsigned long long)kept);
  return 0;
}
