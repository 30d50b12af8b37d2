// Serial CPU oracle for the parallel uniform-grid construction
// (Costa, Pereira, Jorge, "Building An Efficient Grid On GPU", Algorithm 1).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or load
// this file: only the test suite, the smoke check and the CPU-baseline leg of
// the benchmark use it.  It shares no code, header or table with the GPU
// library; it is written from the paper's definitions, one obvious loop per
// step, with no blocking, fusion or reordering.
//
// Readings of points the paper leaves open (they are the project's contract):
//  * world -> cell map: floor((p - lo) * inv) in FP32 with no contraction,
//    clamped to [0, res-1] on both sides, inv = (float)res / (hi - lo) computed
//    once in FP32; a point on a cell face belongs to the upper cell, NaN maps
//    to cell 0 and +-inf to the boundary cells;
//  * a triangle's box per axis is [cell(min p), cell(max p)], with min/max the
//    IEEE minNum/maxNum of its three vertices (NaN coordinates are ignored
//    unless all three are NaN);
//  * cell id = x + rx * (y + ry * z), matching the order of GlobalCoords;
//  * the sort is stable, so each cell lists its objects in ascending id order;
//  * G follows its definition as the exclusive sum of per-cell counts, so an
//    empty cell gets the empty range [G[c], G[c]) and the ranges tile [0, NO).
//
// Build: g++ -O2 -ffp-contract=off -fno-fast-math -fPIC -shared oracle.cpp
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>

namespace {

constexpr int kOk = 0;
constexpr int kInval = -1;
constexpr int kOverflow = -3;
constexpr int kCapacity = -4;
constexpr int kBadIndex = -5;

// One axis of the world -> cell map (reading above).  Every operation is a
// single IEEE FP32 operation; this file is compiled with -ffp-contract=off.
inline uint32_t cell_coord(float p, float lo, float inv, uint32_t res) {
  float s = p - lo;
  float u = s * inv;
  float f = std::floor(u);
  f = std::fmax(f, 0.0f);
  f = std::fmin(f, static_cast<float>(res - 1));
  return static_cast<uint32_t>(f);
}

bool valid_grid(const float lo[3], const float hi[3], const uint32_t res[3]) {
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(lo[a]) || !std::isfinite(hi[a]) || !(lo[a] < hi[a])) return false;
    if (res[a] < 1 || res[a] > 1024) return false;
  }
  return true;
}

}  // namespace

extern "C" {

// The per-axis cell scale, inv[a] = (float)res[a] / (hi[a] - lo[a]) in FP32.
void oracle_inv_cell(const float lo[3], const float hi[3], const uint32_t res[3], float inv[3]) {
  for (int a = 0; a < 3; ++a) {
    float ext = hi[a] - lo[a];
    inv[a] = static_cast<float>(res[a]) / ext;
  }
}

// CountCells (Algorithm 1, first step; Section 3 text): for each triangle the
// inclusive cell box [box_lo, box_lo + m - 1] its bounding box overlaps, and
// V[t] = mx * my * mz cells.  box_lo and m are [T][3].
int oracle_count_cells(const float* verts_soa, uint32_t nverts, const uint32_t* tris, uint32_t ntris,
                       const float lo[3], const float hi[3], const uint32_t res[3],
                       uint32_t* box_lo, uint32_t* box_m, uint32_t* count) {
  if (!valid_grid(lo, hi, res)) return kInval;
  float inv[3];
  oracle_inv_cell(lo, hi, res, inv);
  for (uint32_t t = 0; t < ntris; ++t) {
    const uint32_t* tri = tris + 3 * static_cast<size_t>(t);
    if (tri[0] >= nverts || tri[1] >= nverts || tri[2] >= nverts) return kBadIndex;
  }
  for (uint32_t t = 0; t < ntris; ++t) {
    const uint32_t* tri = tris + 3 * static_cast<size_t>(t);
    uint64_t c = 1;
    for (int a = 0; a < 3; ++a) {
      const float* axis = verts_soa + static_cast<size_t>(a) * nverts;
      float p0 = axis[tri[0]], p1 = axis[tri[1]], p2 = axis[tri[2]];
      float pmin = std::fmin(std::fmin(p0, p1), p2);
      float pmax = std::fmax(std::fmax(p0, p1), p2);
      uint32_t cl = cell_coord(pmin, lo[a], inv[a], res[a]);
      uint32_t ch = cell_coord(pmax, lo[a], inv[a], res[a]);
      box_lo[3 * static_cast<size_t>(t) + a] = cl;
      box_m[3 * static_cast<size_t>(t) + a] = ch - cl + 1;
      c *= ch - cl + 1;
    }
    count[t] = static_cast<uint32_t>(c);
  }
  return kOk;
}

// ExclusiveSum(V) (Algorithm 1, second step): start[t] = sum of V[s] for s < t;
// returns NO, the number of <obj, cell> pairs.
uint64_t oracle_exclusive_sum(const uint32_t* count, uint32_t n, uint64_t* start) {
  uint64_t acc = 0;
  for (uint32_t i = 0; i < n; ++i) {
    start[i] = acc;
    acc += count[i];
  }
  return acc;
}

// GlobalCoords (Section 3): relative cell offset rid inside a box of extent m
// -> the box's global cell coordinates, x varying fastest.
void oracle_global_coords(const uint32_t box_lo[3], const uint32_t m[3], uint32_t rid, uint32_t out[3]) {
  uint32_t z = rid / (m[0] * m[1]);
  uint32_t y = (rid - z * m[0] * m[1]) / m[0];
  uint32_t x = rid - m[0] * (y + m[1] * z);
  out[0] = box_lo[0] + x;
  out[1] = box_lo[1] + y;
  out[2] = box_lo[2] + z;
}

// Object-order pair lists (Algorithm 1, MakeObjectIds through MakeCellIds):
// for each object t in input order and each relative offset rid of its box,
// O = t and C = the linear id of GlobalCoords(box, rid).
void oracle_make_pairs(uint32_t ntris, const uint32_t* box_lo, const uint32_t* box_m,
                       const uint32_t* count, const uint32_t res[3], uint32_t* cells, uint32_t* objs) {
  size_t i = 0;
  for (uint32_t t = 0; t < ntris; ++t) {
    for (uint32_t rid = 0; rid < count[t]; ++rid) {
      uint32_t g[3];
      oracle_global_coords(box_lo + 3 * static_cast<size_t>(t), box_m + 3 * static_cast<size_t>(t), rid, g);
      cells[i] = g[0] + res[0] * (g[1] + res[1] * g[2]);
      objs[i] = t;
      ++i;
    }
  }
}

// RadixSort(C, O) (Algorithm 1): a stable sort of the pairs by cell id.  Any
// stable sort gives the same unique result; std::stable_sort is the textbook one.
void oracle_sort_pairs(uint64_t npairs, uint32_t* cells, uint32_t* objs) {
  std::vector<uint64_t> idx(npairs);
  std::iota(idx.begin(), idx.end(), uint64_t{0});
  std::stable_sort(idx.begin(), idx.end(), [&](uint64_t a, uint64_t b) { return cells[a] < cells[b]; });
  std::vector<uint32_t> c2(npairs), o2(npairs);
  for (uint64_t i = 0; i < npairs; ++i) {
    c2[i] = cells[idx[i]];
    o2[i] = objs[idx[i]];
  }
  std::copy(c2.begin(), c2.end(), cells);
  std::copy(o2.begin(), o2.end(), objs);
}

// RunLengthEncode + NonEmptyCells + ExclusiveSum(G) (Algorithm 1, last
// steps): G[c] = number of pairs with cell < c.  Written out as the per-cell
// [begin, end) table: ranges[2c] = G[c], ranges[2c+1] = G[c] + count of c.
void oracle_ranges(uint64_t npairs, const uint32_t* sorted_cells, uint64_t ncells, uint32_t* ranges) {
  std::vector<uint64_t> per_cell(ncells, 0);
  for (uint64_t i = 0; i < npairs; ++i) per_cell[sorted_cells[i]] += 1;
  uint64_t acc = 0;
  for (uint64_t c = 0; c < ncells; ++c) {
    ranges[2 * c] = static_cast<uint32_t>(acc);
    acc += per_cell[c];
    ranges[2 * c + 1] = static_cast<uint32_t>(acc);
  }
}

// Whole build: BuildParallelGrid(M, boxes) -> (G, O), plus the sorted C.
// cells/objs hold cap_pairs entries and ranges 2 * ncells; when NO exceeds
// cap_pairs only *npairs is written and -4 (capacity) is returned.  With
// ranges == nullptr the call only reports *npairs (a sizing probe).
int oracle_build(const float* verts_soa, uint32_t nverts, const uint32_t* tris, uint32_t ntris,
                 const float lo[3], const float hi[3], const uint32_t res[3],
                 uint32_t* cells, uint32_t* objs, uint32_t* ranges, uint64_t cap_pairs, uint64_t* npairs) {
  std::vector<uint32_t> box_lo(3 * static_cast<size_t>(ntris)), box_m(3 * static_cast<size_t>(ntris)), count(ntris);
  int st = oracle_count_cells(verts_soa, nverts, tris, ntris, lo, hi, res, box_lo.data(), box_m.data(), count.data());
  if (st != kOk) return st;
  std::vector<uint64_t> start(ntris);
  uint64_t no = oracle_exclusive_sum(count.data(), ntris, start.data());
  *npairs = no;
  if (no > 0xFFFFFFFFull) return kOverflow;
  if (ranges == nullptr) return kOk;
  if (no > cap_pairs) return kCapacity;
  oracle_make_pairs(ntris, box_lo.data(), box_m.data(), count.data(), res, cells, objs);
  oracle_sort_pairs(no, cells, objs);
  uint64_t ncells = static_cast<uint64_t>(res[0]) * res[1] * res[2];
  oracle_ranges(no, cells, ncells, ranges);
  return kOk;
}

}  // extern "C"
