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

// Linear cell id, x varying fastest (the order GlobalCoords enumerates a box).
inline uint32_t linear_id(const uint32_t g[3], const uint32_t res[3]) { return g[0] + res[0] * (g[1] + res[1] * g[2]); }

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
      cells[i] = linear_id(g, res);
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

// ---------------------------------------------------------------------------
// Removal of false intersections (the fix the Test Results section suggests for
// scenes of long thin diagonal triangles such as Hairball, and the Conclusions
// list as future work): a pair <t, c> from t's cell box is kept only when the
// triangle touches the cell.  Readings (the paper gives no test):
//  * the test runs in grid coordinates: each vertex coordinate is the FP32
//    value the cell map floors, u = (p - lo) * inv, so cell (x, y, z) is the
//    closed unit box [x, x+1] x [y, y+1] x [z, z+1];
//  * a separating-axis test over the triangle's normal and the nine cross
//    products of its edges with the grid axes (the three face axes are
//    implied by the cell box), every operation one FP32 operation in the
//    order written here, with the cell widened by kOverlapMargin on every
//    side so rounding can keep a false pair but never drop a true one;
//  * a triangle keeps its whole box when a vertex lies outside [0, res] on
//    some axis (or is NaN), and when its box holds at most two cells (it then
//    touches every one of them).
// ---------------------------------------------------------------------------

namespace {

constexpr float kOverlapMargin = 1.0f / 64.0f;  // cells

inline float dot3(const float a[3], const float b[3]) {
  float s = a[0] * b[0];
  s = s + a[1] * b[1];
  s = s + a[2] * b[2];
  return s;
}

// True when axis a separates the triangle (grid coordinates u[j][axis]) from
// the widened cell whose lower corner is b.
bool axis_separates(const float a[3], const float u[3][3], const float b[3]) {
  const float p0 = dot3(a, u[0]), p1 = dot3(a, u[1]), p2 = dot3(a, u[2]);
  const float tmin = std::fmin(std::fmin(p0, p1), p2);
  const float tmax = std::fmax(std::fmax(p0, p1), p2);
  float lo_off = std::fmin(a[0], 0.0f) + std::fmin(a[1], 0.0f);
  lo_off = lo_off + std::fmin(a[2], 0.0f);
  float hi_off = std::fmax(a[0], 0.0f) + std::fmax(a[1], 0.0f);
  hi_off = hi_off + std::fmax(a[2], 0.0f);
  float l1 = std::fabs(a[0]) + std::fabs(a[1]);
  l1 = l1 + std::fabs(a[2]);
  const float mg = kOverlapMargin * l1;
  // the cell projects onto [c + lo_off, c + hi_off] (widened by mg)
  const float c = dot3(a, b);
  const float above = (tmax + mg) - lo_off;
  const float below = (tmin - mg) - hi_off;
  return c > above || c < below;
}

// True when the triangle with grid coordinates u touches the widened cell b.
bool triangle_touches_cell(const float u[3][3], const float b[3]) {
  float e[3][3];
  for (int i = 0; i < 3; ++i)
    for (int a = 0; a < 3; ++a) e[i][a] = u[(i + 1) % 3][a] - u[i][a];
  const float n[3] = {e[0][1] * e[1][2] - e[0][2] * e[1][1], e[0][2] * e[1][0] - e[0][0] * e[1][2],
                      e[0][0] * e[1][1] - e[0][1] * e[1][0]};
  if (axis_separates(n, u, b)) return false;
  for (int i = 0; i < 3; ++i) {
    const float ax[3] = {0.0f, e[i][2], -e[i][1]};   // e x (1, 0, 0)
    const float ay[3] = {-e[i][2], 0.0f, e[i][0]};   // e x (0, 1, 0)
    const float az[3] = {e[i][1], -e[i][0], 0.0f};   // e x (0, 0, 1)
    if (axis_separates(ax, u, b) || axis_separates(ay, u, b) || axis_separates(az, u, b)) return false;
  }
  return true;
}

}  // namespace

extern "C" {

// Grid coordinates of triangle t's vertices (u[j][axis]); returns 1 when the
// overlap test applies to t (every coordinate finite and inside [0, res]).
int oracle_grid_coords(const float* verts_soa, uint32_t nverts, const uint32_t* tri, const float lo[3],
                       const float inv[3], const uint32_t res[3], float u[3][3]) {
  int inside = 1;
  for (int j = 0; j < 3; ++j)
    for (int a = 0; a < 3; ++a) {
      const float p = verts_soa[static_cast<size_t>(a) * nverts + tri[j]];
      const float sft = p - lo[a];
      u[j][a] = sft * inv[a];
      if (!(u[j][a] >= 0.0f && u[j][a] <= static_cast<float>(res[a]))) inside = 0;
    }
  return inside;
}

// 1 when the triangle with grid coordinates u (float [3][3]) touches cell (x, y, z).
int oracle_touches(const float* u, uint32_t x, uint32_t y, uint32_t z) {
  float uu[3][3];
  for (int j = 0; j < 3; ++j)
    for (int a = 0; a < 3; ++a) uu[j][a] = u[3 * j + a];
  const float b[3] = {static_cast<float>(x), static_cast<float>(y), static_cast<float>(z)};
  return triangle_touches_cell(uu, b) ? 1 : 0;
}

// The object-order pair lists with false intersections removed: the pairs of
// oracle_make_pairs, in the same order, less those whose triangle misses the
// cell.  cells/objs hold at least NO (box) entries; returns the kept count and
// writes each triangle's kept count to kept (if not null).
uint64_t oracle_make_pairs_culled(const float* verts_soa, uint32_t nverts, const uint32_t* tris, uint32_t ntris,
                                  const float lo[3], const float hi[3], const uint32_t res[3],
                                  const uint32_t* box_lo, const uint32_t* box_m, const uint32_t* count,
                                  uint32_t* cells, uint32_t* objs, uint32_t* kept) {
  float inv[3];
  oracle_inv_cell(lo, hi, res, inv);
  uint64_t i = 0;
  for (uint32_t t = 0; t < ntris; ++t) {
    float u[3][3];
    const int inside = oracle_grid_coords(verts_soa, nverts, tris + 3 * static_cast<size_t>(t), lo, inv, res, u);
    const bool test = inside && count[t] > 2;
    uint32_t k = 0;
    for (uint32_t rid = 0; rid < count[t]; ++rid) {
      uint32_t g[3];
      oracle_global_coords(box_lo + 3 * static_cast<size_t>(t), box_m + 3 * static_cast<size_t>(t), rid, g);
      if (test) {
        const float b[3] = {static_cast<float>(g[0]), static_cast<float>(g[1]), static_cast<float>(g[2])};
        if (!triangle_touches_cell(u, b)) continue;
      }
      cells[i] = linear_id(g, res);
      objs[i] = t;
      ++i;
      ++k;
    }
    if (kept) kept[t] = k;
  }
  return i;
}

// Whole build with false intersections removed: as oracle_build, over the
// kept pairs.  *npairs = the kept count; with ranges == nullptr only the
// count is reported.  *box_npairs (if not null) = the box pair count.
int oracle_build_culled(const float* verts_soa, uint32_t nverts, const uint32_t* tris, uint32_t ntris,
                        const float lo[3], const float hi[3], const uint32_t res[3], uint32_t* cells, uint32_t* objs,
                        uint32_t* ranges, uint64_t cap_pairs, uint64_t* npairs, uint64_t* box_npairs) {
  std::vector<uint32_t> box_lo(3 * static_cast<size_t>(ntris)), box_m(3 * static_cast<size_t>(ntris)), count(ntris);
  int st = oracle_count_cells(verts_soa, nverts, tris, ntris, lo, hi, res, box_lo.data(), box_m.data(), count.data());
  if (st != kOk) return st;
  std::vector<uint64_t> start(ntris);
  const uint64_t nbox = oracle_exclusive_sum(count.data(), ntris, start.data());
  if (box_npairs) *box_npairs = nbox;
  if (nbox > 0xFFFFFFFFull) return kOverflow;
  std::vector<uint32_t> c(nbox), o(nbox);
  const uint64_t no = oracle_make_pairs_culled(verts_soa, nverts, tris, ntris, lo, hi, res, box_lo.data(),
                                               box_m.data(), count.data(), c.data(), o.data(), nullptr);
  *npairs = no;
  if (ranges == nullptr) return kOk;
  if (no > cap_pairs) return kCapacity;
  std::copy(c.begin(), c.begin() + no, cells);
  std::copy(o.begin(), o.begin() + no, objs);
  oracle_sort_pairs(no, cells, objs);
  uint64_t ncells = static_cast<uint64_t>(res[0]) * res[1] * res[2];
  oracle_ranges(no, cells, ncells, ranges);
  return kOk;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Ray casting, the use the grid is built for (Introduction; Related Work: the
// grid answers ray and spatial queries): the closest triangle a ray hits,
// here by brute force over every triangle, which is the plain definition the
// grid traversal must reproduce.  Readings (the paper gives no query):
//  * a ray is o + t d for t in [t0, t1], where [t0, t1] clips [0, tmax] to
//    the grid box [lo, hi] by the slab test (per axis with d != 0:
//    t = (lo - o) / d and (hi - o) / d; an axis with d = 0 and o outside
//    [lo, hi] leaves no interval); only hits inside the box count, the part
//    of space the grid covers;
//  * the hit test is Moller and Trumbore's, every operation one FP32 operation
//    in the order written (no contraction, IEEE division); a triangle whose
//    plane the ray meets at a grazing angle (det^2 < 1e-8 |e1|^2 |e2|^2 |d|^2,
//    an angle below about 1e-4 rad) or that is degenerate is missed; edges
//    and vertices count as hits;
//  * the result is the smallest hit t and, among triangles hit at exactly that
//    t, the smallest id; no hit gives t = +inf and id 0xFFFFFFFF.
// ---------------------------------------------------------------------------

namespace {

constexpr float kGrazing = 1e-8f;

inline void cross3(const float a[3], const float b[3], float r[3]) {
  r[0] = a[1] * b[2] - a[2] * b[1];
  r[1] = a[2] * b[0] - a[0] * b[2];
  r[2] = a[0] * b[1] - a[1] * b[0];
}

// The hit parameter of ray (o, d) with triangle (v0, v1, v2), or +inf.
float ray_triangle(const float o[3], const float d[3], const float v0[3], const float v1[3], const float v2[3]) {
  float e1[3], e2[3], s[3], p[3], q[3];
  for (int a = 0; a < 3; ++a) {
    e1[a] = v1[a] - v0[a];
    e2[a] = v2[a] - v0[a];
    s[a] = o[a] - v0[a];
  }
  cross3(d, e2, p);
  float det = dot3(e1, p);
  const float lim = ((dot3(e1, e1) * dot3(e2, e2)) * dot3(d, d)) * kGrazing;
  if (!(det * det >= lim) || det == 0.0f) return INFINITY;
  float u = dot3(s, p);
  cross3(s, e1, q);
  float v = dot3(d, q);
  float tn = dot3(e2, q);
  if (det < 0.0f) {
    det = -det;
    u = -u;
    v = -v;
    tn = -tn;
  }
  if (!(u >= 0.0f && v >= 0.0f && u + v <= det)) return INFINITY;
  return tn / det;
}

// [t0, t1]: [0, tmax] clipped to the box; false when empty.
bool clip_to_box(const float o[3], const float d[3], const float lo[3], const float hi[3], float tmax, float* t0,
                 float* t1) {
  float a0 = 0.0f, a1 = tmax;
  for (int a = 0; a < 3; ++a) {
    if (d[a] != 0.0f) {
      const float ta = (lo[a] - o[a]) / d[a];
      const float tb = (hi[a] - o[a]) / d[a];
      a0 = std::fmax(a0, std::fmin(ta, tb));
      a1 = std::fmin(a1, std::fmax(ta, tb));
    } else if (!(o[a] >= lo[a] && o[a] <= hi[a])) {
      return false;
    }
  }
  *t0 = a0;
  *t1 = a1;
  return a0 <= a1;
}

}  // namespace

extern "C" {

// Closest hits of nrays rays (rays: FP32 [6][nrays], origin x, y, z then
// direction x, y, z) with the triangles, within the grid box and tmax.
void oracle_raycast(const float* verts_soa, uint32_t nverts, const uint32_t* tris, uint32_t ntris, const float lo[3],
                    const float hi[3], const float* rays, uint32_t nrays, float tmax, float* hit_t, uint32_t* hit_obj) {
  for (uint32_t r = 0; r < nrays; ++r) {
    float o[3], d[3];
    for (int a = 0; a < 3; ++a) {
      o[a] = rays[static_cast<size_t>(a) * nrays + r];
      d[a] = rays[static_cast<size_t>(3 + a) * nrays + r];
    }
    float best = INFINITY, t0 = 0.0f, t1 = 0.0f;
    uint32_t id = 0xFFFFFFFFu;
    if (clip_to_box(o, d, lo, hi, tmax, &t0, &t1)) {
      for (uint32_t t = 0; t < ntris; ++t) {
        float v[3][3];
        for (int j = 0; j < 3; ++j)
          for (int a = 0; a < 3; ++a) v[j][a] = verts_soa[static_cast<size_t>(a) * nverts + tris[3 * static_cast<size_t>(t) + j]];
        const float th = ray_triangle(o, d, v[0], v[1], v[2]);
        if (th >= t0 && th <= t1 && th < best) {
          best = th;
          id = t;
        }
      }
    }
    hit_t[r] = best;
    hit_obj[r] = id;
  }
}

}  // extern "C"
