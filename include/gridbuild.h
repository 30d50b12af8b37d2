/*
 * gridbuild.h - C ABI of the MI355X (gfx950) parallel uniform-grid builder.
 *
 * The library implements BuildParallelGrid (Algorithm 1 of Costa, Pereira and
 * Jorge, "Building An Efficient Grid On GPU"): for every triangle it counts the
 * grid cells its bounding box overlaps (CountCells), turns the counts into
 * one work item per <object, cell> pair with an exclusive scan (ExclusiveSum,
 * MakeObjectIds, InclusiveSum, SegmentedExclusiveSum), maps each item to its
 * global cell (GlobalCoords, MakeCellIds), sorts the pairs by cell with an LSD
 * radix sort (RadixSort) and extracts each cell's slice of the sorted list
 * (RunLengthEncode, NonEmptyCells, ExclusiveSum over the grid).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Device pointers point to memory the caller owns (e.g. PyTorch tensors);
 *    the library never allocates or frees device memory.  Host pointers are
 *    marked "host".  Scratch memory is passed in as a workspace (ws, ws_bytes)
 *    whose required size the *_workspace_size functions report.
 *  - stream is a hipStream_t (NULL = the default stream).  All device work is
 *    ordered on it.  Entry points that must read a result back (the pair count)
 *    synchronize that stream once and say so.  Their readback lands in one small
 *    pinned host block per calling host thread, allocated on that thread's first
 *    such call and kept until the process ends (grid_build_static excepted: it
 *    reads back through pageable memory and allocates nothing).
 *  - Inputs: verts_soa is FP32 [3][nverts] (all x, then all y, then all z);
 *    tris is uint32 [ntris][3] vertex indices.  lo, hi (host, 3 floats) are the
 *    grid bounds and res (host, 3 uint32) the cells per axis.
 *  - Grid contract (the paper leaves these open; this is the library's reading):
 *      inv[a]  = (float)res[a] / (hi[a] - lo[a])      FP32, on the host
 *      cell(p) = min(max(floor((p - lo) * inv), 0), res - 1)   FP32, no FMA
 *      a triangle's box on axis a = [cell(min p), cell(max p)]  (IEEE minNum/
 *      maxNum over its three vertices), cell id = x + rx * (y + ry * z).
 *    Points outside the bounds are clamped onto the boundary cells; NaN maps to
 *    cell 0.  Every triangle therefore covers at least one cell.
 *  - Outputs (grid_out): cells[i], objs[i] for i < npairs are the pairs sorted
 *    by cell and, within a cell, by ascending object id (a stable sort of the
 *    object-order list; the result is unique).  ranges is uint32 [2 * R]
 *    (R = rx * ry * rz) with ranges[2c] = number of pairs whose cell is < c and
 *    ranges[2c + 1] = number whose cell is <= c, so cell c owns
 *    objs[ranges[2c] .. ranges[2c + 1]) and an empty cell has an empty range.
 *    This is the paper's compact grid G (the begin column) plus each end.
 *  - Return value: GRID_OK or a negative grid_status.  On error the outputs'
 *    contents are unspecified, except that GRID_E_CAPACITY still reports the
 *    required pair count.  No exception or abort crosses the ABI.
 *  - Limits: 1 <= res[a] <= 1024; NO (the pair count) <= 2^32 - 1; ntris < 2^31.
 *  - Thread safety: calls on different workspaces may run concurrently;
 *    calls sharing one workspace must be ordered (same stream or synchronized).
 */
#ifndef GRIDBUILD_H
#define GRIDBUILD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum grid_status {
  GRID_OK = 0,
  GRID_E_INVAL = -1,     /* null pointer, res outside [1, 1024], !(lo < hi), non-finite bounds */
  GRID_E_NOMEM = -2,     /* workspace smaller than the size the library asked for */
  GRID_E_OVERFLOW = -3,  /* NO > 2^32 - 1 */
  GRID_E_CAPACITY = -4,  /* NO > cap_pairs; npairs holds the required count */
  GRID_E_BADINDEX = -5,  /* a triangle references a vertex index >= nverts */
  GRID_E_HIP = -6,       /* a HIP runtime call failed */
  GRID_E_INTERNAL = -7   /* an internal consistency check on the device failed; outputs are invalid */
} grid_status;

/* Output of one grid.  cells/objs/ranges are device pointers owned by the caller. */
typedef struct grid_out {
  uint32_t *cells;     /* [cap_pairs] sorted cell ids                          */
  uint32_t *objs;      /* [cap_pairs] object ids, ascending within each cell    */
  uint32_t *ranges;    /* [2 * R] (begin, end) per cell, x-fastest cell order   */
  uint64_t cap_pairs;  /* in: capacity of cells/objs, in pairs                  */
  uint64_t npairs;     /* out: NO, the number of <obj, cell> pairs              */
} grid_out;

/* One grid of a batch: the same arguments as grid_build, plus its outputs. */
typedef struct grid_desc {
  const float *verts_soa;  /* device, FP32 [3][nverts] */
  const uint32_t *tris;    /* device, uint32 [ntris][3] */
  uint32_t nverts;
  uint32_t ntris;
  float lo[3];
  float hi[3];
  uint32_t res[3];
  grid_out out;
} grid_desc;

/* Human-readable name of a status code (static storage). */
const char *grid_strerror(int status);

/* Bytes of workspace grid_count / grid_build / grid_expand need for a grid of
 * ntris triangles, at most cap_pairs pairs and res cells (host array). */
size_t grid_workspace_size(uint32_t ntris, uint64_t cap_pairs, const uint32_t res[3]);

/* CountCells + ExclusiveSum (Algorithm 1, first two steps; Section 3 text).
 * Writes *npairs (host) = NO.  If start_out (device, uint32 [ntris]) is not
 * NULL it receives each triangle's exclusive pair offset, so its cell count is
 * start[t+1] - start[t] (NO - start[T-1] for the last).  Synchronizes stream. */
int grid_count(const float *verts_soa, uint32_t nverts, const uint32_t *tris, uint32_t ntris,
               const float lo[3], const float hi[3], const uint32_t res[3],
               void *ws, size_t ws_bytes, uint32_t *start_out, uint64_t *npairs, void *stream);

/* The whole build, BuildParallelGrid(M, boxes) -> (G, O) (Algorithm 1), into
 * out (cells, objs: cap_pairs entries; ranges: 2 * R entries).  Every kernel
 * after the count reads NO from device memory and stops before writing if it
 * exceeds cap_pairs, so the whole sequence is launched at once and stream is
 * synchronized once, at the end, to read NO back into out->npairs (also on
 * GRID_E_CAPACITY, which leaves the outputs untouched). */
int grid_build(const float *verts_soa, uint32_t nverts, const uint32_t *tris, uint32_t ntris,
               const float lo[3], const float hi[3], const uint32_t res[3],
               void *ws, size_t ws_bytes, grid_out *out, void *stream);

/* The whole build with false intersections removed (the fix the Test Results
 * section proposes for long thin diagonal triangles, Hairball, and the
 * Conclusions list as future work): a pair <t, c> of triangle t's cell box is
 * kept only when t touches cell c.  The test is a separating-axis test in grid
 * coordinates u = (p - lo) * inv, where cell (x, y, z) is the unit box
 * [x, x+1] x [y, y+1] x [z, z+1]; its axes are the triangle's normal and the
 * nine cross products of its edges with the grid axes, each bound computed in
 * a fixed order of FP32 operations, and each cell is widened by 1/64 of a cell
 * on every side, so rounding may keep a pair the exact test would drop but
 * never drops one it would keep.  A triangle keeps its whole box when some
 * vertex coordinate lies outside [0, res] (or is NaN), or when its box holds
 * at most two cells.  The kept pairs are sorted and ranged as in grid_build.
 * box_cap bounds the box pair count (grid_count's NO): ws must hold
 * grid_workspace_size_culled(ntris, box_cap, res) bytes (the plain build's
 * workspace plus 176 bytes per triangle, where each triangle's axes and
 * bounds are computed once for all its pairs), and out->cap_pairs may be
 * smaller than box_cap (fewer pairs are kept).  *box_npairs (host) receives
 * the box pair count and out->npairs the kept count.  GRID_E_CAPACITY when
 * the box pairs exceed box_cap (out->npairs = 0) or the kept pairs exceed
 * out->cap_pairs (out->npairs = the kept count).  Synchronizes stream once. */
size_t grid_workspace_size_culled(uint32_t ntris, uint64_t box_cap, const uint32_t res[3]);
int grid_build_culled(const float *verts_soa, uint32_t nverts, const uint32_t *tris, uint32_t ntris,
                      const float lo[3], const float hi[3], const uint32_t res[3],
                      void *ws, size_t ws_bytes, uint64_t box_cap, grid_out *out, uint64_t *box_npairs,
                      void *stream);

/* Object-order pair lists (Algorithm 1, MakeObjectIds through MakeCellIds;
 * Section 3 and GlobalCoords): cells[i], objs[i] for i < NO in object order,
 * each object's cells in GlobalCoords order (x fastest).  Device outputs of
 * cap_pairs entries; *npairs (host) = NO.  Synchronizes stream. */
int grid_expand(const float *verts_soa, uint32_t nverts, const uint32_t *tris, uint32_t ntris,
                const float lo[3], const float hi[3], const uint32_t res[3],
                void *ws, size_t ws_bytes, uint32_t *cells, uint32_t *objs, uint64_t cap_pairs,
                uint64_t *npairs, void *stream);

/* Batched builds: ngrids independent grids (host array of descriptors) built
 * in one fixed sequence of launches.  Every grid's outputs are identical to
 * what grid_build returns for it alone: object ids local to the grid, ranges
 * relative to the grid's own pair list.  Internally the cells of all grids are
 * numbered in one space (each grid's cells follow the previous grid's) and the
 * pairs are sorted on that 32-bit number over only the bits in use, so one
 * launch sequence holds at most 2^32 cells in total; grid_count_batched and
 * grid_build_batched split larger batches into runs that fit. */
/* Workspace for the batch as described (out.cap_pairs as set; output pointers
 * may still be NULL when only counting).  0 if a descriptor is invalid. */
size_t grid_workspace_size_batched(const grid_desc *grids, uint32_t ngrids);

/* Per-grid NO into grids[g].out.npairs (host).  Synchronizes stream. */
int grid_count_batched(grid_desc *grids, uint32_t ngrids, void *ws, size_t ws_bytes, void *stream);

/* Build all grids; writes grids[g].out.npairs.  If any grid's NO exceeds its
 * cap_pairs the call returns GRID_E_CAPACITY after the count (every npairs is
 * then set) and builds nothing.  Synchronizes stream once, after the count. */
int grid_build_batched(grid_desc *grids, uint32_t ngrids, void *ws, size_t ws_bytes, void *stream);

/* Batched build with no host synchronisation, for overlapping batches on
 * several streams (serving) and for stream capture.  Every grid's
 * out.cap_pairs must already hold at least its NO (from grid_count_batched);
 * the batch's cells must total at most 2^32 (GRID_E_INVAL otherwise: split
 * the batch).  host_staging is caller-owned pinned host memory of at least
 * grid_batch_staging_size(ngrids) bytes, which must stay untouched until the
 * stream has passed this call.  Errors found on the device (a bad vertex
 * index, a count above capacity, NO above 2^32 - 1) stop every later kernel
 * before it writes; grid_workspace_status reports them.  out.npairs is not
 * written (the counts are the caller's capacities). */
size_t grid_batch_staging_size(uint32_t ngrids);
int grid_build_batched_async(const grid_desc *grids, uint32_t ngrids, void *ws, size_t ws_bytes,
                             void *host_staging, size_t staging_bytes, void *stream);

/* Status of the last build launched on a workspace (the device-side flags of
 * grid_build_batched_async) and, if npairs_total (host) is not NULL, its total
 * pair count.  Synchronizes stream. */
int grid_workspace_status(const void *ws, uint64_t *npairs_total, void *stream);

/* A batched build split in two halves around its count, so that a server can
 * size the outputs from the exact NO (Algorithm 1: CountCells and
 * ExclusiveSum give NO before any pair exists) without counting twice and
 * without a host wait inside either call.
 *
 * grid_count_batched_async enqueues the count of the batch into ws: its
 * triangle starts, cell boxes, tile owners and per-grid pair runs stay there
 * for the second half.  Output pointers are not read.  The workspace layout
 * holds as many pairs as ws_bytes allows; *pair_cap (host, if not NULL)
 * receives that number at once.  When the stream has passed the call,
 * counts_host[g] (host memory of ngrids + 1 words, pinned for the copy to stay
 * asynchronous) holds grid g's NO and counts_host[ngrids] a status word:
 * bit 0 a bad vertex index, bit 1 an internal check failed, bit 2 the pairs
 * exceed *pair_cap, bit 3 they exceed 2^32 - 1.  A nonzero status means the
 * batch cannot be resumed (a resumed build would write nothing).
 * host_staging: caller-owned pinned memory of at least
 * 2 * grid_batch_staging_size(ngrids) bytes; its first half keeps the counted
 * table until the second half has been enqueued.
 *
 * grid_build_batched_counted enqueues the rest of that build: the radix
 * passes and the ranges into the grids' outputs.  grids: the same grids in the
 * same order (GRID_E_INVAL otherwise, checked on the host before anything is
 * enqueued), now with outputs whose cap_pairs hold at least each grid's NO;
 * ws, ws_bytes, host_staging and stream as in the count, with no other build on
 * ws in between and the tuning knobs unchanged.  A grid above its capacity
 * stops every kernel before it writes and is reported by grid_workspace_status.
 * Outputs are identical to grid_build's for each grid. */
int grid_count_batched_async(const grid_desc *grids, uint32_t ngrids, void *ws, size_t ws_bytes,
                             void *host_staging, size_t staging_bytes, uint64_t *counts_host,
                             uint64_t *pair_cap, void *stream);
int grid_build_batched_counted(const grid_desc *grids, uint32_t ngrids, void *ws, size_t ws_bytes,
                               void *host_staging, size_t staging_bytes, void *stream);

/* ---- a build that allocates nothing ----------------------------------------- */

/* For callers that cannot allocate device memory or take a workspace argument
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): grid_build with its workspace in a static device array of
 * GRID_STATIC_SCRATCH_BYTES bytes that the library holds on every GPU it runs
 * on until the process ends.  Arguments, outputs, synchronisation and status
 * codes are grid_build's; the caller still owns inputs and outputs.  A build
 * whose workspace (grid_workspace_size(ntris, out->cap_pairs, res)) exceeds
 * the array returns GRID_E_NOMEM before any device work.  Every call on one
 * GPU uses that GPU's single array, which keeps the last call's contents (the
 * build clears what it needs zeroed): calls that overlap on one GPU (two host
 * threads, or two streams without ordering) race and must be serialised by
 * the caller. */
#define GRID_STATIC_SCRATCH_BYTES (64ull << 20)
int grid_build_static(const float *verts_soa, uint32_t nverts, const uint32_t *tris, uint32_t ntris,
                      const float lo[3], const float hi[3], const uint32_t res[3], grid_out *out, void *stream);

/* ---- using the grid ---------------------------------------------------------- */

/* Ray casting over a built grid, the query the grid exists to speed up
 * (Introduction; Related Work): for each ray, the closest triangle it hits.
 * The grid is (ranges, objs) of a build of these triangles with these lo, hi,
 * res (device arrays as grid_build wrote them; objs holds NO entries).
 * rays: device FP32 [6][nrays], origin x, y, z then direction x, y, z (any
 * length).  A ray is o + t d for t in [t0, t1], [0, tmax] clipped to the grid
 * box [lo, hi] by the slab test (per axis with d != 0, t = (lo - o) / d and
 * (hi - o) / d; an axis with d = 0 and o outside the box leaves nothing): only
 * hits inside the box count.  The hit test is Moller and Trumbore's in a fixed
 * order of FP32 operations (no contraction, IEEE division); a ray at a grazing
 * angle to a triangle (det^2 < 1e-8 |e1|^2 |e2|^2 |d|^2) or a degenerate
 * triangle misses; edges count.  Outputs (device): hit_t[r] = the smallest hit
 * t (+inf if none), hit_obj[r] = its triangle, the smallest id among equal t
 * (0xFFFFFFFF if none): exactly what testing every triangle gives.  Object ids
 * or vertex indices out of range never hit.  Does not synchronize the stream.
 * GRID_E_INVAL for a bad grid, null pointers, or tmax < 0 or NaN. */
int grid_raycast(const float *verts_soa, uint32_t nverts, const uint32_t *tris, uint32_t ntris,
                 const float lo[3], const float hi[3], const uint32_t res[3],
                 const uint32_t *ranges, const uint32_t *objs, const float *rays, uint32_t nrays,
                 float tmax, float *hit_t, uint32_t *hit_obj, void *stream);

/* ---- building blocks, exposed for testing and reuse ------------------------ */

/* Stable LSD radix sort of (keys, vals) by the low nbits bits of keys
 * (0 <= nbits <= 32; higher key bits must be zero).  keys_alt/vals_alt are
 * device buffers of n entries used as the other half of the double buffer; the
 * result is left in keys/vals.  The sort step of Algorithm 1 (RadixSort). */
size_t grid_sort_workspace_size(uint64_t n, uint32_t nbits);
int grid_sort_pairs(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt,
                    uint64_t n, uint32_t nbits, void *ws, size_t ws_bytes, void *stream);

/* Single-pass scans over uint32 device arrays (decoupled look-back):
 *  GRID_SCAN_EXCLUSIVE_SUM   out[i] = in[0] + ... + in[i-1] (mod 2^32);
 *                            *total (host) = full sum in 64 bits
 *  GRID_SCAN_INCLUSIVE_MAX   out[i] = max(in[0..i]);   *total = max
 *  GRID_SCAN_SEGMENTED_EXCLUSIVE_SUM  as the exclusive sum, restarting at 0
 *                            wherever flags[i] != 0 (flags: device uint32 [n]);
 *                            *total = sum of the last segment
 * These are the ExclusiveSum / InclusiveSum / SegmentedExclusiveSum steps of
 * Algorithm 1 (the inclusive scan in its max form, which the library uses to
 * spread object ids over their pair slots).  Synchronizes stream. */
enum { GRID_SCAN_EXCLUSIVE_SUM = 0, GRID_SCAN_INCLUSIVE_MAX = 1, GRID_SCAN_SEGMENTED_EXCLUSIVE_SUM = 2 };
size_t grid_scan_workspace_size(uint64_t n);
int grid_scan_u32(const uint32_t *in, const uint32_t *flags, uint32_t *out, uint64_t n, int op,
                  void *ws, size_t ws_bytes, uint64_t *total, void *stream);

/* ---- tuning ------------------------------------------------------------------- */

/* Process-wide knobs (not thread-safe against concurrent builds; set them
 * before building).  Keys:
 *   "max_digit_bits"  widest radix digit a sort pass may use, 4..11 (default 9):
 *                     a b-bit key is sorted in ceil(b / max) passes (at most 4)
 *                     whose widths differ by at most one, the wider on top
 *   "fused_expand"    1: the first radix pass regenerates its keys from the
 *                     expansion instead of reading them (default 0)
 *   "sort_shape"      workgroup shape of radix passes that read arrays:
 *                     0 = 512 threads x 16 pairs, 1 = 256 x 16, 2 = 1024 x 8,
 *                     3 = 1024 x 16 (default), 4 = 1024 x 15
 *   "small_tiles"     1 (default): a build (or batch) whose pair capacity would
 *                     fill fewer 16384-pair tiles than the GPU has CUs runs
 *                     those passes in 256 x 16 tiles whatever "sort_shape"
 *                     says; 0: "sort_shape" always
 *   "wide_lookback"   0 (default): radix passes of fewer than 2^30 pairs (by
 *                     capacity) keep 32-bit look-back words, larger ones 64-bit;
 *                     1: 64-bit words always
 *   "per_object_pairs" 1: plain builds generate their pairs with one thread per
 *                     object, each writing all of its object's pairs (the
 *                     sorted-grid pair generation of the Related Work
 *                     section, whose MakePairs kernel the Test Results section
 *                     finds dominant on architectural scenes); 0 (default):
 *                     one thread per pair (Section 3), equal work
 *                     whatever an object's size.  Ignored by batched builds and
 *                     while "fused_expand" is 1.
 *   "build_path"      plain builds (grid_build, grid_build_static): 0 (default) the
 *                     sorted path of Algorithm 1; 1 the compact path, the atomic
 *                     construction the Related Work section compares against: per-cell
 *                     counts with atomics, their exclusive scan into the range table,
 *                     a counting scatter with atomics, then each cell's object ids
 *                     sorted; 2 chosen per build after the count from its pair count
 *                     and cell count (the statistics pass the Conclusions propose;
 *                     one extra readback).  Culled and batched builds ignore it.
 *   "last_path"       (read only) the path the last plain build took, 0 or 1.
 * Outputs never depend on the knobs.  GRID_E_INVAL for an unknown key or value. */
int grid_tune_set(const char *key, int value);
int grid_tune_get(const char *key, int *value);

/* The radix plan a key of nbits bits gets under the current knobs: *passes
 * (host) passes (at most 4) of widths[0..passes) bits, lowest digit first,
 * run by the kernel built for *kernel_digit_bits-bit digits. */
int grid_sort_plan(uint32_t nbits, uint32_t *passes, uint32_t widths[4], uint32_t *kernel_digit_bits);

/* ---- kernel timing ------------------------------------------------------------ */

/* Per-kernel totals collected while tracing is on. */
typedef struct grid_trace_entry {
  char name[48];       /* kernel: zero, count_scan, plan, sink, expand, expand_hist, expand_straddle,
                          hist, makepairs, makepairs_hist, onesweep_expand, onesweep,
                          onesweep_grids, split, ranges */
  uint32_t launches;   /* launches since the last read */
  double total_ms;     /* summed event-measured duration */
} grid_trace_entry;

/* Turn tracing on (1) or off (0) for the whole process.  While on, each kernel
 * launch is bracketed by HIP events recorded on the launch's own stream. */
int grid_trace_enable(int on);

/* Restrict tracing to the launches of one kernel (a name as reported by
 * grid_trace_read, at most 47 characters), or trace every kernel again when
 * name is NULL.  Fewer events keep the traced run closer to an untraced one.
 * GRID_E_INVAL for an empty or too long name. */
int grid_trace_only(const char *name);

/* Wait for the traced launches, fold them into per-kernel totals and reset.
 * Writes up to max_entries entries (host array) and *n_entries (host) = the
 * number of distinct kernels seen. */
int grid_trace_read(grid_trace_entry *out, int max_entries, int *n_entries);

#ifdef __cplusplus
}
#endif

#endif /* GRIDBUILD_H */
