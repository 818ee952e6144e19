// Internal interface between the C ABI layer (abi.hip) and the kernels
// (trace.hip, sweep.hip).  Not installed, not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pct.h"

namespace pct {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kSegPerRound = 63;   // path segments a wavefront traces per round (64 points)
constexpr int kPathRecBytes = 128;    // workspace slot of one proton's path set-up record
constexpr int kMaxPieces = 6;      // voxel pieces one segment can yield (<= 4 when step <= voxel)
constexpr int kDedupWindow = 8;    // look-back for voxels revisited after a short excursion

// LDS row buffer of one wavefront: voxel (int32), length (float32) and dedup
// link (int16: an entry index, below emax <= 6553 since a buffer holds at
// most 64 KiB) of up to emax entries, padded to 4 bytes
__host__ __device__ inline size_t row_buf_bytes(int emax) { return ((size_t)emax * 10 + 3) & ~(size_t)3; }

// status word bits (device)
constexpr uint32_t kStNonFinite = 1u;
constexpr uint32_t kStOverflow = 2u;
constexpr uint32_t kStRowMismatch = 4u;
constexpr uint32_t kStBadIndex = 8u;   // an order entry or a cached voxel index out of range
constexpr uint32_t kStRowCap = 16u;    // the rows need more entries than their capacity
constexpr uint32_t kStCountSat = 32u;  // a block count exceeded 16 bits (stored counts unusable; not an error)

// Everything a path kernel needs, precomputed on the host and passed by value.
struct PathParams {
  // scanner and hull
  double u_in, u_out;
  double hull_ia2, hull_ib2, hull_zmin, hull_zmax;
  float step, inv_step;
  int32_t highland;
  float inv_X0;
  // prior f(s) = sum_n a_n s^n (zero-padded to 8 terms):
  //   F_p(x) = int_0^x f(s) s^p ds = x^(p+1) sum_n cF[p][n] x^n, cF = a_n / (n + p + 1)
  double cF_d[3][8];
  float cF_f[3][8];
  int32_t path_fp32;  // 1: path positions in float (reduced-precision variant)
  // grid
  int32_t nx, ny, nz;
  float dx, dy, dz;
  double idx, idy, idz, ox, oy, oz;
  float eps_len;      // pieces shorter than this (mm) are dropped
  // voxel numbering of the rows: 0 = linear (k ny + j) nx + i; 1 = in 4 x 4 x 4
  // bricks (brick (bi, bj, bk) of nbx x nby x ... bricks, then (k, j, i) in
  // it), so that the voxels a path crosses share cache lines
  int32_t brick, nbx, nby;
  // bounds
  int32_t kmax;       // max path segments
  int32_t emax;       // max row entries held in LDS per wavefront
  int32_t waves_per_block;
};

struct HistPtrs {
  const float *phi, *t_in, *v_in, *dt_in, *dv_in, *t_out, *v_out, *dt_out, *dv_out, *wepl;
};

// workspace layout
struct Workspace {
  int64_t *plan_scratch; // [plan_bt]: per (block, tile) and per block counters of a plan sizing pass
  uint32_t *status;      // [4]
  float *num;            // [M]
  uint32_t *cnt;         // [M]
  double *partials;      // [kMaxPartials]
  float *xb;             // [M] the image in brick order (rebuilt-row sweeps)
  int64_t *scan;         // [scan_len]
  int32_t *st_idx;       // [stage_slots] staged row entries of one chunk of rows (trace)
  float *st_len;         // [stage_slots]
  uint16_t *blk_cnt;     // [blk_cnt_elems] per-block voxel counts s_j of the fused sweep (or NULL)
  unsigned long long *pk; // [M] packed numerators and counts of fused counting sweeps (fused workspaces)
  void *recs;            // [rec_rows] path set-up records (kPathRecBytes each)
  int64_t rec_rows;      // n (one record per history, fused sweeps) or min(n, kStageRows) (chunks)
  void *tvs;             // [tvs_scratch_bytes(M)] TV superiorization scratch (kWsTvs) or NULL
  float *carp_xs;        // [M] CARP: one string's image (kWsCarp) or NULL
  float *carp_acc;       // [M] CARP: per-voxel sums of the string images
  uint16_t *carp_tc;     // [M] CARP: strings touching each voxel
  uint8_t *carp_touched; // [M] CARP: voxels the current string touches
};
// optional workspace regions (the `extra` flags below)
constexpr int kWsTvs = 1, kWsCarp = 2;
constexpr int64_t kMaxPartials = 1 << 16;
constexpr int64_t kScanChunk = 4096;
constexpr int64_t kStageRows = 1 << 20;  // rows traced per staging chunk

// the per-block counts of the fused sweep (n_blocks x M uint16) are kept only
// up to this size; above it the counts are re-formed with atomics every sweep
constexpr int64_t kMaxBlkCntBytes = int64_t(32) << 30;
// recs_all: one path record per history (the fused sweeps set every proton up
// once per call), else records for one chunk of kStageRows rows
size_t workspace_bytes(int64_t M, int64_t n_hist, int64_t plan_bt, int64_t stage_slots = 0,
                       int64_t blk_cnt_elems = 0, bool recs_all = false, int extra = 0);
Workspace carve_workspace(void *base, int64_t M, int64_t n_hist, int64_t plan_bt, int64_t stage_slots = 0,
                          int64_t blk_cnt_elems = 0, bool recs_all = false, int extra = 0);

// ---- tiled sweep plan (cached rows regrouped by block and spatial tile)
constexpr int kTX = 16, kTY = 16, kTZ = 8;           // tile of 2048 voxels
constexpr int kTileVox = kTX * kTY * kTZ;
constexpr int kRowBits = 18;                          // row-in-block index bits
constexpr int64_t kMaxPlanBlock = int64_t(1) << kRowBits;
// layout-A entry (16 bits): bit 0 valid, bit 1 last entry of a piece, bits
// 2..12 voxel in tile
__host__ __device__ inline uint16_t pack_entry(uint32_t last, uint32_t vox) {
  return (uint16_t)(1u | (last << 1) | (vox << 2));
}

struct PlanView {
  int64_t n, B, nb, T, E, C, R, P, maxc;
  int32_t ntx, nty, ntz, nx, ny, nz;
  int32_t len_dtype;
  float len_unit;
  int64_t *bt_off;          // [nb*T + 1] entry offsets of each (block, tile) list (multiples of 64)
  unsigned long long *bt_cur;  // [nb*T] fill cursors
  uint32_t *ord_row;        // [R] per piece end (global ordinal): its row in the block
  float *rvals;             // [B] r_i of one block
  uint64_t *end_mask;       // [C] lanes that close a piece (or a chunk)
  int64_t *chunk_first_end; // [C + 1]
  uint16_t *packed;         // [E] layout-A entries (see pack_entry)
  void *len;                // [E] float or half
  int64_t *ref_base;        // [n + 1]
  int32_t *ref_cnt;         // [n]
  uint32_t *refs;           // [R] per row, entry positions that close its pieces
  uint32_t *end_slot;       // [R] per piece end (chunk order): its row-ordered slot in the block
  float *b_perm;            // [n] b in block order
  double *n2_perm;          // [n] ||a||^2 in block order
  float *partial;           // [P] per-piece partial dot products of one block, in row order
  double *res_part;         // [kResidAllGrid] residual partial sums (one per workgroup)
  void *meta;               // [C] build only: per chunk, end_mask and chunk_first_end side by side (16 B)
};
constexpr int kResidAllGrid = 1024;     // workgroups of the whole-plan residual rows pass

hipError_t launch_plan_count(const int64_t *row_ptr, const int32_t *idx, const int64_t *order, int64_t n, int64_t B,
                             int64_t M, const PlanView &V, int64_t *bt_cnt, int64_t *row_cap, int64_t *blk_cap,
                             uint32_t *status, hipStream_t s);
hipError_t launch_plan_fill(const int64_t *row_ptr, const int32_t *idx, const void *len_in, int32_t len_in_dtype,
                            const int64_t *order, const float *wepl, const double *norm2, int64_t M,
                            const PlanView &V, uint32_t *status, hipStream_t s);
hipError_t launch_plan_pad_counts(int64_t *cnt, int64_t k, hipStream_t s);
hipError_t launch_plan_chunks(const PlanView &V, hipStream_t s);
hipError_t launch_plan_ref_ordinals(const PlanView &V, hipStream_t s);
hipError_t launch_copy_i64_to_u64(unsigned long long *dst, const int64_t *src, int64_t k, hipStream_t s);
hipError_t launch_plan_dot(const PlanView &V, int64_t b, const float *x, hipStream_t s);
hipError_t launch_plan_rows(const PlanView &V, int64_t b, hipStream_t s);
hipError_t launch_plan_scatter(const PlanView &V, int64_t b, float *x, const uint8_t *mask, float lambda, hipStream_t s);
hipError_t launch_plan_dot_all(const PlanView &V, const float *x, hipStream_t s);
hipError_t launch_plan_resid_all(const PlanView &V, double *partials, hipStream_t s);
hipError_t launch_sum_partials(const double *partials, int64_t np, double *out, int sqrt_it, hipStream_t s);

// launchers (return hipError_t of the launch)
// per-proton set-up records of rows [first, first + count) (through order
// when given) into recs (kPathRecBytes each)
hipError_t launch_path_setup(const PathParams &P, const HistPtrs &H, const int64_t *order, int64_t first,
                             int64_t count, int64_t n, void *recs, uint32_t *status, bool flag_nonfinite,
                             hipStream_t s);
hipError_t launch_trace_stage(const PathParams &P, const void *recs, int64_t i0, int64_t nrows, int64_t *cnt,
                              int32_t *st_idx, float *st_len, double *norm2, uint32_t *status, hipStream_t s);
hipError_t launch_trace_compact(int64_t i0, int64_t nrows, const int64_t *row_ptr, const int32_t *st_idx,
                                const float *st_len, int emax, int32_t *idx, void *len, int32_t len_dtype,
                                float len_scale, int64_t cap, uint32_t *status, hipStream_t s);
// counts at row_ptr[i0 + 1 .. i0 + nrows] -> offsets continuing from row_ptr[i0]
// (row_ptr[0] is set to 0 when i0 == 0)
hipError_t launch_scan_rows(int64_t *row_ptr, int64_t i0, int64_t nrows, int64_t *scan_tmp, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t s);
hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t s);
hipError_t launch_fill_u8(uint8_t *p, int64_t n, uint8_t v, hipStream_t s);

hipError_t launch_mask(float *x, const uint8_t *mask, int64_t M, hipStream_t s);
// xb = x in brick order (zero in the padding of partial bricks)
hipError_t launch_to_bricks(const PathParams &P, const float *x, float *xb, int64_t Mb, hipStream_t s);
hipError_t launch_project_cached(const int64_t *row_ptr, const int32_t *idx, const void *len, int32_t len_dtype,
                                 float len_unit, const double *norm2, const float *b, const int64_t *order,
                                 int64_t first, int64_t count, int64_t n, int64_t M, const float *x, float *num,
                                 uint32_t *cnt, uint32_t *status, hipStream_t s);
// rows of block positions [first, first + count): records recs[order[first + q]]
// (global: one record per history) or recs[q] (one chunk's records); cnt
// NULL: the block counts are not formed; pk (with cnt): numerators and counts
// added as one packed 64-bit integer per entry (count field of pk_bits bits,
// numerator in units of 2^-pk_k; see packed_counts)
hipError_t launch_project_fused(const PathParams &P, const void *recs, const int64_t *order, int64_t first, int64_t n,
                                bool global, int64_t count, const float *x, float *num, uint32_t *cnt,
                                uint32_t *status, hipStream_t s, unsigned long long *pk = nullptr, int pk_bits = 0,
                                int pk_k = 0);
// mode 0: counts from cnt (cleared); 1: also store them as uint16 into blk_cnt;
// 2: counts read from blk_cnt (cnt unused).  Bp (or NULL): num, cnt and
// blk_cnt are in brick order over Mb voxels, and xb (x in brick order) is
// kept equal to x
hipError_t launch_apply_counts(float *x, float *num, uint32_t *cnt, uint16_t *blk_cnt, int mode, const uint8_t *mask,
                               int64_t M, float lambda, uint32_t *status, hipStream_t s, uint8_t *touched = nullptr,
                               const PathParams *Bp = nullptr, float *xb = nullptr, int64_t Mb = 0,
                               unsigned long long *pk = nullptr, int pk_bits = 0, int pk_k = 0);
// Packed numerator-and-count atomics for blocks of B rows: a voxel's block
// count is at most B, so a count field of `bits` bits with 2^bits > B never
// overflows; with contributions below 4 in magnitude (|fixed| < 2^(k + 2))
// the numerator field (64 - bits, signed) holds any sum of B of them when
// k + 2 + 2 bits <= 63, and one fixed value fits 32 bits when k <= 29.  Used
// when k >= 20 (blocks of up to 2^20 - 1 rows).
inline bool packed_counts(int64_t B, int &bits, int &k) {
  bits = 1;
  while (bits < 62 && (int64_t(1) << bits) <= B) ++bits;
  k = 61 - 2 * bits;
  if (k > 29) k = 29;
  return k >= 20;
}
// CARP: xs into the per-voxel sums of the strings touching it (touched
// cleared), then x = mean where some string touched (acc, tc cleared)
hipError_t launch_carp_accumulate(const float *xs, uint8_t *touched, float *acc, uint16_t *tc, int64_t M,
                                  hipStream_t s);
hipError_t launch_carp_average(float *x, float *acc, uint16_t *tc, int64_t M, hipStream_t s);
hipError_t launch_copy_f32(const float *a, float *b, int64_t n, hipStream_t s);
// total-variation superiorization steps on x (tvs.hip); scratch of
// tvs_scratch_bytes(M) bytes; state: device double[8], state[0] = step size
size_t tvs_scratch_bytes(int64_t M);
hipError_t launch_tvs(int32_t nx, int32_t ny, int32_t nz, float *x, const uint8_t *mask, int32_t n_steps,
                      int32_t max_trials, double a, double eps, double *state, void *scratch, hipStream_t s);
// space carving (tvs.hip): hull[j] = 0 for every voxel crossed for more than
// min_len mm by the straight line of a history with WEPL < wepl_max; *used
// += histories used
hipError_t launch_carve(const PathParams &P, const HistPtrs &H, int64_t n, double wepl_max, double min_len,
                        uint8_t *hull, unsigned long long *used, hipStream_t s);
hipError_t launch_art(const int64_t *row_ptr, const int32_t *idx, const void *len, int32_t len_dtype,
                      float len_unit, const double *norm2, const float *b, const int64_t *order, int64_t n,
                      int64_t M, float *x, const uint8_t *mask, float lambda, uint32_t *status, hipStream_t s);
hipError_t launch_residual_cached(const int64_t *row_ptr, const int32_t *idx, const void *len, int32_t len_dtype,
                                  float len_unit, const float *b, int64_t n, int64_t M, const float *x,
                                  double *partials, double *out, hipStream_t s);
// one chunk of the fused residual (kResidFusedGrid partial sums, stored or,
// with accumulate, added), then the final ordered sum
constexpr int kResidFusedGrid = 4096;
hipError_t launch_residual_fused(const PathParams &P, const void *recs, int64_t n, const float *x, double *partials,
                                 uint32_t *status, bool accumulate, hipStream_t s);
hipError_t launch_residual_final(const double *partials, int64_t np, double *out, hipStream_t s);
// *out = NaN if any status bit is set (asynchronous error report)
hipError_t launch_poison_on_status(double *out, const uint32_t *status, hipStream_t s);
// memory-path microbenchmarks (probe.hip)
constexpr int64_t kProbeGrid = 2048;
size_t probe_bytes(int kind, int64_t region, int64_t n_ops, int64_t grid);
hipError_t launch_probe(int kind, void *buf, int64_t region, int64_t n_ops, int64_t grid, hipStream_t s);
hipError_t launch_roi(const float *x, const uint8_t *labels, int64_t M, int32_t n_labels, double *sums,
                      int64_t *counts, hipStream_t s);

}  // namespace pct
