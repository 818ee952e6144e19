// Tiled sweep plan: the cached rows of A regrouped, block by block, into
// spatial tiles of 16 x 16 x 8 voxels, so that one DROP block (paper Sec. 2.1)
// runs without global atomics:
//
//   k_plan_dot     workgroups per (block, tile) list, x of the tile staged in
//                  LDS: each 64-entry chunk multiplies lengths by x and sums
//                  each piece (a run of one row's entries) with a segmented
//                  wave scan -> one partial dot product per piece end, stored
//                  next to the other partials of its row;
//   k_plan_rows    one thread per row of the block: adds the row's partials in
//                  a fixed order -> r_i = (b_i - a_i.x)/||a_i||^2;
//   k_plan_scatter one workgroup per (block, tile) list: each entry's
//                  r_i a_ij and count are added into LDS images of the tile
//                  (the numerators as exact 64-bit fixed-point integers),
//                  then x_j += lambda num_j / s_j.
//
// Entries are packed in 16 bits (voxel in tile, valid and piece-closing
// flags) next to their lengths (float32 or float16), so both passes stream the
// same lists with coalesced loads.
#include <cmath>

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "path_device.h"

namespace pct {

__device__ __forceinline__ int voxel_tile(int j, const PlanView &V, int &local) {
  const int i = j % V.nx;
  const int r = j / V.nx;
  const int jj = r % V.ny;
  const int k = r / V.ny;
  local = ((k % kTZ) * kTY + (jj % kTY)) * kTX + (i % kTX);
  return ((k / kTZ) * V.nty + (jj / kTY)) * V.ntx + (i / kTX);
}

__device__ __forceinline__ int tile_voxel(int t, int local, const PlanView &V, bool &inside) {
  const int tx = t % V.ntx, r = t / V.ntx, ty = r % V.nty, tz = r / V.nty;
  const int lx = local % kTX, ly = (local / kTX) % kTY, lz = local / (kTX * kTY);
  const int i = tx * kTX + lx, j = ty * kTY + ly, k = tz * kTZ + lz;
  inside = i < V.nx && j < V.ny && k < V.nz;
  return (k * V.ny + j) * V.nx + i;
}

// A row is read 64 entries at a time; within such a window a new piece begins
// at lane 0 and wherever the tile changes.
__device__ __forceinline__ int piece_start_lane(uint64_t starts, int lane) {
  const uint64_t m = starts & ((lane == 63) ? ~0ull : ((2ull << lane) - 1));
  return 63 - __clzll(m);
}
__device__ __forceinline__ int piece_end_lane(uint64_t starts, int s, int nv) {
  const uint64_t above = (s == 63) ? 0ull : (starts >> (s + 1));
  const int nxt = above ? (s + 1 + __ffsll((long long)above) - 1) : 64;
  return nxt < nv ? nxt : nv;  // one past the last lane of the piece
}

// Sizing / capacity pass: entries per (block, tile) and reference slots per
// row.  A workgroup takes up to kCountRows rows of one block; entry counts are
// gathered in an LDS histogram over tiles (when the tiles fit) and added to
// the global counters once per workgroup.
constexpr int kCountRows = 1024;
constexpr int kCountHist = 4096;
constexpr int kCountWin = 4;

__global__ void __launch_bounds__(256) k_plan_count(const int64_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ idx,
                                                    const int64_t *__restrict__ order, int64_t n, int64_t B,
                                                    int64_t M, PlanView V, int64_t *bt_cnt, int64_t *row_cap,
                                                    int64_t *blk_cap, uint32_t *status) {
  __shared__ uint32_t s_hist[kCountHist];
  __shared__ unsigned long long s_cap;
  const int lane = wave_lane();
  const int64_t wg_per_block = (B + kCountRows - 1) / kCountRows;
  const int64_t b = blockIdx.x / wg_per_block;
  const int64_t r0 = (blockIdx.x % wg_per_block) * kCountRows;
  const int64_t q0 = b * B + r0;
  int64_t q1 = b * B + (r0 + kCountRows < B ? r0 + kCountRows : B);
  if (q1 > n) q1 = n;
  const bool use_lds = V.T <= kCountHist;
  if (use_lds)
    for (int e = threadIdx.x; e < V.T; e += blockDim.x) s_hist[e] = 0u;
  if (threadIdx.x == 0) s_cap = 0ull;
  __syncthreads();
  for (int64_t q = q0 + threadIdx.x / kWave; q < q1; q += blockDim.x / kWave) {
    const int64_t i = order ? order[q] : q;
    if ((uint64_t)i >= (uint64_t)n) {
      if (lane == 0) atomicOr(status, kStBadIndex);
      continue;
    }
    const int64_t e0 = row_ptr[i], e1 = row_ptr[i + 1];
    int64_t pieces = 0;
    // kCountWin windows of 64 entries per round, their loads issued together
    for (int64_t w0 = e0; w0 < e1; w0 += kCountWin * kWave) {
      int jv[kCountWin];
#pragma unroll
      for (int k = 0; k < kCountWin; ++k) {
        const int64_t e = w0 + k * kWave + lane;
        jv[k] = e < e1 ? idx[e] : -1;
      }
#pragma unroll
      for (int k = 0; k < kCountWin; ++k) {
        const bool valid = w0 + k * kWave + lane < e1;
        int t = -1, local = 0;
        if (valid) {
          if ((uint32_t)jv[k] >= (uint64_t)M)
            atomicOr(status, kStBadIndex);
          else
            t = voxel_tile(jv[k], V, local);
        }
        int tp = lane_prev(t);
        if (lane == 0) tp = -2;
        const bool start = valid && (lane == 0 || t != tp);
        const uint64_t starts = __ballot(start);
        const int nv = __popcll(__ballot(valid));
        if (start && t >= 0) {
          const int end = piece_end_lane(starts, lane, nv);
          if (use_lds)
            atomicAdd(&s_hist[t], (uint32_t)(end - lane));
          else
            atomicAdd((unsigned long long *)&bt_cnt[b * V.T + t], (unsigned long long)(end - lane));
        }
        pieces += __popcll(starts);
      }
    }
    if (lane == 0) {
      if (row_cap) row_cap[q + 1] = 2 * pieces;
      atomicAdd(&s_cap, (unsigned long long)(2 * pieces));
    }
  }
  __syncthreads();
  if (use_lds)
    for (int e = threadIdx.x; e < V.T; e += blockDim.x)
      if (s_hist[e]) atomicAdd((unsigned long long *)&bt_cnt[b * V.T + e], (unsigned long long)s_hist[e]);
  if (threadIdx.x == 0 && blk_cap && s_cap) atomicAdd((unsigned long long *)&blk_cap[b], s_cap);
}

// round each (block, tile) count up to a whole number of 64-entry chunks
__global__ void k_plan_pad(int64_t *cnt, int64_t k) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < k; e += stride)
    cnt[e] = (cnt[e] + kWave - 1) / kWave * kWave;
}

__global__ void k_copy_i64_u64(unsigned long long *dst, const int64_t *src, int64_t k) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < k; e += stride)
    dst[e] = (unsigned long long)src[e];
}

// Fill pass: place each piece in its (block, tile) list, record where each
// row's pieces end, gather b and ||a||^2 into block order.  Wavefronts walk
// the rows of the block order (persistent grid).  A row is taken kFillWin
// windows of 64 entries at a time: the windows' entry loads are issued
// together, then their list reservations (one returning atomic per piece),
// then their stores, so a row costs one load and one atomic round trip per
// kFillWin windows instead of per window; the next row's history index and
// CSR bounds are loaded while the current row is placed.
#ifndef PCT_FILL_WIN
#define PCT_FILL_WIN 3
#endif
#ifndef PCT_FILL_MINW
#define PCT_FILL_MINW 8
#endif
#ifndef PCT_FILL_WGS_PER_CU
#define PCT_FILL_WGS_PER_CU 8
#endif
constexpr int kFillWin = PCT_FILL_WIN;

template <int LDI>
__device__ __forceinline__ void fill_row(const int32_t *__restrict__ idx, const void *__restrict__ len_in, int64_t M,
                                         const PlanView &V, uint32_t *status, int64_t q, int64_t e0, int64_t e1,
                                         int lane) {
  const int64_t b = q / V.B;
  const int64_t rbase = V.ref_base[q], rcap = V.ref_base[q + 1] - rbase;
  int64_t nref = 0;
  for (int64_t w0 = e0; w0 < e1; w0 += kFillWin * kWave) {
    int jv[kFillWin];
    float l[kFillWin];
    __half lh[kFillWin];
#pragma unroll
    for (int k = 0; k < kFillWin; ++k) {
      const int64_t e = w0 + k * kWave + lane;
      jv[k] = -1;
      l[k] = 0.f;
      lh[k] = __float2half(0.f);
      if (e < e1) {
        jv[k] = idx[e];
        if (LDI == 0)
          l[k] = reinterpret_cast<const float *>(len_in)[e];
        else
          lh[k] = reinterpret_cast<const __half *>(len_in)[e];
      }
    }
    int t[kFillWin], local[kFillWin], end[kFillWin], nv[kFillWin];
    uint64_t starts[kFillWin];
    unsigned long long pos[kFillWin];
    int64_t lim[kFillWin];
#pragma unroll
    for (int k = 0; k < kFillWin; ++k) {
      const bool valid = w0 + k * kWave + lane < e1;
      t[k] = -1;
      local[k] = 0;
      if (valid && (uint32_t)jv[k] < (uint64_t)M) t[k] = voxel_tile(jv[k], V, local[k]);
      int tp = lane_prev(t[k]);
      if (lane == 0) tp = -2;
      const bool start = valid && (lane == 0 || t[k] != tp);
      starts[k] = __ballot(start);
      nv[k] = __popcll(__ballot(valid));
      pos[k] = 0;
      end[k] = 0;
      lim[k] = 0;
      if (start && t[k] >= 0) {
        end[k] = piece_end_lane(starts[k], lane, nv[k]);
        pos[k] = atomicAdd(&V.bt_cur[b * V.T + t[k]], (unsigned long long)(end[k] - lane));
        lim[k] = V.bt_off[b * V.T + t[k] + 1];
      }
    }
#pragma unroll
    for (int k = 0; k < kFillWin; ++k) {
      if (nv[k] == 0) break;  // wave-uniform: no entries from this window on
      const bool valid = lane < nv[k];
      const bool ok = end[k] == 0 || (int64_t)pos[k] + (end[k] - lane) <= lim[k];
      const int s = valid ? piece_start_lane(starts[k], lane) : 0;
      const unsigned long long ps = __shfl(pos[k], s, kWave);
      const int pe = __shfl(end[k], s, kWave);
      const bool pok = __shfl((int)ok, s, kWave) != 0;
      const int ts = __shfl(t[k], s, kWave);
      const int64_t p = (int64_t)ps + (lane - s);
      const bool write = valid && ts >= 0 && pok;
      if (valid && !pok && lane == s) atomicOr(status, kStOverflow);
      const bool last = lane == pe - 1;
      bool is_ref = false;
      if (write) {
        V.packed[p] = pack_entry(last ? 1u : 0u, (uint32_t)local[k]);
        if (V.len_dtype == 0)
          reinterpret_cast<float *>(V.len)[p] = LDI == 0 ? l[k] : __half2float(lh[k]) * V.len_unit;
        else
          reinterpret_cast<__half *>(V.len)[p] = LDI == 1 ? lh[k] : __float2half(l[k] / V.len_unit);
        is_ref = last || ((p & (kWave - 1)) == kWave - 1);
      }
      const uint64_t rm = __ballot(is_ref);
      if (is_ref) {
        const int64_t kk = nref + __popcll(rm & ((1ull << lane) - 1));
        if (kk < rcap)
          V.refs[rbase + kk] = (uint32_t)p;
        else
          atomicOr(status, kStOverflow);
      }
      nref += __popcll(rm);
    }
  }
  if (lane == 0) V.ref_cnt[q] = (int32_t)(nref < rcap ? nref : rcap);
}

template <int LDI>
__global__ void __launch_bounds__(256, PCT_FILL_MINW) k_plan_fill(const int64_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ idx, const void *__restrict__ len_in,
                                                   const int64_t *__restrict__ order, const float *__restrict__ wepl,
                                                   const double *__restrict__ norm2, int64_t M, PlanView V,
                                                   uint32_t *status) {
  const int lane = wave_lane();
  const int64_t nw = (int64_t)gridDim.x * 4;
  int64_t q = (int64_t)blockIdx.x * 4 + uniform((int)(threadIdx.x / kWave));
  if (q >= V.n) return;
  // history index and CSR bounds of row q; history index of the row after it
  int64_t i = order ? order[q] : q;
  int64_t i_next = q + nw < V.n ? (order ? order[q + nw] : q + nw) : 0;
  bool bad = (uint64_t)i >= (uint64_t)V.n;
  int64_t e0 = bad ? 0 : row_ptr[i], e1 = bad ? 0 : row_ptr[i + 1];
  for (; q < V.n; q += nw) {
    // loads for the next row, in flight while this one is placed
    const bool has_next = q + nw < V.n;
    const bool bad_next = !has_next || (uint64_t)i_next >= (uint64_t)V.n;
    const int64_t e0n = bad_next ? 0 : row_ptr[i_next], e1n = bad_next ? 0 : row_ptr[i_next + 1];
    const int64_t q2 = q + 2 * nw;
    const int64_t i_next2 = q2 < V.n ? (order ? order[q2] : q2) : 0;
    float bq = 0.f;
    double nq = 0.0;
    if (!bad && lane == 0) {
      bq = wepl[i];
      nq = norm2[i];
    }
    if (!bad) fill_row<LDI>(idx, len_in, M, V, status, q, e0, e1, lane);
    if (lane == 0) {
      if (!bad) {
        V.b_perm[q] = bq;
        V.n2_perm[q] = nq;
      } else {
        atomicOr(status, kStBadIndex);
      }
    }
    i = i_next;
    i_next = i_next2;
    bad = bad_next;
    e0 = e0n;
    e1 = e1n;
  }
}

// lanes that close a piece (or a chunk) and their count per chunk; a
// wavefront takes kEndsChunks consecutive chunks, loads first
constexpr int kEndsChunks = 4;

__global__ void __launch_bounds__(256) k_plan_chunk_ends(PlanView V) {
  const int lane = wave_lane();
  const int64_t cw = ((int64_t)blockIdx.x * 4 + threadIdx.x / kWave) * kEndsChunks;
  if (cw >= V.C) return;
  uint32_t v[kEndsChunks];
#pragma unroll
  for (int q = 0; q < kEndsChunks; ++q) v[q] = cw + q < V.C ? (uint32_t)V.packed[(cw + q) * kWave + lane] : 0u;
#pragma unroll
  for (int q = 0; q < kEndsChunks; ++q) {
    const bool valid = v[q] & 1u;
    const bool close = valid && (((v[q] >> 1) & 1u) || lane == kWave - 1);
    const uint64_t m = __ballot(close);
    if (lane == 0 && cw + q < V.C) {
      V.end_mask[cw + q] = m;
      V.chunk_first_end[cw + q + 1] = __popcll(m);
    }
  }
}

template <int LD>
__device__ __forceinline__ float plan_len(const PlanView &V, int64_t p) {
  if constexpr (LD == 0)
    return __builtin_nontemporal_load(reinterpret_cast<const float *>(V.len) + p);
  else
    return __half2float(__builtin_bit_cast(
               __half, __builtin_nontemporal_load(reinterpret_cast<const uint16_t *>(V.len) + p))) * V.len_unit;
}

// Partial dot products of every piece of block b.  kDotSplit workgroups of
// kDotWaves wavefronts per (block, tile) list, each on an equal share of
// its chunks (many more workgroups than CUs can hold at once, so the work
// spreads evenly): x of the tile is staged in LDS (the entries then read it
// with LDS gathers instead of L1/L2 gathers).  A wavefront walks batches of
// kDotBatch consecutive chunks (batch j, j + kDotWaves, ...) in a
// three-stage software pipeline: stage A loads a batch's entries, lengths and
// per-chunk piece-end ordinals; stage B loads the end_slot slices of the
// batch's chunks (it needs stage A's ordinals); stage C reduces the batch.
// While batch j is reduced, stage A of j + 2 and stage B of j + 1 are in
// flight.  Every load is issued unconditionally (addresses clamped into the
// list, results masked), so the wait counts stay static.
#ifndef PCT_DOT_BATCH
#define PCT_DOT_BATCH 3
#endif
constexpr int kDotBatch = PCT_DOT_BATCH;
#ifndef PCT_DOT_SPLIT
#define PCT_DOT_SPLIT 4
#endif
#ifndef PCT_DOT_WAVES
#define PCT_DOT_WAVES 8
#endif
constexpr int kDotSplit = PCT_DOT_SPLIT;  // workgroups per (block, tile) list, each on an equal share of its chunks
constexpr int kDotWaves = PCT_DOT_WAVES;  // wavefronts per dot workgroup
constexpr int kDotThreads = kDotWaves * kWave;
static_assert(kTileVox % kDotThreads == 0, "a dot workgroup stages the tile's x in whole rounds");
constexpr int64_t kDotAllMaxWgs = int64_t(1) << 20;  // workgroups per launch of the whole-plan dot

struct DotStageA {
  uint32_t v[kDotBatch];  // entry codes (0 past the share's end)
  float l[kDotBatch];     // lengths
  int64_t fe[kDotBatch];  // first piece-end ordinal of each chunk
  int ne[kDotBatch];      // piece ends of each chunk (>= 1 for any chunk holding an entry)
};

template <int LD>
__device__ __forceinline__ void dot_stage_a(const PlanView &V, int64_t ca, int64_t cb, int64_t j, int lane,
                                            DotStageA &a) {
#pragma unroll
  for (int k = 0; k < kDotBatch; ++k) {
    const int64_t c0 = ca + j * kDotBatch + k;
    const bool in = c0 < cb;
    const int64_t c = in ? c0 : cb - 1;
    const int64_t p = c * kWave + lane;
    const uint32_t v = (uint32_t)__builtin_nontemporal_load(V.packed + p);
    const float l = plan_len<LD>(V, p);
    a.v[k] = in ? v : 0u;
    a.l[k] = l;
    const int64_t f0 = V.chunk_first_end[c], f1 = V.chunk_first_end[c + 1];
    a.fe[k] = f0;
    a.ne[k] = (int)(f1 - f0);
  }
}

__device__ __forceinline__ void dot_stage_b(const PlanView &V, const DotStageA &a, int lane,
                                            uint32_t (&es)[kDotBatch]) {
#pragma unroll
  for (int k = 0; k < kDotBatch; ++k) {
    const int n = a.ne[k] > 0 ? a.ne[k] : 1;
    es[k] = V.end_slot[a.fe[k] + (lane < n ? lane : n - 1)];
  }
}

// x of tile t (2048 voxels, zero outside the grid) -> s_x; every thread
// issues its kTileVox / kDotThreads loads before storing any (voxels outside
// the grid load voxel 0 and store 0)
__device__ __forceinline__ void stage_tile_x(const PlanView &V, int64_t t, const float *__restrict__ x, float *s_x) {
  constexpr int kPer = kTileVox / kDotThreads;
  const int tx = (int)(t % V.ntx), r = (int)(t / V.ntx), ty = r % V.nty, tz = r / V.nty;
  float xv[kPer];
  bool in[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int i = (int)threadIdx.x + u * kDotThreads;
    const int ix = tx * kTX + (i & 15), iy = ty * kTY + ((i >> 4) & 15), iz = tz * kTZ + (i >> 8);
    in[u] = ix < V.nx && iy < V.ny && iz < V.nz;
    xv[u] = x[in[u] ? ((int64_t)iz * V.ny + iy) * V.nx + ix : 0];
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) s_x[(int)threadIdx.x + u * kDotThreads] = in[u] ? xv[u] : 0.0f;
}

// ALL: one launch over the lists of blocks b0, b0 + 1, ... (kDotSplit x T
// workgroups per block), each block's partials stored at its rows' absolute
// slots in the build-only reference array (free once the plan is built), so
// that a residual pass over every block needs one launch instead of one per
// block.
template <int LD, bool ALL>
__global__ void __launch_bounds__(kDotThreads) k_plan_dot(PlanView V, int64_t b0, const float *__restrict__ x) {
  __shared__ float s_x[kTileVox];
  const int lane = wave_lane();
  const int64_t per_blk = V.T * kDotSplit;
  const int64_t b = ALL ? b0 + (int64_t)blockIdx.x / per_blk : b0;
  const int64_t w = ALL ? (int64_t)blockIdx.x % per_blk : (int64_t)blockIdx.x;
  const int64_t t = w / kDotSplit;
  const int part = (int)(w % kDotSplit);
  float *__restrict__ out = ALL ? reinterpret_cast<float *>(V.refs) + V.ref_base[b * V.B] : V.partial;
  const int64_t lk = b * V.T + t;
  const int64_t la = V.bt_off[lk] / kWave, lb = V.bt_off[lk + 1] / kWave;
  const int64_t ca = la + (lb - la) * part / kDotSplit, cb = la + (lb - la) * (part + 1) / kDotSplit;
  if (ca == cb) return;  // the whole workgroup leaves
  stage_tile_x(V, t, x, s_x);
  __syncthreads();
  const int64_t nbat = (cb - ca + kDotBatch - 1) / kDotBatch;
  int64_t j = uniform((int)(threadIdx.x / kWave));
  if (j >= nbat) return;
  // batches past the last are loaded as the last one again (never reduced)
  const int64_t jlast = j + (nbat - 1 - j) / kDotWaves * kDotWaves;
  DotStageA a0, a1, a2;
  uint32_t e0[kDotBatch], e1[kDotBatch];
  dot_stage_a<LD>(V, ca, cb, j, lane, a0);
  dot_stage_a<LD>(V, ca, cb, j + kDotWaves <= jlast ? j + kDotWaves : jlast, lane, a1);
  dot_stage_b(V, a0, lane, e0);
  for (;;) {
    const int64_t j1 = j + kDotWaves, j2 = j + 2 * kDotWaves;
    dot_stage_b(V, a1, lane, e1);
    dot_stage_a<LD>(V, ca, cb, j2 <= jlast ? j2 : jlast, lane, a2);
    const int nc = (int)(cb - (ca + j * kDotBatch) < kDotBatch ? cb - (ca + j * kDotBatch) : kDotBatch);
#pragma unroll
    for (int k = 0; k < kDotBatch; ++k) {
      if (k >= nc) continue;  // nc is wave-uniform
      const uint32_t v = a0.v[k];
      const bool valid = v & 1u;
      const float xv = valid ? s_x[(v >> 2) & (kTileVox - 1)] : 0.f;
      const bool close = valid && (((v >> 1) & 1u) || lane == kWave - 1);
      const uint64_t m = __ballot(close);
      // a piece's sum is the difference of the prefix sums at its closing lane
      // and at the previous closing lane
      const float S = wave_incl_scan_dpp(valid ? a0.l[k] * xv : 0.0f);
      const uint64_t below = m & ((1ull << lane) - 1);
      const int prev = below ? 63 - __clzll(below) : lane;
      const float Sp = __shfl(S, prev, kWave);
      // the end_slot entry of this chunk's n-th piece end sits in lane n
      const uint32_t slot = (uint32_t)__shfl((int)e0[k], __popcll(below), kWave);
      if (close) out[slot] = below ? S - Sp : S;
    }
    if (j1 > jlast) break;
    j = j1;
    a0 = a1;
    a1 = a2;
#pragma unroll
    for (int k = 0; k < kDotBatch; ++k) e0[k] = e1[k];
  }
}

// Per chunk, its piece-end mask and first ordinal side by side (16 B), so
// that k_plan_ref_ordinals, which visits chunks in row order (scattered),
// fetches one cache line per reference instead of two (a build-only area of
// the plan).
struct __align__(16) ChunkMeta {
  uint64_t mask;
  int64_t first;
};

__global__ void __launch_bounds__(256) k_plan_chunk_meta(PlanView V, ChunkMeta *meta) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < V.C; c += stride) {
    ChunkMeta m;
    m.mask = V.end_mask[c];
    m.first = V.chunk_first_end[c];
    meta[c] = m;
  }
}

// references hold entry positions after the fill pass; record, for every
// piece end (global ordinal in chunk order), the row-ordered slot of its
// reference, so k_plan_dot can store each partial next to the other partials
// of its row, and its row in the block, so k_plan_scatter can give it r
template <bool META>
__global__ void __launch_bounds__(256) k_plan_ref_ordinals(PlanView V, const ChunkMeta *__restrict__ meta) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= V.n) return;
  const int64_t b = q / V.B;
  const int64_t rb = V.ref_base[b * V.B];
  const int64_t k0 = V.ref_base[q];
  const int nref = V.ref_cnt[q];
  constexpr int U = 4;  // references whose loads are issued together
  for (int k = 0; k < nref; k += U) {
    uint32_t p[U];
#pragma unroll
    for (int u = 0; u < U; ++u) p[u] = k + u < nref ? V.refs[k0 + k + u] : 0u;
    uint64_t em[U];
    int64_t fe[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      em[u] = 0ull;
      fe[u] = 0;
      if (k + u < nref) {
        if (META) {
          const ChunkMeta m = meta[p[u] / kWave];
          em[u] = m.mask;
          fe[u] = m.first;
        } else {
          em[u] = V.end_mask[p[u] / kWave];
          fe[u] = V.chunk_first_end[p[u] / kWave];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (k + u >= nref) break;
      const int l = p[u] & (kWave - 1);
      const int64_t ord = fe[u] + __popcll(em[u] & ((1ull << l) - 1));
      V.end_slot[ord] = (uint32_t)(k0 + k + u - rb);
      V.ord_row[ord] = (uint32_t)(q - b * V.B);
    }
  }
}

// sum of a row's piece partials (p: its first slot); four references per step
// so that their loads overlap (fixed summation order, so results are
// reproducible)
__device__ __forceinline__ float row_dot(const float *p, int nref) {
  float d = 0.0f;
  int k = 0;
  for (; k + 4 <= nref; k += 4) d += (p[k] + p[k + 1]) + (p[k + 2] + p[k + 3]);
  for (; k < nref; ++k) d += p[k];
  return d;
}

// r_i of every row of block b
__global__ void __launch_bounds__(256) k_plan_rows(PlanView V, int64_t b) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t q = b * V.B + r;
  if (r >= V.B || q >= V.n) return;
  const int nref = V.ref_cnt[q];
  const float d = row_dot(V.partial + (V.ref_base[q] - V.ref_base[b * V.B]), nref);
  V.rvals[r] = nref ? (float)(((double)V.b_perm[q] - (double)d) / V.n2_perm[q]) : 0.0f;
}

// squared residuals of every row from the partials of a whole-plan dot pass
// (absolute slots): rows q = blockIdx.x * 256 + threadIdx.x + k * gridDim.x *
// 256, one FP64 sum per workgroup (fixed grid, so a fixed summation order)
__global__ void __launch_bounds__(256) k_plan_resid_all(PlanView V, double *partials) {
  __shared__ double red[256];
  const float *part = reinterpret_cast<const float *>(V.refs);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double acc = 0.0;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < V.n; q += stride) {
    const int nref = V.ref_cnt[q];
    if (nref) {
      const double rr = (double)row_dot(part + V.ref_base[q], nref) - (double)V.b_perm[q];
      acc += rr * rr;
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// ---- scatter and update of one block, from the lists the dot reads.
//
// One workgroup per (block, tile) list.  Every entry adds r_i a_ij to the
// numerator of its voxel and 1 to s_j, in LDS images of the tile: the
// numerator as a 64-bit fixed-point integer, r_i a_ij x 2^k rounded to the
// nearest integer, with k set from the block size so that no sum of up to
// block_size contributions of magnitude below kFixBig can overflow.  Integer
// additions are exact, so the sums (and the image) do not depend on the order
// in which the entries arrive; LDS integer atomics also run about fifteen
// times as fast as LDS float atomics on this chip.  A contribution of
// magnitude kFixBig or more (or one that is not finite) goes to a float LDS
// image instead, whose sum does depend on the order (no physical row comes
// near it: |r_i a_ij| <= |b_i - a_i.x| / ||a_i||).  Then x_j += lambda num_j /
// s_j for every voxel of the tile that the block touches.
//
// A wavefront takes batches of kScatBatch consecutive chunks (batch j, j +
// kScatWaves, ...) in a three-stage software pipeline: the loads of a batch's
// entries, lengths and per-chunk piece-end records are issued two batches
// ahead of its additions, the loads of the rows of its lanes' piece ends one
// batch ahead, and the loads of r of those rows (a small array, cached) just
// before.
constexpr float kFixBig = 16.0f;
#ifndef PCT_SCAT_WAVES
#define PCT_SCAT_WAVES 16
#endif
#ifndef PCT_SCAT_BATCH
#define PCT_SCAT_BATCH 2
#endif
constexpr int kScatWaves = PCT_SCAT_WAVES;  // wavefronts per scatter workgroup (one workgroup per list)
constexpr int kScatThreads = kScatWaves * kWave;
constexpr int kScatBatch = PCT_SCAT_BATCH;  // chunks per pipeline stage of a wavefront

// fixed-point exponent for blocks of B rows: B x kFixBig x 2^k <= 2^62
__host__ __device__ inline int fix_exponent(int64_t B) {
  int lg = 0;
  while ((int64_t(1) << lg) < B) ++lg;
  return 58 - lg;
}

struct ScatStage {
  uint32_t v[kScatBatch];    // entry codes (0 past the list's end)
  float l[kScatBatch];       // lengths
  uint32_t ord[kScatBatch];  // piece-end ordinal of the lane's piece, from the block's first
};

// loads of a batch (chunks are wave-uniform, so the addresses are a uniform
// base plus a 32-bit lane offset)
template <int LD>
__device__ __forceinline__ void scat_stage_a(const PlanView &V, int64_t ca, int64_t cb, int64_t j, int64_t ob,
                                             int lane, ScatStage &a) {
#pragma unroll
  for (int k = 0; k < kScatBatch; ++k) {
    const int64_t c0 = ca + j * kScatBatch + k;
    const bool in = c0 < cb;
    const int64_t c = in ? c0 : cb - 1;
    const uint16_t *__restrict__ pk = V.packed + c * kWave;
    const uint32_t v = (uint32_t)__builtin_nontemporal_load(pk + lane);
    if constexpr (LD == 0)
      a.l[k] = __builtin_nontemporal_load(reinterpret_cast<const float *>(V.len) + c * kWave + lane);
    else
      a.l[k] = __half2float(__builtin_bit_cast(
                   __half, __builtin_nontemporal_load(reinterpret_cast<const uint16_t *>(V.len) + c * kWave + lane))) *
               V.len_unit;
    a.v[k] = in ? v : 0u;
    const uint64_t m = V.end_mask[c];
    const uint32_t fe = (uint32_t)(V.chunk_first_end[c] - ob);
    // the lane's piece closes at the first closing lane at or above it; lanes
    // past the chunk's last piece end (padding, never added) take that end
    const int below = __popcll(m & ((1ull << lane) - 1ull)), n = __popcll(m);
    a.ord[k] = fe + (uint32_t)(below < n ? below : n - 1);
  }
}

// r a_ij as a 64-bit fixed-point integer: with t = v 2^(k-32) (|t| < 2^30),
// the high word is floor(t) and the low word the fraction t - floor(t)
// (exact in float) times 2^32, truncated
__device__ __forceinline__ unsigned long long fixed_point(float val, float hi_scale) {
  const float t = val * hi_scale;
  const float hi = floorf(t);
  const uint32_t lo = (uint32_t)((t - hi) * 4294967296.0f);
  return ((unsigned long long)(uint32_t)(int)hi << 32) | lo;
}

template <int LD>
__global__ void __launch_bounds__(kScatThreads) k_plan_scatter(PlanView V, int64_t b, float *__restrict__ x,
                                                               const uint8_t *__restrict__ mask, float lambda,
                                                               float hi_scale, float fix_unscale) {
  __shared__ unsigned long long s_num[kTileVox];
  __shared__ uint32_t s_cnt[kTileVox];
  __shared__ float s_big[kTileVox];
  const int lane = wave_lane();
  const int64_t t = blockIdx.x;
  const int64_t lk = b * V.T + t;
  const int64_t ca = V.bt_off[lk] / kWave, cb = V.bt_off[lk + 1] / kWave;
  if (ca == cb) return;  // the whole workgroup leaves
  for (int q = threadIdx.x; q < kTileVox; q += kScatThreads) {
    s_num[q] = 0ull;
    s_cnt[q] = 0u;
    s_big[q] = 0.0f;
  }
  __syncthreads();
  const int64_t ob = V.chunk_first_end[V.bt_off[b * V.T] / kWave];  // the block's first piece-end ordinal
  const uint32_t *__restrict__ ord_row = V.ord_row + ob;
  const float *__restrict__ rvals = V.rvals;
  const int64_t nbat = (cb - ca + kScatBatch - 1) / kScatBatch;
  int64_t j = uniform((int)(threadIdx.x / kWave));
  if (j < nbat) {
    // batches past the last are loaded as the last one again (never added)
    const int64_t jlast = j + (nbat - 1 - j) / kScatWaves * kScatWaves;
    ScatStage a0, a1, a2;
    uint32_t row0[kScatBatch], row1[kScatBatch];
    float r0[kScatBatch];
    scat_stage_a<LD>(V, ca, cb, j, ob, lane, a0);
    scat_stage_a<LD>(V, ca, cb, j + kScatWaves <= jlast ? j + kScatWaves : jlast, ob, lane, a1);
#pragma unroll
    for (int k = 0; k < kScatBatch; ++k) row0[k] = ord_row[a0.ord[k]];
    for (;;) {
      const int64_t j1 = j + kScatWaves, j2 = j + 2 * kScatWaves;
#pragma unroll
      for (int k = 0; k < kScatBatch; ++k) r0[k] = rvals[row0[k]];
#pragma unroll
      for (int k = 0; k < kScatBatch; ++k) row1[k] = ord_row[a1.ord[k]];
      scat_stage_a<LD>(V, ca, cb, j2 <= jlast ? j2 : jlast, ob, lane, a2);
#pragma unroll
      for (int k = 0; k < kScatBatch; ++k) {
        const uint32_t v = a0.v[k];
        if (!(v & 1u)) continue;
        const int loc = (int)((v >> 2) & (kTileVox - 1));
        const float val = r0[k] * a0.l[k];
        if (fabsf(val) < kFixBig)
          atomicAdd(&s_num[loc], fixed_point(val, hi_scale));
        else
          atomicAdd(&s_big[loc], val);
        atomicAdd(&s_cnt[loc], 1u);
      }
      if (j1 > jlast) break;
      j = j1;
      a0 = a1;
      a1 = a2;
#pragma unroll
      for (int k = 0; k < kScatBatch; ++k) row0[k] = row1[k];
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < kTileVox; q += kScatThreads) {
    const uint32_t c = s_cnt[q];
    bool inside;
    const int gv = tile_voxel((int)t, q, V, inside);
    if (!c || !inside) continue;
    const bool keep = !mask || mask[gv] != 0;
    const float num = (float)((double)(long long)s_num[q] * (double)fix_unscale) + s_big[q];
    x[gv] = keep ? x[gv] + lambda * num / (float)c : 0.0f;
  }
}

__global__ void __launch_bounds__(256) k_sum_partials(const double *partials, int64_t np, double *out, int sqrt_it) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t k = threadIdx.x; k < np; k += 256) acc += partials[k];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sqrt_it ? sqrt(red[0]) : red[0];
}

static inline unsigned grid_for(int64_t n, int per_block, unsigned cap) {
  int64_t g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

hipError_t launch_plan_count(const int64_t *row_ptr, const int32_t *idx, const int64_t *order, int64_t n, int64_t B,
                             int64_t M, const PlanView &V, int64_t *bt_cnt, int64_t *row_cap, int64_t *blk_cap,
                             uint32_t *status, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nb = (n + B - 1) / B;
  const int64_t wg = nb * ((B + kCountRows - 1) / kCountRows);
  if (wg > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_plan_count, dim3((unsigned)wg), dim3(256), 0, s, row_ptr, idx, order, n, B, M, V, bt_cnt,
                     row_cap, blk_cap, status);
  return hipGetLastError();
}

hipError_t launch_plan_pad_counts(int64_t *cnt, int64_t k, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_plan_pad, dim3(grid_for(k, 256, 4096)), dim3(256), 0, s, cnt, k);
  return hipGetLastError();
}

hipError_t launch_copy_i64_to_u64(unsigned long long *dst, const int64_t *src, int64_t k, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_i64_u64, dim3(grid_for(k, 256, 4096)), dim3(256), 0, s, dst, src, k);
  return hipGetLastError();
}

hipError_t launch_plan_fill(const int64_t *row_ptr, const int32_t *idx, const void *len_in, int32_t len_in_dtype,
                            const int64_t *order, const float *wepl, const double *norm2, int64_t M,
                            const PlanView &V, uint32_t *status, hipStream_t s) {
  if (V.n <= 0) return hipSuccess;
  const unsigned g = grid_for(V.n, 4, 256 * PCT_FILL_WGS_PER_CU);
  if (len_in_dtype == 0)
    hipLaunchKernelGGL(k_plan_fill<0>, dim3(g), dim3(256), 0, s, row_ptr, idx, len_in, order, wepl, norm2, M, V,
                       status);
  else
    hipLaunchKernelGGL(k_plan_fill<1>, dim3(g), dim3(256), 0, s, row_ptr, idx, len_in, order, wepl, norm2, M, V,
                       status);
  return hipGetLastError();
}

hipError_t launch_plan_ref_ordinals(const PlanView &V, hipStream_t s) {
  if (V.n <= 0) return hipSuccess;
  const dim3 grid(grid_for(V.n, 256, 0x7fffffffu));
  if (V.C > 0 && V.meta) {
    ChunkMeta *meta = reinterpret_cast<ChunkMeta *>(V.meta);
    hipLaunchKernelGGL(k_plan_chunk_meta, dim3(grid_for(V.C, 256, 8192)), dim3(256), 0, s, V, meta);
    hipLaunchKernelGGL(k_plan_ref_ordinals<true>, grid, dim3(256), 0, s, V, meta);
  } else {
    hipLaunchKernelGGL(k_plan_ref_ordinals<false>, grid, dim3(256), 0, s, V, nullptr);
  }
  return hipGetLastError();
}

hipError_t launch_plan_chunks(const PlanView &V, hipStream_t s) {
  if (V.C > 0)
    hipLaunchKernelGGL(k_plan_chunk_ends, dim3(grid_for(V.C, 4 * kEndsChunks, 0x7fffffffu)), dim3(256), 0, s, V);
  return hipGetLastError();
}

hipError_t launch_plan_dot(const PlanView &V, int64_t b, const float *x, hipStream_t s) {
  if (V.T <= 0) return hipSuccess;
  if (V.len_dtype == 0)
    hipLaunchKernelGGL((k_plan_dot<0, false>), dim3((unsigned)(V.T * kDotSplit)), dim3(kDotThreads), 0, s, V, b, x);
  else
    hipLaunchKernelGGL((k_plan_dot<1, false>), dim3((unsigned)(V.T * kDotSplit)), dim3(kDotThreads), 0, s, V, b, x);
  return hipGetLastError();
}

hipError_t launch_plan_dot_all(const PlanView &V, const float *x, hipStream_t s) {
  if (V.T <= 0 || V.nb <= 0) return hipSuccess;
  const int64_t per_blk = V.T * kDotSplit;
  const int64_t blk_per_launch = (kDotAllMaxWgs / per_blk) > 0 ? kDotAllMaxWgs / per_blk : 1;
  for (int64_t b0 = 0; b0 < V.nb; b0 += blk_per_launch) {
    const int64_t nbl = V.nb - b0 < blk_per_launch ? V.nb - b0 : blk_per_launch;
    const dim3 grid((unsigned)(nbl * per_blk));
    if (V.len_dtype == 0)
      hipLaunchKernelGGL((k_plan_dot<0, true>), grid, dim3(kDotThreads), 0, s, V, b0, x);
    else
      hipLaunchKernelGGL((k_plan_dot<1, true>), grid, dim3(kDotThreads), 0, s, V, b0, x);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_plan_rows(const PlanView &V, int64_t b, hipStream_t s) {
  hipLaunchKernelGGL(k_plan_rows, dim3(grid_for(V.B, 256, 0x7fffffffu)), dim3(256), 0, s, V, b);
  return hipGetLastError();
}

hipError_t launch_plan_resid_all(const PlanView &V, double *partials, hipStream_t s) {
  if (V.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_plan_resid_all, dim3((unsigned)kResidAllGrid), dim3(256), 0, s, V, partials);
  return hipGetLastError();
}

hipError_t launch_plan_scatter(const PlanView &V, int64_t b, float *x, const uint8_t *mask, float lambda,
                               hipStream_t s) {
  if (V.T <= 0) return hipSuccess;
  const int k = fix_exponent(V.B);
  const float hi_scale = std::ldexp(1.0f, k - 32), unscale = std::ldexp(1.0f, -k);
  if (V.len_dtype == 0)
    hipLaunchKernelGGL(k_plan_scatter<0>, dim3((unsigned)V.T), dim3(kScatThreads), 0, s, V, b, x, mask, lambda,
                       hi_scale, unscale);
  else
    hipLaunchKernelGGL(k_plan_scatter<1>, dim3((unsigned)V.T), dim3(kScatThreads), 0, s, V, b, x, mask, lambda,
                       hi_scale, unscale);
  return hipGetLastError();
}

hipError_t launch_sum_partials(const double *partials, int64_t np, double *out, int sqrt_it, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, partials, np, out, sqrt_it);
  return hipGetLastError();
}

}  // namespace pct
