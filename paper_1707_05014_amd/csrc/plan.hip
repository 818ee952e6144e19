// Tiled sweep plan: the cached rows of A regrouped, block by block, into
// spatial tiles of 16 x 16 x 8 voxels, so that one DROP block (paper Sec. 2.1)
// runs without global atomics:
//
//   k_plan_dot     one wavefront per 64-entry chunk of a tile's list: gathers
//                  x, multiplies by the lengths and sums each row's piece with a
//                  segmented wave scan -> one partial dot product per piece;
//   k_plan_rows    one thread per row of the block: adds the row's partials in
//                  path order (deterministic) -> r_i = (b_i - a_i.x)/||a_i||^2;
//   k_plan_scatter one workgroup per tile: accumulates r_i a_ij and the row
//                  counts s_j of the block in LDS, then applies
//                  x_j += lambda num_j / s_j to the tile and writes it back.
//
// Entries are packed in 32 bits (row in block, voxel in tile, two flags) next
// to their lengths (float32 or float16), so both passes stream the lists with
// coalesced loads.
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
    for (int64_t w = e0; w < e1; w += kWave) {
      const int64_t e = w + lane;
      const bool valid = e < e1;
      int t = -1, local = 0;
      if (valid) {
        const int j = idx[e];
        if ((uint32_t)j >= (uint64_t)M)
          atomicOr(status, kStBadIndex);
        else
          t = voxel_tile(j, V, local);
      }
      int tp = __shfl_up(t, 1, kWave);
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
// row's pieces end, gather b and ||a||^2 into block order.
template <int LDI>
__global__ void __launch_bounds__(256) k_plan_fill(const int64_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ idx, const void *__restrict__ len_in,
                                                   const int64_t *__restrict__ order, const float *__restrict__ wepl,
                                                   const double *__restrict__ norm2, int64_t M, PlanView V,
                                                   uint32_t *status) {
  const int lane = wave_lane();
  const int64_t q = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave;
  if (q >= V.n) return;
  const int64_t i = order ? order[q] : q;
  if ((uint64_t)i >= (uint64_t)V.n) {
    if (lane == 0) atomicOr(status, kStBadIndex);
    return;
  }
  const int64_t b = q / V.B;
  const uint32_t row_local = (uint32_t)(q - b * V.B);
  if (lane == 0) {
    V.b_perm[q] = wepl[i];
    V.n2_perm[q] = norm2[i];
  }
  const int64_t e0 = row_ptr[i], e1 = row_ptr[i + 1];
  const int64_t rbase = V.ref_base[q], rcap = V.ref_base[q + 1] - rbase;
  int64_t nref = 0;
  for (int64_t w = e0; w < e1; w += kWave) {
    const int64_t e = w + lane;
    const bool valid = e < e1;
    int t = -1, local = 0;
    if (valid) {
      const int j = idx[e];
      if ((uint32_t)j < (uint64_t)M) t = voxel_tile(j, V, local);
    }
    int tp = __shfl_up(t, 1, kWave);
    if (lane == 0) tp = -2;
    const bool start = valid && (lane == 0 || t != tp);
    const uint64_t starts = __ballot(start);
    const int nv = __popcll(__ballot(valid));
    unsigned long long pos = 0;
    int end = 0;
    bool ok = true;
    if (start && t >= 0) {
      end = piece_end_lane(starts, lane, nv);
      const int64_t bt = b * V.T + t;
      pos = atomicAdd(&V.bt_cur[bt], (unsigned long long)(end - lane));
      ok = (int64_t)pos + (end - lane) <= V.bt_off[bt + 1];
    }
    const int s = valid ? piece_start_lane(starts, lane) : 0;
    const unsigned long long ps = __shfl(pos, s, kWave);
    const int pe = __shfl(end, s, kWave);
    const bool pok = __shfl((int)ok, s, kWave) != 0;
    const int ts = __shfl(t, s, kWave);
    const int64_t p = (int64_t)ps + (lane - s);
    const bool write = valid && ts >= 0 && pok;
    if (valid && !pok && lane == s) atomicOr(status, kStOverflow);
    const bool last = lane == pe - 1;
    bool is_ref = false;
    if (write) {
      V.packed[p] = pack_entry(last ? 1u : 0u, (uint32_t)local, row_local);
      if (V.len_dtype == 0) {
        const float l = LDI == 0 ? reinterpret_cast<const float *>(len_in)[e]
                                 : __half2float(reinterpret_cast<const __half *>(len_in)[e]) * V.len_unit;
        reinterpret_cast<float *>(V.len)[p] = l;
      } else {
        reinterpret_cast<__half *>(V.len)[p] =
            LDI == 1 ? reinterpret_cast<const __half *>(len_in)[e]
                     : __float2half(reinterpret_cast<const float *>(len_in)[e] / V.len_unit);
      }
      is_ref = last || ((p & (kWave - 1)) == kWave - 1);
    }
    const uint64_t rm = __ballot(is_ref);
    if (is_ref) {
      const int64_t k = nref + __popcll(rm & ((1ull << lane) - 1));
      if (k < rcap)
        V.refs[rbase + k] = (uint32_t)p;
      else
        atomicOr(status, kStOverflow);
    }
    nref += __popcll(rm);
  }
  if (lane == 0) V.ref_cnt[q] = (int32_t)(nref < rcap ? nref : rcap);
}

// chunk -> linear index of its tile's first voxel (one workgroup per (block, tile) list)
__global__ void __launch_bounds__(256) k_plan_chunk_tile(PlanView V) {
  const int64_t k = blockIdx.x;
  if (k >= V.nb * V.T) return;
  const int64_t c0 = V.bt_off[k] / kWave, c1 = V.bt_off[k + 1] / kWave;
  bool inside;
  const int base = tile_voxel((int)(k % V.T), 0, V, inside);
  for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) V.chunk_tile[c] = base;
}

// lanes that close a piece (or a chunk) and their count per chunk
__global__ void __launch_bounds__(256) k_plan_chunk_ends(PlanView V) {
  const int lane = wave_lane();
  const int64_t c = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave;
  if (c >= V.C) return;
  const uint32_t v = V.packed[c * kWave + lane];
  const bool valid = v & 1u;
  const bool close = valid && (((v >> 1) & 1u) || lane == kWave - 1);
  const uint64_t m = __ballot(close);
  if (lane == 0) {
    V.end_mask[c] = m;
    V.chunk_first_end[c + 1] = __popcll(m);
  }
}

// Inclusive prefix sum over the 64 lanes with DPP row shifts and row
// broadcasts (GFX9 cross-lane data movement; no LDS traffic).
__device__ __forceinline__ float wave_incl_scan_dpp(float x) {
  constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
  constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143;
  x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), kRowShr1, 0xf, 0xf, false));
  x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), kRowShr2, 0xf, 0xf, false));
  x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), kRowShr4, 0xf, 0xf, false));
  x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), kRowShr8, 0xf, 0xf, false));
  x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), kRowBcast15, 0xa, 0xf, false));
  x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), kRowBcast31, 0xc, 0xf, false));
  return x;
}

template <int LD>
__device__ __forceinline__ float plan_len(const PlanView &V, int64_t p) {
  if constexpr (LD == 0)
    return __builtin_nontemporal_load(reinterpret_cast<const float *>(V.len) + p);
  else
    return __half2float(reinterpret_cast<const __half *>(V.len)[p]) * V.len_unit;
}

// partial dot products of every piece of block b; a wavefront takes
// kChunksPerWave consecutive chunks
constexpr int kChunksPerWave = 8;

template <int LD>
__global__ void __launch_bounds__(256) k_plan_dot(PlanView V, int64_t b, const float *__restrict__ x) {
  const int lane = wave_lane();
  const int64_t c0 = V.bt_off[b * V.T] / kWave, c1 = V.bt_off[(b + 1) * V.T] / kWave;
  const int64_t cw = c0 + ((int64_t)blockIdx.x * 4 + threadIdx.x / kWave) * kChunksPerWave;
  if (cw >= c1) return;
  const int nc = (int)(cw + kChunksPerWave < c1 ? kChunksPerWave : c1 - cw);
  const int nxy = V.nx * V.ny;
  // issue every load of the wavefront's chunks before using any of them
  uint32_t v[kChunksPerWave];
  float l[kChunksPerWave];
  int cb[kChunksPerWave];
#pragma unroll
  for (int k = 0; k < kChunksPerWave; ++k) {
    v[k] = 0u;
    l[k] = 0.f;
    cb[k] = 0;
    if (k < nc) {
      const int64_t p = (cw + k) * kWave + lane;
      v[k] = __builtin_nontemporal_load(V.packed + p);
      l[k] = plan_len<LD>(V, p);
      cb[k] = V.chunk_tile[cw + k];
    }
  }
  float xv[kChunksPerWave];
#pragma unroll
  for (int k = 0; k < kChunksPerWave; ++k) {
    xv[k] = 0.f;
    if (v[k] & 1u) {
      const int local = (v[k] >> 2) & (kTileVox - 1);
      const int gv = cb[k] + (local >> 8) * nxy + ((local >> 4) & 15) * V.nx + (local & 15);
      xv[k] = x[gv];
    }
  }
#pragma unroll
  for (int k = 0; k < kChunksPerWave; ++k) {
    if (k >= nc) break;
    const bool valid = v[k] & 1u;
    const bool close = valid && (((v[k] >> 1) & 1u) || lane == kWave - 1);
    const uint64_t m = __ballot(close);
    // a piece's sum is the difference of the prefix sums at its closing lane
    // and at the previous closing lane
    const float S = wave_incl_scan_dpp(valid ? l[k] * xv[k] : 0.0f);
    const uint64_t below = m & ((1ull << lane) - 1);
    const int prev = below ? 63 - __clzll(below) : lane;
    const float Sp = __shfl(S, prev, kWave);
    if (close) {
      // end_slot is indexed by the global ordinal of the piece end
      const int64_t ord = V.chunk_first_end[cw + k] + __popcll(below);
      V.partial[V.end_slot[ord]] = below ? S - Sp : S;
    }
  }
}

// references hold entry positions after the fill pass; record, for every
// piece end (block-relative ordinal in chunk order), the row-ordered slot of
// its reference, so k_plan_dot can store each partial next to the other
// partials of its row
__global__ void __launch_bounds__(256) k_plan_ref_ordinals(PlanView V) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= V.n) return;
  const int64_t b = q / V.B;
  const int64_t rb = V.ref_base[b * V.B];
  const int64_t k0 = V.ref_base[q];
  const int nref = V.ref_cnt[q];
  for (int k = 0; k < nref; ++k) {
    const uint32_t p = V.refs[k0 + k];
    const int64_t c = p / kWave;
    const int l = p & (kWave - 1);
    const int64_t ord = V.chunk_first_end[c] + __popcll(V.end_mask[c] & ((1ull << l) - 1));
    V.end_slot[ord] = (uint32_t)(k0 + k - rb);
  }
}

// sum of a row's piece partials; four references per step so that their
// loads overlap (fixed summation order, so results are reproducible)
__device__ __forceinline__ float row_dot(const PlanView &V, int64_t q, int64_t rb, int &nref) {
  const float *p = V.partial + (V.ref_base[q] - rb);
  nref = V.ref_cnt[q];
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
  int nref;
  const float d = row_dot(V, q, V.ref_base[b * V.B], nref);
  V.rvals[r] = nref ? (float)(((double)V.b_perm[q] - (double)d) / V.n2_perm[q]) : 0.0f;
}

// squared residuals of block b's rows: per-workgroup FP64 sums
__global__ void __launch_bounds__(256) k_plan_resid_rows(PlanView V, int64_t b, double *partials) {
  __shared__ double red[256];
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t q = b * V.B + r;
  double acc = 0.0;
  if (r < V.B && q < V.n) {
    int nref;
    const float d = row_dot(V, q, V.ref_base[b * V.B], nref);
    if (nref) {
      const double rr = (double)d - (double)V.b_perm[q];
      acc = rr * rr;
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

// Voxel-major copy of one (block, tile) list: counting sort by tile-local
// voxel in LDS (one workgroup per list).  Group offsets go to grp_off; the
// last entry of each voxel's run is flagged.
__global__ void __launch_bounds__(256) k_plan_voxel_major(PlanView V) {
  __shared__ uint32_t s_cnt[kTileVox];
  __shared__ uint32_t s_pos[kTileVox];
  __shared__ uint32_t s_start[kTileVox];
  __shared__ uint32_t s_part[256];
  const int64_t k = blockIdx.x;  // (block, tile)
  if (k >= V.nb * V.T) return;
  const int64_t a0 = V.bt_off[k], a1 = V.bt_off[k + 1];
  for (int e = threadIdx.x; e < kTileVox; e += blockDim.x) s_cnt[e] = 0u;
  __syncthreads();
  for (int64_t p = a0 + threadIdx.x; p < a1; p += blockDim.x) {
    const uint32_t v = V.packed[p];
    if (v & 1u) atomicAdd(&s_cnt[(v >> 2) & (kTileVox - 1)], 1u);
  }
  __syncthreads();
  // exclusive scan of the 2048 counts: 8 per thread, then across threads
  const int per = kTileVox / 256;
  uint32_t loc[per];
  uint32_t tot = 0;
#pragma unroll
  for (int q = 0; q < per; ++q) {
    loc[q] = tot;
    tot += s_cnt[threadIdx.x * per + q];
  }
  s_part[threadIdx.x] = tot;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const uint32_t add = (int)threadIdx.x >= o ? s_part[threadIdx.x - o] : 0u;
    __syncthreads();
    s_part[threadIdx.x] += add;
    __syncthreads();
  }
  const uint32_t excl = s_part[threadIdx.x] - tot;
  // list start in the voxel-major arrays: entries before this list are the
  // valid entries of all earlier lists, i.e. grp_off[k * kGroups] (filled by
  // the host from the per-list valid counts)
  const int64_t base = V.grp_off[k * kGroups];
#pragma unroll
  for (int q = 0; q < per; ++q) {
    const int vox = threadIdx.x * per + q;
    s_pos[vox] = excl + loc[q];
    s_start[vox] = excl + loc[q];
    if ((vox & 63) == 0 && vox > 0) V.grp_off[k * kGroups + vox / 64] = base + excl + loc[q];
  }
  __syncthreads();
  for (int64_t p = a0 + threadIdx.x; p < a1; p += blockDim.x) {
    const uint32_t v = V.packed[p];
    if (!(v & 1u)) continue;
    const int vox = (v >> 2) & (kTileVox - 1);
    const uint32_t slot = atomicAdd(&s_pos[vox], 1u);
    const uint32_t last = slot == s_start[vox] + s_cnt[vox] - 1u ? 2u : 0u;  // closes the voxel's run
    const int64_t dst = base + slot;
    if (dst >= V.grp_off[(k + 1) * kGroups]) continue;  // cannot happen when the counts agree
    V.packedB[dst] = 1u | last | ((uint32_t)(vox & 63) << 2) | (v & ~((1u << 13) - 1u));
    if (V.len_dtype == 0)
      reinterpret_cast<float *>(V.lenB)[dst] = reinterpret_cast<const float *>(V.len)[p];
    else
      reinterpret_cast<__half *>(V.lenB)[dst] = reinterpret_cast<const __half *>(V.len)[p];
  }
}

// Scatter of block b, voxel-major: one wavefront per 64-voxel group of a tile.
// Each voxel's run is reduced with DPP prefix sums (its length is s_j); the
// lane closing the run applies x_j += lambda num_j / s_j.  No atomics.
template <int LD>
__global__ void __launch_bounds__(256) k_plan_scatter(PlanView V, int64_t b, float *__restrict__ x,
                                                      const uint8_t *__restrict__ mask, float lambda) {
  const int lane = wave_lane();
  const int64_t g = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave;  // group within the block
  if (g >= V.T * kGroups) return;
  const int64_t t = g / kGroups;
  const int grp = (int)(g % kGroups);
  const int64_t gi = (b * V.T + t) * kGroups + grp;
  const int64_t e0 = V.grp_off[gi], e1 = V.grp_off[gi + 1];
  if (e0 == e1) return;
  bool inside;
  const int tile_base = tile_voxel((int)t, 0, V, inside);
  const int nxy = V.nx * V.ny;
  float carry = 0.0f;  // sum of the run that continues from the previous chunk
  int carry_n = 0;
  constexpr int U = 4;  // chunks whose loads are issued together
  for (int64_t wb = e0; wb < e1; wb += (int64_t)U * kWave) {
    uint32_t v[U];
    float val[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int64_t p = wb + (int64_t)k * kWave + lane;
      v[k] = 0u;
      val[k] = 0.0f;
      if (p < e1) {
        v[k] = __builtin_nontemporal_load(V.packedB + p);
        val[k] = LD == 0 ? __builtin_nontemporal_load(reinterpret_cast<const float *>(V.lenB) + p)
                         : __half2float(reinterpret_cast<const __half *>(V.lenB)[p]) * V.len_unit;
      }
    }
#pragma unroll
    for (int k = 0; k < U; ++k)
      if (v[k] & 1u) val[k] *= V.rvals[v[k] >> 13];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int64_t w = wb + (int64_t)k * kWave;
      if (w >= e1) break;
      const bool close = (v[k] & 1u) && ((v[k] >> 1) & 1u);
      const uint64_t m = __ballot(close);
      const float S = wave_incl_scan_dpp(val[k]);
      const uint64_t below = m & ((1ull << lane) - 1);
      const int prev = below ? 63 - __clzll(below) : -1;
      const float Sp = __shfl(S, prev < 0 ? 0 : prev, kWave);
      if (close) {
        const float num = prev >= 0 ? S - Sp : S + carry;
        const int cnt = prev >= 0 ? lane - prev : lane + 1 + carry_n;
        const int local = grp * 64 + ((v[k] >> 2) & 63);
        const int gv = tile_base + (local >> 8) * nxy + ((local >> 4) & 15) * V.nx + (local & 15);
        const float xn = x[gv] + lambda * num / (float)cnt;
        x[gv] = (mask && !mask[gv]) ? 0.0f : xn;
      }
      // the run still open at the end of this chunk carries into the next one
      const int nv = (int)(e1 - w < kWave ? e1 - w : kWave);
      const int last_close = m ? 63 - __clzll(m) : -1;
      const float S_end = __shfl(S, nv - 1, kWave);
      const float S_lc = __shfl(S, last_close < 0 ? 0 : last_close, kWave);
      if (last_close == nv - 1) {
        carry = 0.0f;
        carry_n = 0;
      } else if (last_close < 0) {
        carry += S_end;
        carry_n += nv;
      } else {
        carry = S_end - S_lc;
        carry_n = nv - 1 - last_close;
      }
    }
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
  const unsigned g = grid_for(V.n, 4, 0x7fffffffu);
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
  hipLaunchKernelGGL(k_plan_ref_ordinals, dim3(grid_for(V.n, 256, 0x7fffffffu)), dim3(256), 0, s, V);
  return hipGetLastError();
}

hipError_t launch_plan_chunks(const PlanView &V, hipStream_t s) {
  if (V.nb * V.T > 0)
    hipLaunchKernelGGL(k_plan_chunk_tile, dim3((unsigned)(V.nb * V.T)), dim3(256), 0, s, V);
  if (V.C > 0) hipLaunchKernelGGL(k_plan_chunk_ends, dim3(grid_for(V.C, 4, 0x7fffffffu)), dim3(256), 0, s, V);
  return hipGetLastError();
}

hipError_t launch_plan_dot(const PlanView &V, int64_t b, const float *x, hipStream_t s) {
  // chunks of the block are not known on the host: launch for the largest block
  // (wavefronts past the block's last chunk exit at once)
  const unsigned g = grid_for((V.maxc + kChunksPerWave - 1) / kChunksPerWave, 4, 0x7fffffffu);
  if (V.len_dtype == 0)
    hipLaunchKernelGGL(k_plan_dot<0>, dim3(g), dim3(256), 0, s, V, b, x);
  else
    hipLaunchKernelGGL(k_plan_dot<1>, dim3(g), dim3(256), 0, s, V, b, x);
  return hipGetLastError();
}

hipError_t launch_plan_rows(const PlanView &V, int64_t b, hipStream_t s) {
  hipLaunchKernelGGL(k_plan_rows, dim3(grid_for(V.B, 256, 0x7fffffffu)), dim3(256), 0, s, V, b);
  return hipGetLastError();
}

hipError_t launch_plan_resid_rows(const PlanView &V, int64_t b, double *partials, hipStream_t s) {
  hipLaunchKernelGGL(k_plan_resid_rows, dim3(grid_for(V.B, 256, 0x7fffffffu)), dim3(256), 0, s, V, b, partials);
  return hipGetLastError();
}

hipError_t launch_plan_scatter(const PlanView &V, int64_t b, float *x, const uint8_t *mask, float lambda,
                               hipStream_t s) {
  const unsigned g = grid_for(V.T * kGroups, 4, 0x7fffffffu);
  if (V.len_dtype == 0)
    hipLaunchKernelGGL(k_plan_scatter<0>, dim3(g), dim3(256), 0, s, V, b, x, mask, lambda);
  else
    hipLaunchKernelGGL(k_plan_scatter<1>, dim3(g), dim3(256), 0, s, V, b, x, mask, lambda);
  return hipGetLastError();
}

hipError_t launch_plan_build_voxel_major(const PlanView &V, hipStream_t s) {
  if (V.nb * V.T <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_plan_voxel_major, dim3((unsigned)(V.nb * V.T)), dim3(256), 0, s, V);
  return hipGetLastError();
}

hipError_t launch_sum_partials(const double *partials, int64_t np, double *out, int sqrt_it, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, partials, np, out, sqrt_it);
  return hipGetLastError();
}

}  // namespace pct
