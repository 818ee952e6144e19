// Block-iterative row projections (paper Sec. 2.1, DROP; ART as the block
// size one case), the residual ||Ax - b|| and the ROI reduction.
//
// For one block B with x fixed at its block-start value:
//   r_i = (b_i - a_i . x) / ||a_i||^2,  num_j = sum_i r_i a_ij,
//   s_j = #{i in B : a_ij > 0},         x_j += lambda num_j / s_j.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "path_device.h"

namespace pct {

template <int LD>
__device__ __forceinline__ float load_len(const void *len, int64_t e, float unit) {
  if constexpr (LD == 0) {
    return __builtin_nontemporal_load(reinterpret_cast<const float *>(len) + e);
  } else {
    return __half2float(reinterpret_cast<const __half *>(len)[e]) * unit;
  }
}

// one wavefront per cached row of the block
template <int LD>
__global__ void __launch_bounds__(256) k_project_cached(const int64_t *__restrict__ row_ptr,
                                                        const int32_t *__restrict__ idx, const void *__restrict__ len,
                                                        float unit, const double *__restrict__ norm2,
                                                        const float *__restrict__ b, const int64_t *__restrict__ order,
                                                        int64_t first, int64_t count, int64_t n, int64_t M,
                                                        const float *__restrict__ x, float *num, uint32_t *cnt,
                                                        uint32_t *status) {
  const int lane = wave_lane();
  const int64_t q = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (q >= count) return;
  const int64_t i = order ? order[first + q] : first + q;
  if ((uint64_t)i >= (uint64_t)n) {
    if (lane == 0) atomicOr(status, kStBadIndex);
    return;
  }
  const int64_t e0 = row_ptr[i], e1 = row_ptr[i + 1];
  if (e1 == e0) return;
  float d = 0.0f;
  bool bad = false;
  for (int64_t e = e0 + lane; e < e1; e += kWave) {
    const int j = idx[e];
    if ((uint32_t)j >= (uint64_t)M) { bad = true; continue; }
    d = fmaf(load_len<LD>(len, e, unit), x[j], d);
  }
  if (__ballot(bad)) {
    if (lane == 0) atomicOr(status, kStBadIndex);
    return;
  }
  d = wave_sum_f32(d);
  const float r = (float)(((double)b[i] - (double)d) / norm2[i]);
  for (int64_t e = e0 + lane; e < e1; e += kWave) {
    const int j = idx[e];
    atomicAdd(&num[j], r * load_len<LD>(len, e, unit));
    atomicAdd(&cnt[j], 1u);
  }
}

// one wavefront per proton of the block: the row is rebuilt in LDS.  MODE 0:
// the block's voxel counts s_j are not formed (an earlier sweep stored them),
// one FP32 atomic per entry; 1: an FP32 numerator atomic and an integer count
// atomic per entry; 2: one 64-bit integer atomic per entry that adds both, the
// contribution as a fixed-point integer (r a_ij 2^pk_k rounded to nearest)
// above a count field of pk_bits bits: pk += (fixed << pk_bits) + 1.  The
// host sets pk_bits so that no block count can reach the numerator field and
// pk_k so that no sum of contributions below kPackBig can overflow it; a
// contribution of kPackBig or more takes the two separate atomics of mode 1.
// One 64-bit add runs at 4.8e10/s along path-like runs in brick order, two
// separate adds at 3.4e10 entries/s.
// Records: with `global` they are indexed by history (recs[order[first + q]],
// an order entry outside [0, n) sets kStBadIndex), else by position in the
// chunk (recs[q]).
constexpr float kPackBig = 4.0f;

template <typename R, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) k_project_fused(PathParams P, const PathRec<R> *__restrict__ recs,
                                                       const int64_t *__restrict__ order, int64_t first, int64_t n,
                                                       int global, int64_t count, const float *__restrict__ x,
                                                       float *num, uint32_t *cnt, unsigned long long *pk,
                                                       int pk_bits, float pk_scale, uint32_t *status) {
  extern __shared__ int smem[];
  const int wid = threadIdx.x / kWave;
  const int lane = wave_lane();
  const RowBuf rb = row_buf(smem, wid, P.emax);
  int *s_vox = rb.vox;
  float *s_len = rb.len;
  int16_t *s_aux = rb.aux;
  __shared__ R s_cF[24];
  stage_prior<R>(P, s_cF);
  const int64_t stride = (int64_t)gridDim.x * P.waves_per_block;
  for (int64_t q = (int64_t)blockIdx.x * P.waves_per_block + wid; q < count; q += stride) {
    int64_t ri = q;
    if (global) {
      ri = order ? order[first + q] : first + q;
      if ((uint64_t)ri >= (uint64_t)n) {
        if (lane == 0) atomicOr(status, kStBadIndex);
        continue;
      }
    }
    ProtonPath<R> pp;
    float b;
    load_record<R>(recs + ri, pp, b);
    const int ne = build_row<R>(P, s_cF, pp, s_vox, s_len, s_aux, status);
    if (ne == 0) continue;
    float d = 0.0f;
    double n2 = 0.0;
    for (int e = lane; e < ne; e += kWave) {
      const float l = s_len[e];
      d = fmaf(l, x[s_vox[e]], d);
      n2 += (double)l * (double)l;
    }
    d = wave_sum_f32(d);
    n2 = wave_sum_f64(n2);
    const float r = (float)(((double)b - (double)d) / n2);
    for (int e = lane; e < ne; e += kWave) {
      const int j = s_vox[e];
      const float v = r * s_len[e];
      if constexpr (MODE == 2) {
        if (fabsf(v) < kPackBig) {
          const long long f = (long long)(int)rintf(v * pk_scale);  // |f| < 2^31
          atomicAdd(&pk[j], ((unsigned long long)f << pk_bits) + 1ull);
        } else {
          atomicAdd(&num[j], v);
          atomicAdd(&cnt[j], 1u);
        }
      } else {
        atomicAdd(&num[j], v);
        if constexpr (MODE == 1) atomicAdd(&cnt[j], 1u);
      }
    }
  }
}

// Block update x_j += lambda num_j / s_j for s_j > 0 (hull mask: x_j = 0
// outside), num_j cleared.  MODE 0: s_j from cnt (cleared); 1: also stored
// as uint16 into blk_cnt; 2: s_j read from blk_cnt (cnt untouched).
// BRICK: the accumulators and blk_cnt are in brick order (position q of Mb),
// x and the mask linear, and xb (x in brick order) is updated with x.
// touched (or NULL): set to 1 for every voxel the block's rows touch (CARP's
// component averaging counts the strings that touch a voxel).  pk (or NULL,
// modes 0 and 1): packed fixed-point numerators and counts of the projection's
// mode 2, added to num and cnt (count field of pk_bits bits, numerator
// 2^-pk_k units, pk_unscale = 2^-pk_k) and cleared.
template <int MODE, bool BRICK>
__global__ void __launch_bounds__(256) k_apply(float *__restrict__ x, float *__restrict__ num,
                                               uint32_t *__restrict__ cnt, uint16_t *__restrict__ blk_cnt,
                                               const uint8_t *__restrict__ mask, int64_t M, float lambda,
                                               uint32_t *status, uint8_t *__restrict__ touched, int32_t nx,
                                               int32_t ny, int32_t nz, int32_t nbx, int32_t nby,
                                               float *__restrict__ xb, int64_t Mq, unsigned long long *__restrict__ pk,
                                               int pk_bits, double pk_unscale) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool sat = false;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < Mq; q += stride) {
    int64_t j = q;
    if constexpr (BRICK) {
      const int64_t br = q >> 6;
      const int w = (int)(q & 63);
      const int ix = (int)(br % nbx) * 4 + (w & 3);
      const int iy = (int)((br / nbx) % nby) * 4 + ((w >> 2) & 3);
      const int iz = (int)(br / ((int64_t)nbx * nby)) * 4 + (w >> 4);
      if (ix >= nx || iy >= ny || iz >= nz) continue;
      j = ((int64_t)iz * ny + iy) * nx + ix;
    }
    uint32_t c;
    float nq = num[q];
    unsigned long long pq = 0ull;
    if constexpr (MODE == 2) {
      c = blk_cnt[q];
    } else {
      c = cnt[q];
      if (pk) {
        pq = pk[q];
        // the count field, and the numerator above it (an arithmetic shift:
        // the field holds 0 <= count < 2^pk_bits, so it rounds nothing away)
        c += (uint32_t)(pq & ((1ull << pk_bits) - 1ull));
        nq += (float)((double)((long long)pq >> pk_bits) * pk_unscale);
      }
      if constexpr (MODE == 1) {
        sat |= c > 0xffffu;
        blk_cnt[q] = (uint16_t)(c > 0xffffu ? 0xffffu : c);
      }
    }
    if (c) {
      if (touched) touched[j] = 1;
      const float v = (mask && !mask[j]) ? 0.0f : x[j] + lambda * nq / (float)c;
      x[j] = v;
      if constexpr (BRICK) xb[q] = v;
      num[q] = 0.0f;
      if constexpr (MODE != 2) cnt[q] = 0u;
      if (pq) pk[q] = 0ull;
    }
  }
  if (MODE == 1 && __ballot(sat) && wave_lane() == 0) atomicOr(status, kStCountSat);
}

__global__ void __launch_bounds__(256) k_to_bricks(const float *__restrict__ x, float *__restrict__ xb, int32_t nx,
                                                   int32_t ny, int32_t nz, int32_t nbx, int32_t nby, int64_t Mb) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < Mb; q += stride) {
    const int64_t br = q >> 6;
    const int w = (int)(q & 63);
    const int ix = (int)(br % nbx) * 4 + (w & 3);
    const int iy = (int)((br / nbx) % nby) * 4 + ((w >> 2) & 3);
    const int iz = (int)(br / ((int64_t)nbx * nby)) * 4 + (w >> 4);
    xb[q] = (ix < nx && iy < ny && iz < nz) ? x[((int64_t)iz * ny + iy) * nx + ix] : 0.0f;
  }
}

// CARP (Sec. 2.2): string image xs into the component sums over the strings
// that touch each voxel (touched cleared for the next string), then the mean
__global__ void __launch_bounds__(256) k_carp_accumulate(const float *__restrict__ xs, uint8_t *__restrict__ touched,
                                                         float *__restrict__ acc, uint16_t *__restrict__ tc,
                                                         int64_t M) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < M; j += stride) {
    if (touched[j]) {
      acc[j] += xs[j];
      tc[j] = (uint16_t)(tc[j] + 1);
      touched[j] = 0;
    }
  }
}

__global__ void __launch_bounds__(256) k_carp_average(float *__restrict__ x, float *__restrict__ acc,
                                                      uint16_t *__restrict__ tc, int64_t M) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < M; j += stride) {
    const uint16_t c = tc[j];
    if (c) x[j] = acc[j] / (float)c;
    acc[j] = 0.0f;
    tc[j] = 0;
  }
}

__global__ void __launch_bounds__(256) k_copy_f32(const float *__restrict__ a, float *__restrict__ b, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) b[j] = a[j];
}

__global__ void __launch_bounds__(256) k_mask(float *__restrict__ x, const uint8_t *__restrict__ mask, int64_t M) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < M; j += stride)
    if (!mask[j]) x[j] = 0.0f;
}

// ART: rows strictly in sequence, one wavefront.  x is read with agent-scope
// loads (past the per-CU cache) and each row's update is made visible before
// the next row reads.
template <int LD>
__global__ void __launch_bounds__(64) k_art(const int64_t *__restrict__ row_ptr, const int32_t *__restrict__ idx,
                                            const void *__restrict__ len, float unit,
                                            const double *__restrict__ norm2, const float *__restrict__ b,
                                            const int64_t *__restrict__ order, int64_t n, int64_t M, float *x,
                                            const uint8_t *__restrict__ mask, float lambda, uint32_t *status) {
  const int lane = wave_lane();
  for (int64_t q = 0; q < n; ++q) {
    const int64_t i = order ? order[q] : q;
    if ((uint64_t)i >= (uint64_t)n) {
      if (lane == 0) atomicOr(status, kStBadIndex);
      continue;
    }
    const int64_t e0 = row_ptr[i], e1 = row_ptr[i + 1];
    if (e1 == e0) continue;
    float d = 0.0f;
    bool bad = false;
    for (int64_t e = e0 + lane; e < e1; e += kWave) {
      const int j = idx[e];
      if ((uint32_t)j >= (uint64_t)M) { bad = true; continue; }
      d = fmaf(load_len<LD>(len, e, unit), __hip_atomic_load(&x[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), d);
    }
    if (__ballot(bad)) {
      if (lane == 0) atomicOr(status, kStBadIndex);
      continue;
    }
    d = wave_sum_f32(d);
    const float r = (float)(((double)b[i] - (double)d) / norm2[i]);
    const float lr = lambda * r;
    for (int64_t e = e0 + lane; e < e1; e += kWave) {
      const int j = idx[e];
      if (!mask || mask[j]) atomicAdd(&x[j], lr * load_len<LD>(len, e, unit));
    }
    __threadfence();
  }
}

// residual: per-workgroup FP64 partial sums, then one ordered final sum
template <int LD>
__global__ void __launch_bounds__(256) k_resid_cached(const int64_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ idx, const void *__restrict__ len,
                                                      float unit, const float *__restrict__ b, int64_t n, int64_t M,
                                                      const float *__restrict__ x, double *partials) {
  __shared__ double red[4];
  const int lane = wave_lane();
  const int wid = threadIdx.x / kWave;
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * 4;
  for (int64_t i = (int64_t)blockIdx.x * 4 + wid; i < n; i += stride) {
    const int64_t e0 = row_ptr[i], e1 = row_ptr[i + 1];
    if (e1 == e0) continue;
    float d = 0.0f;
    for (int64_t e = e0 + lane; e < e1; e += kWave) {
      const int j = idx[e];
      if ((uint32_t)j < (uint64_t)M) d = fmaf(load_len<LD>(len, e, unit), x[j], d);
    }
    d = wave_sum_f32(d);
    const double rr = (double)d - (double)b[i];
    acc += rr * rr;
  }
  if (lane == 0) red[wid] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// rows of one chunk (set-up records recs[0, n)); workgroup g's sum is stored
// to partials[g] (accumulate = 0) or added to it (later chunks)
template <typename R>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) k_resid_fused(PathParams P, const PathRec<R> *__restrict__ recs, int64_t n,
                                                     const float *__restrict__ x, double *partials,
                                                     uint32_t *status, int accumulate) {
  extern __shared__ int smem[];
  __shared__ double red[4];
  const int wid = threadIdx.x / kWave;
  const int lane = wave_lane();
  const RowBuf rb = row_buf(smem, wid, P.emax);
  int *s_vox = rb.vox;
  float *s_len = rb.len;
  int16_t *s_aux = rb.aux;
  __shared__ R s_cF[24];
  stage_prior<R>(P, s_cF);
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * P.waves_per_block;
  for (int64_t i = (int64_t)blockIdx.x * P.waves_per_block + wid; i < n; i += stride) {
    ProtonPath<R> pp;
    float b;
    load_record<R>(recs + i, pp, b);
    const int ne = build_row<R>(P, s_cF, pp, s_vox, s_len, s_aux, status);
    if (ne == 0) continue;
    float d = 0.0f;
    for (int e = lane; e < ne; e += kWave) d = fmaf(s_len[e], x[s_vox[e]], d);
    d = wave_sum_f32(d);
    const double rr = (double)d - (double)b;
    acc += rr * rr;
  }
  if (lane == 0) red[wid] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < P.waves_per_block; ++w) s += red[w];
    partials[blockIdx.x] = accumulate ? partials[blockIdx.x] + s : s;
  }
}

__global__ void __launch_bounds__(256) k_resid_final(const double *partials, int64_t np, double *out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t k = threadIdx.x; k < np; k += 256) acc += partials[k];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sqrt(red[0]);
}

__global__ void __launch_bounds__(256) k_roi(const float *__restrict__ x, const uint8_t *__restrict__ labels,
                                             int64_t M, int32_t n_labels, double *sums,
                                             unsigned long long *counts) {
  __shared__ double s_sum[256];
  __shared__ unsigned int s_cnt[256];
  for (int l = threadIdx.x; l < 256; l += blockDim.x) { s_sum[l] = 0.0; s_cnt[l] = 0u; }
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < M; j += stride) {
    const int l = labels[j];
    if (l > 0 && l <= n_labels) {
      atomicAdd(&s_sum[l], (double)x[j]);
      atomicAdd(&s_cnt[l], 1u);
    }
  }
  __syncthreads();
  for (int l = 1 + threadIdx.x; l <= n_labels; l += blockDim.x) {
    if (s_cnt[l]) {
      atomicAdd(&sums[l - 1], s_sum[l]);
      atomicAdd(&counts[l - 1], (unsigned long long)s_cnt[l]);
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_zero_small(T *p, int64_t n) {
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) p[i] = T(0);
}

__global__ void k_poison(double *out, const uint32_t *status) {
  if (status[0] != 0u) *out = __builtin_nan("");
}

static inline unsigned grid_for(int64_t n, int per_block, unsigned cap) {
  int64_t g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

hipError_t launch_mask(float *x, const uint8_t *mask, int64_t M, hipStream_t s) {
  if (!mask || M <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mask, dim3(grid_for(M, 256, 8192)), dim3(256), 0, s, x, mask, M);
  return hipGetLastError();
}

hipError_t launch_project_cached(const int64_t *row_ptr, const int32_t *idx, const void *len, int32_t len_dtype,
                                 float len_unit, const double *norm2, const float *b, const int64_t *order,
                                 int64_t first, int64_t count, int64_t n, int64_t M, const float *x, float *num,
                                 uint32_t *cnt, uint32_t *status, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const unsigned grid = grid_for(count, 4, 0x7fffffffu);
  if (len_dtype == 0)
    hipLaunchKernelGGL(k_project_cached<0>, dim3(grid), dim3(256), 0, s, row_ptr, idx, len, len_unit, norm2, b,
                       order, first, count, n, M, x, num, cnt, status);
  else
    hipLaunchKernelGGL(k_project_cached<1>, dim3(grid), dim3(256), 0, s, row_ptr, idx, len, len_unit, norm2, b,
                       order, first, count, n, M, x, num, cnt, status);
  return hipGetLastError();
}

hipError_t launch_project_fused(const PathParams &P, const void *recs, const int64_t *order, int64_t first, int64_t n,
                                bool global, int64_t count, const float *x, float *num, uint32_t *cnt,
                                uint32_t *status, hipStream_t s, unsigned long long *pk, int pk_bits, int pk_k) {
  const int gl = global ? 1 : 0;
  if (count <= 0) return hipSuccess;
  const size_t lds = (size_t)P.waves_per_block * row_buf_bytes(P.emax);
  const unsigned grid = grid_for(count, P.waves_per_block, 1u << 20);
  const dim3 g(grid), b(P.waves_per_block * kWave);
  const int mode = cnt ? (pk ? 2 : 1) : 0;
  const float pk_scale = pk ? std::ldexp(1.0f, pk_k) : 0.0f;
#define PCT_FUSED(R, MODE)                                                                                          \
  hipLaunchKernelGGL((k_project_fused<R, MODE>), g, b, lds, s, P, static_cast<const PathRec<R> *>(recs), order,    \
                     first, n, gl, count, x, num, cnt, pk, pk_bits, pk_scale, status)
  if (P.path_fp32) {
    if (mode == 2) PCT_FUSED(float, 2);
    else if (mode == 1) PCT_FUSED(float, 1);
    else PCT_FUSED(float, 0);
  } else {
    if (mode == 2) PCT_FUSED(double, 2);
    else if (mode == 1) PCT_FUSED(double, 1);
    else PCT_FUSED(double, 0);
  }
#undef PCT_FUSED
  return hipGetLastError();
}

hipError_t launch_apply_counts(float *x, float *num, uint32_t *cnt, uint16_t *blk_cnt, int mode, const uint8_t *mask,
                               int64_t M, float lambda, uint32_t *status, hipStream_t s, uint8_t *touched,
                               const PathParams *Bp, float *xb, int64_t Mb, unsigned long long *pk, int pk_bits,
                               int pk_k) {
  const int64_t Mq = Bp ? Mb : M;
  const dim3 g(grid_for(Mq, 256, 8192)), b(256);
  const int32_t nx = Bp ? Bp->nx : 0, ny = Bp ? Bp->ny : 0, nz = Bp ? Bp->nz : 0;
  const int32_t nbx = Bp ? Bp->nbx : 1, nby = Bp ? Bp->nby : 1;
#define PCT_APPLY(MODE, BRICK)                                                                                     \
  hipLaunchKernelGGL((k_apply<MODE, BRICK>), g, b, 0, s, x, num, cnt, blk_cnt, mask, M, lambda, status, touched, nx, \
                     ny, nz, nbx, nby, xb, Mq, mode == 2 ? nullptr : pk, pk_bits, std::ldexp(1.0, -pk_k))
  if (Bp) {
    if (mode == 0) PCT_APPLY(0, true);
    else if (mode == 1) PCT_APPLY(1, true);
    else PCT_APPLY(2, true);
  } else {
    if (mode == 0) PCT_APPLY(0, false);
    else if (mode == 1) PCT_APPLY(1, false);
    else PCT_APPLY(2, false);
  }
#undef PCT_APPLY
  return hipGetLastError();
}

hipError_t launch_to_bricks(const PathParams &P, const float *x, float *xb, int64_t Mb, hipStream_t s) {
  if (Mb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_bricks, dim3(grid_for(Mb, 256, 8192)), dim3(256), 0, s, x, xb, P.nx, P.ny, P.nz, P.nbx,
                     P.nby, Mb);
  return hipGetLastError();
}

hipError_t launch_carp_accumulate(const float *xs, uint8_t *touched, float *acc, uint16_t *tc, int64_t M,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_carp_accumulate, dim3(grid_for(M, 256, 8192)), dim3(256), 0, s, xs, touched, acc, tc, M);
  return hipGetLastError();
}

hipError_t launch_carp_average(float *x, float *acc, uint16_t *tc, int64_t M, hipStream_t s) {
  hipLaunchKernelGGL(k_carp_average, dim3(grid_for(M, 256, 8192)), dim3(256), 0, s, x, acc, tc, M);
  return hipGetLastError();
}

hipError_t launch_copy_f32(const float *a, float *b, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_f32, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, a, b, n);
  return hipGetLastError();
}

hipError_t launch_art(const int64_t *row_ptr, const int32_t *idx, const void *len, int32_t len_dtype,
                      float len_unit, const double *norm2, const float *b, const int64_t *order, int64_t n,
                      int64_t M, float *x, const uint8_t *mask, float lambda, uint32_t *status, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (len_dtype == 0)
    hipLaunchKernelGGL(k_art<0>, dim3(1), dim3(64), 0, s, row_ptr, idx, len, len_unit, norm2, b, order, n, M, x,
                       mask, lambda, status);
  else
    hipLaunchKernelGGL(k_art<1>, dim3(1), dim3(64), 0, s, row_ptr, idx, len, len_unit, norm2, b, order, n, M, x,
                       mask, lambda, status);
  return hipGetLastError();
}

hipError_t launch_residual_cached(const int64_t *row_ptr, const int32_t *idx, const void *len, int32_t len_dtype,
                                  float len_unit, const float *b, int64_t n, int64_t M, const float *x,
                                  double *partials, double *out, hipStream_t s) {
  const unsigned grid = grid_for(n, 4, (unsigned)(kMaxPartials - 1));
  if (len_dtype == 0)
    hipLaunchKernelGGL(k_resid_cached<0>, dim3(grid), dim3(256), 0, s, row_ptr, idx, len, len_unit, b, n, M, x,
                       partials);
  else
    hipLaunchKernelGGL(k_resid_cached<1>, dim3(grid), dim3(256), 0, s, row_ptr, idx, len, len_unit, b, n, M, x,
                       partials);
  hipLaunchKernelGGL(k_resid_final, dim3(1), dim3(256), 0, s, partials, (int64_t)grid, out);
  return hipGetLastError();
}

// one chunk of rows of the fused residual (accumulate: add to the partial
// sums of earlier chunks); the final sum is launch_residual_final
hipError_t launch_residual_fused(const PathParams &P, const void *recs, int64_t n, const float *x, double *partials,
                                 uint32_t *status, bool accumulate, hipStream_t s) {
  const size_t lds = (size_t)P.waves_per_block * row_buf_bytes(P.emax);
  const unsigned grid = kResidFusedGrid;
  if (P.path_fp32)
    hipLaunchKernelGGL(k_resid_fused<float>, dim3(grid), dim3(P.waves_per_block * kWave), lds, s, P,
                       static_cast<const PathRec<float> *>(recs), n, x, partials, status, accumulate ? 1 : 0);
  else
    hipLaunchKernelGGL(k_resid_fused<double>, dim3(grid), dim3(P.waves_per_block * kWave), lds, s, P,
                       static_cast<const PathRec<double> *>(recs), n, x, partials, status, accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_residual_final(const double *partials, int64_t np, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_resid_final, dim3(1), dim3(256), 0, s, partials, np, out);
  return hipGetLastError();
}

hipError_t launch_poison_on_status(double *out, const uint32_t *status, hipStream_t s) {
  hipLaunchKernelGGL(k_poison, dim3(1), dim3(1), 0, s, out, status);
  return hipGetLastError();
}

hipError_t launch_roi(const float *x, const uint8_t *labels, int64_t M, int32_t n_labels, double *sums,
                      int64_t *counts, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_small<double>, dim3(1), dim3(256), 0, s, sums, (int64_t)n_labels);
  hipLaunchKernelGGL(k_zero_small<int64_t>, dim3(1), dim3(256), 0, s, counts, (int64_t)n_labels);
  if (M > 0)
    hipLaunchKernelGGL(k_roi, dim3(grid_for(M, 256, 1024)), dim3(256), 0, s, x, labels, M, n_labels, sums,
                       reinterpret_cast<unsigned long long *>(counts));
  return hipGetLastError();
}

}  // namespace pct
