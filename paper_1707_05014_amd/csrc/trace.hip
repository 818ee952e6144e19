// Row construction kernels (paper Sec. 2: MLP per proton -> its row of A)
// and small utility kernels (fills, the row-pointer scan).
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "path_device.h"

namespace pct {

// Per-proton set-up of rows [first, first + count) (history order[first + q]
// when order is given, else first + q), one thread per proton: hull entry and
// exit, end states, the prior's moments at the path's end and b_i, into
// recs[q].  Histories with non-finite values get no path (flagged when
// flag_nonfinite); an order entry outside [0, n) sets kStBadIndex.
template <typename R>
__global__ void __launch_bounds__(256) k_path_setup(PathParams P, HistPtrs H, const int64_t *__restrict__ order,
                                                    int64_t first, int64_t count, int64_t n,
                                                    PathRec<R> *__restrict__ recs, uint32_t *status,
                                                    int flag_nonfinite) {
  __shared__ R s_cF[24];
  stage_prior<R>(P, s_cF);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += stride) {
    const int64_t i = order ? order[first + q] : first + q;
    ProtonPath<R> pp;
    pp.valid = false;
    pp.K = 0;
    float b = 0.0f;
    if ((uint64_t)i >= (uint64_t)n) {
      atomicOr(status, kStBadIndex);
    } else {
      float h[10];
      load_history(H, i, h);
      bool fin = true;
#pragma unroll
      for (int k = 0; k < 10; ++k) fin = fin && isfinite(h[k]);
      if (!fin && flag_nonfinite) atomicOr(status, kStNonFinite);
      setup_path<R>(P, s_cF, h, pp);
      b = h[9];
    }
    store_record<R>(pp, b, recs + q);
  }
}

// One wavefront per proton of rows [i0, i0 + nrows) (set-up records
// recs[0, nrows)): the row is built in LDS, its entry count goes to cnt[q]
// and, when st_idx is given, its entries to the staging slots
// [q * emax, q * emax + count) with ||a_i||^2 (FP64, from the FP32 lengths)
// to norm2[i0 + q].  A single path pass per proton: the compaction below
// moves the staged rows into CSR order once the counts are scanned.
#ifndef PCT_TRACE_WAVES
#define PCT_TRACE_WAVES 6
#endif
template <typename R>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PCT_TRACE_WAVES))) k_trace_stage(PathParams P, const PathRec<R> *__restrict__ recs, int64_t i0, int64_t nrows,
                                                     int64_t *cnt, int32_t *st_idx, float *st_len, double *norm2,
                                                     uint32_t *status) {
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
  for (int64_t q = (int64_t)blockIdx.x * P.waves_per_block + wid; q < nrows; q += stride) {
    const int64_t i = i0 + q;
    ProtonPath<R> pp;
    float b;
    load_record<R>(recs + q, pp, b);
    const int c = build_row<R>(P, s_cF, pp, s_vox, s_len, s_aux, status);
    if (lane == 0) cnt[q] = c;
    if (!st_idx) continue;
    int32_t *di = st_idx + q * P.emax;
    float *dl = st_len + q * P.emax;
    double acc = 0.0;
    for (int e = lane; e < c; e += kWave) {
      const float l = s_len[e];
      di[e] = s_vox[e];
      dl[e] = l;
      acc += (double)l * (double)l;
    }
    acc = wave_sum_f64(acc);
    if (lane == 0) norm2[i] = acc;
  }
}

// Staged rows [i0, i0 + nrows) -> CSR at row_ptr (already scanned), one
// wavefront per row.  Rows that would end past the capacity are not written
// (kStRowCap).  LDO: 0 float lengths, 1 half lengths in units of len_unit.
template <int LDO>
__global__ void __launch_bounds__(256) k_trace_compact(int64_t i0, int64_t nrows, const int64_t *__restrict__ row_ptr,
                                                       const int32_t *__restrict__ st_idx,
                                                       const float *__restrict__ st_len, int emax, int32_t *idx,
                                                       void *len, float len_scale, int64_t cap, uint32_t *status) {
  const int lane = wave_lane();
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x / kWave);
  for (int64_t q = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; q < nrows; q += stride) {
    const int64_t e0 = row_ptr[i0 + q], e1 = row_ptr[i0 + q + 1];
    if (e1 > cap) {
      if (lane == 0) atomicOr(status, kStRowCap);
      continue;
    }
    const int c = (int)(e1 - e0);
    const int32_t *si = st_idx + q * emax;
    const float *sl = st_len + q * emax;
    for (int e = lane; e < c; e += kWave) {
      idx[e0 + e] = si[e];
      if (LDO == 0)
        reinterpret_cast<float *>(len)[e0 + e] = sl[e];
      else
        reinterpret_cast<__half *>(len)[e0 + e] = __float2half(sl[e] * len_scale);
    }
  }
}

// cnt[0..n) hold counts (cnt = row_ptr + i0 + 1); turn them into offsets that
// continue from row_ptr[i0].  Three passes over chunks of kScanChunk: chunk
// totals, a scan of the totals by one workgroup, then in-chunk scans with the
// chunk offset.
__global__ void __launch_bounds__(256) k_scan_totals(const int64_t *cnt, int64_t n, int64_t *tot) {
  __shared__ int64_t red[256];
  const int64_t c0 = (int64_t)blockIdx.x * kScanChunk;
  int64_t acc = 0;
  for (int64_t e = c0 + threadIdx.x; e < c0 + kScanChunk && e < n; e += 256) acc += cnt[e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) tot[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_scan_offsets(int64_t *tot, int64_t nchunks, const int64_t *base) {
  __shared__ int64_t buf[256];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = *base;
  __syncthreads();
  for (int64_t b = 0; b < nchunks; b += 256) {
    const int64_t e = b + threadIdx.x;
    int64_t v = e < nchunks ? tot[e] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      int64_t add = (int)threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
      __syncthreads();
      buf[threadIdx.x] += add;
      __syncthreads();
    }
    if (e < nchunks) tot[e] = carry + buf[threadIdx.x] - v;  // exclusive
    __syncthreads();
    if (threadIdx.x == 255) carry += buf[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) tot[nchunks] = carry;
}

// in-chunk inclusive scan of cnt[e] (= row_ptr[e + 1]) plus the chunk offset
__global__ void __launch_bounds__(256) k_scan_apply(int64_t *cnt, int64_t n, const int64_t *tot) {
  __shared__ int64_t buf[256];
  __shared__ int64_t carry;
  const int64_t c0 = (int64_t)blockIdx.x * kScanChunk;
  if (threadIdx.x == 0) carry = tot[blockIdx.x];
  __syncthreads();
  for (int64_t b = c0; b < c0 + kScanChunk && b < n; b += 256) {
    const int64_t e = b + threadIdx.x;
    const int64_t v = (e < n && e < c0 + kScanChunk) ? cnt[e] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      int64_t add = (int)threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
      __syncthreads();
      buf[threadIdx.x] += add;
      __syncthreads();
    }
    if (e < n && e < c0 + kScanChunk) cnt[e] = carry + buf[threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 255) carry += buf[255];
    __syncthreads();
  }
}

__global__ void k_zero_first(int64_t *p) { p[0] = 0; }

template <typename T>
__global__ void __launch_bounds__(256) k_fill(T *p, int64_t n, T v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

static inline unsigned grid_for(int64_t n, int per_block, unsigned cap) {
  int64_t g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

hipError_t launch_path_setup(const PathParams &P, const HistPtrs &H, const int64_t *order, int64_t first,
                             int64_t count, int64_t n, void *recs, uint32_t *status, bool flag_nonfinite,
                             hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const unsigned grid = grid_for(count, 256, 1u << 16);
  if (P.path_fp32)
    hipLaunchKernelGGL(k_path_setup<float>, dim3(grid), dim3(256), 0, s, P, H, order, first, count, n,
                       static_cast<PathRec<float> *>(recs), status, flag_nonfinite ? 1 : 0);
  else
    hipLaunchKernelGGL(k_path_setup<double>, dim3(grid), dim3(256), 0, s, P, H, order, first, count, n,
                       static_cast<PathRec<double> *>(recs), status, flag_nonfinite ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_trace_stage(const PathParams &P, const void *recs, int64_t i0, int64_t nrows, int64_t *cnt,
                              int32_t *st_idx, float *st_len, double *norm2, uint32_t *status, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  const unsigned threads = (unsigned)(P.waves_per_block * kWave);
  const size_t lds = (size_t)P.waves_per_block * row_buf_bytes(P.emax);
  const unsigned grid = grid_for(nrows, P.waves_per_block, 1u << 20);
  if (P.path_fp32)
    hipLaunchKernelGGL(k_trace_stage<float>, dim3(grid), dim3(threads), lds, s, P,
                       static_cast<const PathRec<float> *>(recs), i0, nrows, cnt, st_idx, st_len, norm2, status);
  else
    hipLaunchKernelGGL(k_trace_stage<double>, dim3(grid), dim3(threads), lds, s, P,
                       static_cast<const PathRec<double> *>(recs), i0, nrows, cnt, st_idx, st_len, norm2, status);
  return hipGetLastError();
}

hipError_t launch_trace_compact(int64_t i0, int64_t nrows, const int64_t *row_ptr, const int32_t *st_idx,
                                const float *st_len, int emax, int32_t *idx, void *len, int32_t len_dtype,
                                float len_scale, int64_t cap, uint32_t *status, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  const unsigned grid = grid_for(nrows, 4, 1u << 20);
  if (len_dtype == 0)
    hipLaunchKernelGGL(k_trace_compact<0>, dim3(grid), dim3(256), 0, s, i0, nrows, row_ptr, st_idx, st_len, emax,
                       idx, len, len_scale, cap, status);
  else
    hipLaunchKernelGGL(k_trace_compact<1>, dim3(grid), dim3(256), 0, s, i0, nrows, row_ptr, st_idx, st_len, emax,
                       idx, len, len_scale, cap, status);
  return hipGetLastError();
}

hipError_t launch_scan_rows(int64_t *row_ptr, int64_t i0, int64_t nrows, int64_t *scan_tmp, hipStream_t s) {
  if (i0 == 0) hipLaunchKernelGGL(k_zero_first, dim3(1), dim3(1), 0, s, row_ptr);
  if (nrows <= 0) return hipGetLastError();
  const int64_t nchunks = (nrows + kScanChunk - 1) / kScanChunk;
  int64_t *cnt = row_ptr + i0 + 1;
  hipLaunchKernelGGL(k_scan_totals, dim3((unsigned)nchunks), dim3(256), 0, s, cnt, nrows, scan_tmp);
  hipLaunchKernelGGL(k_scan_offsets, dim3(1), dim3(256), 0, s, scan_tmp, nchunks, row_ptr + i0);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nchunks), dim3(256), 0, s, cnt, nrows, scan_tmp);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_u8(uint8_t *p, int64_t n, uint8_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill<uint8_t>, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace pct
