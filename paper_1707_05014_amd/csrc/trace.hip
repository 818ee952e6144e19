// Row construction kernels (paper Sec. 2: MLP per proton -> its row of A)
// and small utility kernels (fills, the row-pointer scan).
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "path_device.h"

namespace pct {

// One wavefront per proton.  mode 0: write the entry count to row_ptr[i + 1];
// mode 1: write the row (idx, len, norm2) at row_ptr[i] (row_ptr already
// scanned).  Both modes run the same code on the same inputs, so the fill
// pass reproduces the counted rows exactly.
__global__ void __launch_bounds__(256) k_trace(PathParams P, HistPtrs H, int64_t n, int mode, int64_t *row_ptr,
                                               int32_t *idx, void *len, int32_t len_dtype, float len_scale,
                                               double *norm2, uint32_t *status) {
  extern __shared__ int smem[];
  const int wid = threadIdx.x / kWave;
  const int lane = wave_lane();
  int *s_vox = smem + wid * 3 * P.emax;
  float *s_len = reinterpret_cast<float *>(s_vox + P.emax);
  int *s_aux = s_vox + 2 * P.emax;
  const int64_t stride = (int64_t)gridDim.x * P.waves_per_block;
  for (int64_t i = (int64_t)blockIdx.x * P.waves_per_block + wid; i < n; i += stride) {
    float h[10];
    load_history(H, i, h);
    bool fin = true;
    for (int q = 0; q < 10; ++q) fin = fin && isfinite(h[q]);
    if (!fin && lane == 0) atomicOr(status, kStNonFinite);
    const int cnt = build_row_any(P, h, s_vox, s_len, s_aux, status);
    if (mode == 0) {
      if (lane == 0) row_ptr[i + 1] = cnt;
      continue;
    }
    const int64_t start = row_ptr[i];
    const int64_t want = row_ptr[i + 1] - start;
    if (want != cnt) {
      if (lane == 0) atomicOr(status, kStRowMismatch);
      if (lane == 0) norm2[i] = 0.0;
      continue;
    }
    double acc = 0.0;
    for (int e = lane; e < cnt; e += kWave) {
      const float l = s_len[e];
      idx[start + e] = s_vox[e];
      if (len_dtype == 0)
        reinterpret_cast<float *>(len)[start + e] = l;
      else
        reinterpret_cast<__half *>(len)[start + e] = __float2half(l * len_scale);
      acc += (double)l * (double)l;
    }
    acc = wave_sum_f64(acc);
    if (lane == 0) norm2[i] = acc;
  }
}

// row_ptr[1..n] hold counts; turn them into offsets (row_ptr[0] = 0).
// Three passes over chunks of kScanChunk: chunk totals, a scan of the totals
// by one workgroup, then in-chunk scans with the chunk offset.
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

__global__ void __launch_bounds__(256) k_scan_offsets(int64_t *tot, int64_t nchunks) {
  __shared__ int64_t buf[256];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
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

hipError_t launch_trace(const PathParams &P, const HistPtrs &H, int64_t n, int mode, int64_t *row_ptr,
                        int32_t *idx, void *len, int32_t len_dtype, double *norm2, uint32_t *status,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned threads = (unsigned)(P.waves_per_block * kWave);
  const size_t lds = (size_t)P.waves_per_block * 3 * P.emax * sizeof(int);
  const unsigned grid = grid_for(n, P.waves_per_block, 1u << 20);
  const float len_scale = 1.0f / fminf(P.dx, fminf(P.dy, P.dz));
  hipLaunchKernelGGL(k_trace, dim3(grid), dim3(threads), lds, s, P, H, n, mode, row_ptr, idx, len, len_dtype,
                     len_scale, norm2, status);
  return hipGetLastError();
}

hipError_t launch_scan_rows(int64_t *row_ptr, int64_t n, int64_t *scan_tmp, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_first, dim3(1), dim3(1), 0, s, row_ptr);
  if (n <= 0) return hipGetLastError();
  const int64_t nchunks = (n + kScanChunk - 1) / kScanChunk;
  int64_t *cnt = row_ptr + 1;
  hipLaunchKernelGGL(k_scan_totals, dim3((unsigned)nchunks), dim3(256), 0, s, cnt, n, scan_tmp);
  hipLaunchKernelGGL(k_scan_offsets, dim3(1), dim3(256), 0, s, scan_tmp, nchunks);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nchunks), dim3(256), 0, s, cnt, n, scan_tmp);
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

}  // namespace pct
