// Microbenchmarks of the memory paths that bound the sweep kernels, run on
// the device the library is used on: the peaks against which the sweeps'
// achieved rates are reported (no published figure exists for the
// last-level-cache bandwidth or for the atomic rate of an MI355X).
//
//   copy          plain device copy: HBM bandwidth
//   gather        4-byte reads at hashed positions inside a region (a
//                 region that fits the last-level cache gives its gather
//                 bandwidth; the sweeps gather x this way)
//   atomic        FP32 atomic adds along path-like voxel runs (one row of 64
//                 consecutive voxels of a random line per wavefront pass)
//                 into one image of `region` voxels: the global atomic rate
//   atomic_xcd    the same adds into a private copy of the image per
//                 accelerator complex die (XCD), the copy chosen by the
//                 die's hardware id, with workgroup-scope atomics
//   lds_atomic    the same adds into a 16384-float LDS image per workgroup
#include <hip/hip_runtime.h>

#include "pct_internal.h"

namespace pct {

namespace {

constexpr int kProbeBlock = 256;
constexpr int kLdsImage = 16384;

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

// index of lane `lane` in path-like row r of an image of `region` voxels:
// start voxel and stride (1, 200, 201, 40000 or 40201: along x, y, a diagonal,
// z or a space diagonal of a 200 x 200 x ... grid) from a hash of r
__device__ __forceinline__ int64_t path_index(uint64_t r, int lane, int64_t region) {
  const uint32_t h = mix32((uint32_t)r ^ 0x9e3779b9U * (uint32_t)(r >> 32));
  const uint32_t sel = mix32(h + 1u) % 5u;
  const int64_t stride = sel == 0 ? 1 : (sel == 1 ? 200 : (sel == 2 ? 201 : (sel == 3 ? 40000 : 40201)));
  const int64_t start = (int64_t)(h % (uint32_t)region);
  return (start + stride * lane) % region;
}

__global__ void __launch_bounds__(kProbeBlock) k_probe_copy(const float4 *__restrict__ a, float4 *__restrict__ b,
                                                            int64_t n4) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) b[i] = a[i];
}

__global__ void __launch_bounds__(kProbeBlock) k_probe_gather(const float *__restrict__ src, int64_t region,
                                                              int64_t per_thread, float *__restrict__ out) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  float acc = 0.f;
  uint32_t h = mix32(t * 2654435761U + 12345U);
  for (int64_t k = 0; k < per_thread; ++k) {
    h = h * 1664525U + 1013904223U;
    acc += src[(int64_t)(mix32(h) % (uint32_t)region)];
  }
  out[t] = acc;
}

template <int KIND>  // 0: one image, agent-scope adds; 1: per-die image, workgroup-scope adds
__global__ void __launch_bounds__(kProbeBlock) k_probe_atomic(float *img, int64_t region, int64_t rows) {
  const int lane = __lane_id();
  const int64_t nw = (int64_t)gridDim.x * (kProbeBlock / 64);
  float *dst = img;
  if constexpr (KIND == 1) {
    const int xcc = __builtin_amdgcn_s_getreg((3 << 11) | 20) & 7;  // HW_REG_XCC_ID, bits 3:0
    dst = img + (int64_t)xcc * region;
  }
  for (int64_t r = (int64_t)blockIdx.x * (kProbeBlock / 64) + threadIdx.x / 64; r < rows; r += nw) {
    const int64_t j = path_index((uint64_t)r, lane, region);
    if constexpr (KIND == 0)
      atomicAdd(&dst[j], 1.0f);
    else
      __hip_atomic_fetch_add(&dst[j], 1.0f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

__global__ void __launch_bounds__(kProbeBlock) k_probe_lds_atomic(int64_t rows_per_block, float *out) {
  __shared__ float img[kLdsImage];
  for (int q = threadIdx.x; q < kLdsImage; q += kProbeBlock) img[q] = 0.f;
  __syncthreads();
  const int lane = __lane_id();
  const int w = threadIdx.x / 64;
  for (int64_t r = w; r < rows_per_block; r += kProbeBlock / 64) {
    const int64_t j = path_index((uint64_t)r * 977u + blockIdx.x, lane, kLdsImage);
    atomicAdd(&img[j], 1.0f);
  }
  __syncthreads();
  float s = 0.f;
  for (int q = threadIdx.x; q < kLdsImage; q += kProbeBlock) s += img[q];
  if (s != 0.f && threadIdx.x == 0) out[blockIdx.x] = s;
}

}  // namespace

// bytes of `buf` each probe needs for (region, n_ops); see pct.h
size_t probe_bytes(int kind, int64_t region, int64_t n_ops, int64_t grid) {
  switch (kind) {
    case 0: return (size_t)region * 8;
    case 1: return (size_t)region * 4 + (size_t)grid * kProbeBlock * 4;
    case 2: return (size_t)region * 4;
    case 3: return (size_t)region * 4 * 8;
    case 4: return (size_t)grid * 4;
    default: (void)n_ops; return 0;
  }
}

// one launch of probe `kind` (sizes checked by the caller)
hipError_t launch_probe(int kind, void *buf, int64_t region, int64_t n_ops, int64_t grid, hipStream_t s) {
  const dim3 g((unsigned)grid), b(kProbeBlock);
  switch (kind) {
    case 0: {
      const int64_t n4 = region / 4;  // region floats per half, copied as float4
      hipLaunchKernelGGL(k_probe_copy, g, b, 0, s, static_cast<const float4 *>(buf),
                         reinterpret_cast<float4 *>(static_cast<float *>(buf) + region), n4);
      break;
    }
    case 1: {
      const int64_t per = (n_ops + grid * kProbeBlock - 1) / (grid * kProbeBlock);
      hipLaunchKernelGGL(k_probe_gather, g, b, 0, s, static_cast<const float *>(buf), region, per,
                         static_cast<float *>(buf) + region);
      break;
    }
    case 2:
      hipLaunchKernelGGL(k_probe_atomic<0>, g, b, 0, s, static_cast<float *>(buf), region, n_ops / 64);
      break;
    case 3:
      hipLaunchKernelGGL(k_probe_atomic<1>, g, b, 0, s, static_cast<float *>(buf), region, n_ops / 64);
      break;
    case 4:
      hipLaunchKernelGGL(k_probe_lds_atomic, g, b, 0, s, n_ops / 64 / grid, static_cast<float *>(buf));
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pct
