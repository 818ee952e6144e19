// Microbenchmarks of the memory paths that bound the sweep kernels, run on
// the device the library is used on: the peaks against which the sweeps'
// achieved rates are reported (no published figure exists for the
// last-level-cache bandwidth or for the atomic rate of an MI355X).
//
//   copy          plain device copy: HBM bandwidth
//   gather        4-byte reads along path-like voxel runs (64 voxels of a
//                 line per wavefront pass, in brick order) of an image of
//                 `region` voxels: one that fits the last-level cache gives
//                 its gather rate, the way the rebuilt-row sweeps read x
//   atomic        FP32 atomic adds along the same runs into the image: the
//                 global atomic rate of the rebuilt-row sweeps' scatter
//   atomic_xcd    the same adds into a private copy of the image per
//                 accelerator complex die (XCD), the copy chosen by the
//                 die's hardware id, with workgroup-scope atomics
//   lds_atomic    FP32 atomic adds at hashed positions of a 2048-float LDS
//                 image per workgroup (a tile's numerators, entries in no
//                 particular order)
#include <hip/hip_runtime.h>

#include "pct_internal.h"

namespace pct {

namespace {

constexpr int kProbeBlock = 256;
constexpr int kLdsImage = 2048;

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

// Path-like rows: row r is a straight line in the z plane of a grid of 200 x
// 200 x (region / 40000) voxels, at a hashed angle, start and slice; lane l
// takes the voxel at distance l (voxel units) along it (wrapped into the
// grid), numbered in 4 x 4 x 4 bricks as the rebuilt-row sweeps number
// theirs (50 x 50 x ... bricks).
__device__ __forceinline__ int64_t path_index(uint64_t r, int lane, int64_t region) {
  const int nz = (int)(region / 40000);
  const uint32_t h = mix32((uint32_t)r ^ 0x9e3779b9U * (uint32_t)(r >> 32));
  const float phi = (float)(mix32(h + 1u) & 0xffffu) * (6.2831853f / 65536.0f);
  const float x0 = (float)(h % 200u), y0 = (float)((h >> 8) % 200u);
  const int iz = (int)(mix32(h + 2u) % (uint32_t)nz);
  int ix = (int)floorf(x0 + lane * cosf(phi)), iy = (int)floorf(y0 + lane * sinf(phi));
  ix = ((ix % 200) + 200) % 200;
  iy = ((iy % 200) + 200) % 200;
  return ((((int64_t)(iz >> 2) * 50 + (iy >> 2)) * 50 + (ix >> 2)) << 6) | ((iz & 3) << 4) | ((iy & 3) << 2) | (ix & 3);
}

typedef float v4f __attribute__((ext_vector_type(4)));

// four 16-byte loads in flight per thread before their stores
__global__ void __launch_bounds__(kProbeBlock) k_probe_copy(const v4f *__restrict__ a, v4f *__restrict__ b,
                                                            int64_t n4) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < n4; i += 4 * stride) {
    const v4f v0 = __builtin_nontemporal_load(a + i), v1 = __builtin_nontemporal_load(a + i + stride);
    const v4f v2 = __builtin_nontemporal_load(a + i + 2 * stride), v3 = __builtin_nontemporal_load(a + i + 3 * stride);
    __builtin_nontemporal_store(v0, b + i);
    __builtin_nontemporal_store(v1, b + i + stride);
    __builtin_nontemporal_store(v2, b + i + 2 * stride);
    __builtin_nontemporal_store(v3, b + i + 3 * stride);
  }
  for (; i < n4; i += stride) b[i] = a[i];
}

__global__ void __launch_bounds__(kProbeBlock) k_probe_gather(const float *__restrict__ src, int64_t region,
                                                              int64_t rows, float *__restrict__ out) {
  const int lane = __lane_id();
  const int64_t nw = (int64_t)gridDim.x * (kProbeBlock / 64);
  float acc = 0.f;
  for (int64_t r = (int64_t)blockIdx.x * (kProbeBlock / 64) + threadIdx.x / 64; r < rows; r += nw)
    acc += src[path_index((uint64_t)r, lane, region)];
  out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
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
    const uint32_t j = mix32((uint32_t)(r * 64 + lane) * 2654435761U + blockIdx.x) & (kLdsImage - 1);
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
      hipLaunchKernelGGL(k_probe_copy, g, b, 0, s, static_cast<const v4f *>(buf),
                         reinterpret_cast<v4f *>(static_cast<float *>(buf) + region), n4);
      break;
    }
    case 1:
      hipLaunchKernelGGL(k_probe_gather, g, b, 0, s, static_cast<const float *>(buf), region, n_ops / 64,
                         static_cast<float *>(buf) + region);
      break;
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
