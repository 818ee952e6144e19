// Kernels of the learned warm start: a small 3D U-Net over the image volume
// (channels-first, one volume at a time: tensor [C][D][H][W], W fastest).
// Operations: 3x3x3 convolution with zero padding (forward, input gradient,
// weight and bias gradients), ReLU, 2x2x2 average pooling, nearest 2x
// upsampling, addition, mean squared error and an Adam step.  FP32 storage
// and accumulation; reductions (weight gradients, loss) are formed in a fixed
// order, so every result is reproducible.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "cnn_internal.h"
#include "path_device.h"

namespace pct {
namespace cnn {

constexpr int kThreads = 256;
constexpr int kTaps = 27;

struct Vol {
  int D, H, W;
  int64_t V;
};

__device__ __forceinline__ Vol make_vol(int D, int H, int W) { return {D, H, W, (int64_t)D * H * W}; }

// The 27 neighbour offsets of voxel p and which of them lie inside the volume.
__device__ __forceinline__ uint32_t tap_mask(const Vol &v, int z, int y, int x) {
  uint32_t m = 0;
#pragma unroll
  for (int t = 0; t < kTaps; ++t) {
    const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    const bool in = z + dz >= 0 && z + dz < v.D && y + dy >= 0 && y + dy < v.H && x + dx >= 0 && x + dx < v.W;
    m |= in ? (1u << t) : 0u;
  }
  return m;
}

__device__ __forceinline__ int64_t tap_offset(const Vol &v, int t) {
  const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
  return ((int64_t)dz * v.H + dy) * v.W + dx;
}

// y[co] = b[co] + sum_ci sum_t w[co][ci][t] x[ci][p + off(t)], for a block of
// COB output channels per thread (weights are wave-uniform: scalar loads).
template <int COB>
__global__ void __launch_bounds__(kThreads) k_conv3d(const float *__restrict__ x, const float *__restrict__ w,
                                                     const float *__restrict__ b, float *__restrict__ y, int cin,
                                                     int cout, int D, int H, int W) {
  const Vol v = make_vol(D, H, W);
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int co0 = blockIdx.y * COB;
  const bool live = p < v.V;
  const int64_t pc = live ? p : 0;
  const int xq = (int)(pc % W), yq = (int)((pc / W) % H), zq = (int)(pc / ((int64_t)W * H));
  const uint32_t m = tap_mask(v, zq, yq, xq);
  float acc[COB];
#pragma unroll
  for (int c = 0; c < COB; ++c) acc[c] = (b && co0 + c < cout) ? b[co0 + c] : 0.0f;
  for (int ci = 0; ci < cin; ++ci) {
    const float *xc = x + (int64_t)ci * v.V + pc;
    float xt[kTaps];
#pragma unroll
    for (int t = 0; t < kTaps; ++t) {
      // taps outside the volume read the centre voxel (always in bounds) and use 0
      const bool in = (m >> t) & 1u;
      const float xv = xc[in ? tap_offset(v, t) : 0];
      xt[t] = in ? xv : 0.0f;
    }
#pragma unroll
    for (int c = 0; c < COB; ++c) {
      if (co0 + c < cout) {
        const float *wc = w + ((int64_t)(co0 + c) * cin + ci) * kTaps;
#pragma unroll
        for (int t = 0; t < kTaps; ++t) acc[c] = fmaf(wc[t], xt[t], acc[c]);
      }
    }
  }
  if (!live) return;
#pragma unroll
  for (int c = 0; c < COB; ++c)
    if (co0 + c < cout) y[(int64_t)(co0 + c) * v.V + p] = acc[c];
}

// wt[ci][co][26 - t] = w[co][ci][t]: the input gradient of a convolution is the
// convolution of the output gradient with these weights
__global__ void __launch_bounds__(kThreads) k_flip(const float *__restrict__ w, float *__restrict__ wt, int cin,
                                                   int cout) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t n = (int64_t)cin * cout * kTaps;
  if (i >= n) return;
  const int t = (int)(i % kTaps);
  const int64_t r = i / kTaps;
  const int ci = (int)(r % cin), co = (int)(r / cin);
  wt[((int64_t)ci * cout + co) * kTaps + (kTaps - 1 - t)] = w[i];
}

// Weight and bias gradients, stage 1: workgroup (tile g, channel block)
// sums over the tile's voxels
//   part[g][co][ci*27 + t] = sum_p dy[co][p] x[ci][p + off(t)],  part[g][co][cin*27] = sum_p dy[co][p]
// A tile is 64 voxels along W (one per lane) x kTileY rows x kTileZ planes;
// the four wavefronts take every fourth row, so row coordinates are
// wave-uniform and only the W-neighbours' validity varies per lane.  Each
// lane folds its rows into kWgCob x 27 register accumulators per input
// channel; each wavefront then adds its lanes with DPP prefix sums and the
// workgroup adds its wavefronts in order (fixed summation order throughout).
// Small volumes also split the input channels over workgroups (grid z), so
// that every level of the network fills the chip.
constexpr int kWaves = kThreads / 64;
constexpr int kWgCob = 4;
constexpr int kTileY = 16, kTileZ = 16;

__device__ __forceinline__ float wave_total(float v) {
  const float s = wave_incl_scan_dpp(v);
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, s), 63));
}

__global__ void __launch_bounds__(kThreads) k_wgrad_part(const float *__restrict__ x, const float *__restrict__ dy,
                                                         float *__restrict__ part, int cin, int cout, int D, int H,
                                                         int W, int tiles_x, int tiles_y, int ci_per_wg) {
  __shared__ float red[kWaves][kWgCob][kTaps + 1];
  const int tile = blockIdx.x;
  const int txi = tile % tiles_x, tyi = (tile / tiles_x) % tiles_y, tzi = tile / (tiles_x * tiles_y);
  const int co0 = blockIdx.y * kWgCob;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int xq = txi * 64 + lane;
  const bool xin = xq < W;
  const int xc = xin ? xq : W - 1;  // lanes past the edge read a valid voxel and use 0
  const bool xm = xin && xq >= 1, xp = xin && xq + 1 < W;
  const int y0 = tyi * kTileY, z0 = tzi * kTileZ;
  const int ny = min(kTileY, H - y0), nz = min(kTileZ, D - z0);
  const int nrows = ny * nz;
  const int64_t V = (int64_t)D * H * W;
  const int64_t stride = (int64_t)cin * kTaps + 1;
  // input channels [ci0, ci1) of this workgroup; the bias gradient comes from
  // the workgroups that start at channel 0
  const int ci0 = blockIdx.z * ci_per_wg, ci1 = min(cin, ci0 + ci_per_wg);
  float gsum[kWgCob];
#pragma unroll
  for (int c = 0; c < kWgCob; ++c) gsum[c] = 0.0f;
  for (int ci = ci0; ci < ci1; ++ci) {
    const float *xch = x + (int64_t)ci * V;
    float acc[kWgCob][kTaps];
#pragma unroll
    for (int c = 0; c < kWgCob; ++c)
#pragma unroll
      for (int t = 0; t < kTaps; ++t) acc[c][t] = 0.0f;
    for (int r = wid; r < nrows; r += kWaves) {
      const int zz = z0 + r / ny, yy = y0 + r % ny;  // wave-uniform
      const int64_t p = ((int64_t)zz * H + yy) * W + xc;
      float g[kWgCob];
#pragma unroll
      for (int c = 0; c < kWgCob; ++c) {
        const float gv = (co0 + c < cout) ? dy[(int64_t)(co0 + c) * V + p] : 0.0f;
        g[c] = xin ? gv : 0.0f;
        if (ci == 0) gsum[c] += g[c];
      }
#pragma unroll
      for (int a = 0; a < 9; ++a) {
        const int dz = a / 3 - 1, dyy = a % 3 - 1;
        const bool rowin = zz + dz >= 0 && zz + dz < D && yy + dyy >= 0 && yy + dyy < H;  // wave-uniform
        if (!rowin) continue;
        const float *row = xch + p + ((int64_t)dz * H + dyy) * W;
        const float vm = row[xm ? -1 : 0], v0 = row[0], vp = row[xp ? 1 : 0];
        const float xv[3] = {xm ? vm : 0.0f, v0, xp ? vp : 0.0f};
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
          for (int c = 0; c < kWgCob; ++c) acc[c][a * 3 + b] = fmaf(g[c], xv[b], acc[c][a * 3 + b]);
      }
    }
#pragma unroll
    for (int c = 0; c < kWgCob; ++c)
#pragma unroll
      for (int t = 0; t < kTaps; ++t) {
        const float sw = wave_total(acc[c][t]);
        if (lane == 0) red[wid][c][t] = sw;
      }
    if (ci == 0) {
#pragma unroll
      for (int c = 0; c < kWgCob; ++c) {
        const float sg = wave_total(gsum[c]);
        if (lane == 0) red[wid][c][kTaps] = sg;
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < kWgCob * (kTaps + 1)) {
      const int c = threadIdx.x / (kTaps + 1), t = threadIdx.x % (kTaps + 1);
      if (co0 + c < cout && (t < kTaps || ci == 0)) {
        float sum = 0.0f;
        for (int w2 = 0; w2 < kWaves; ++w2) sum += red[w2][c][t];
        float *out = part + ((int64_t)tile * cout + co0 + c) * stride;
        out[t < kTaps ? (int64_t)ci * kTaps + t : (int64_t)cin * kTaps] = sum;
      }
    }
    __syncthreads();
  }
}

// stage 2: dw[co][ci][t] = sum_g part[g][co][ci][t] (g in order), db likewise
__global__ void __launch_bounds__(kThreads) k_wgrad_sum(const float *__restrict__ part, float *__restrict__ dw,
                                                        float *__restrict__ db, int64_t chunks, int cin, int cout) {
  const int64_t stride = (int64_t)cin * kTaps + 1;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= (int64_t)cout * stride) return;
  const int64_t co = i / stride, j = i % stride;
  float s = 0.0f;
  for (int64_t g = 0; g < chunks; ++g) s += part[(g * cout + co) * stride + j];
  if (j < (int64_t)cin * kTaps)
    dw[co * cin * kTaps + j] = s;
  else if (db)
    db[co] = s;
}

__global__ void __launch_bounds__(kThreads) k_relu(const float *x, float *y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) y[i] = fmaxf(x[i], 0.0f);
}

// dx = dy where y > 0 (y = the ReLU output), else 0.  The elementwise kernels
// read and write element i only, so they may run in place.
__global__ void __launch_bounds__(kThreads) k_relu_bwd(const float *y, const float *dy, float *dx,
                                                       int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) dx[i] = y[i] > 0.0f ? dy[i] : 0.0f;
}

// 2x2x2 average pooling of [C][D][H][W] (even D, H, W) -> [C][D/2][H/2][W/2]
__global__ void __launch_bounds__(kThreads) k_pool(const float *__restrict__ x, float *__restrict__ y, int C, int D,
                                                   int H, int W) {
  const int d = D / 2, h = H / 2, w = W / 2;
  const int64_t n = (int64_t)C * d * h * w;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const int xo = (int)(i % w), yo = (int)((i / w) % h), zo = (int)((i / ((int64_t)w * h)) % d);
  const int64_t c = i / ((int64_t)w * h * d);
  const float *xc = x + c * D * H * W;
  float s = 0.0f;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int z = 2 * zo + (q >> 2), yy = 2 * yo + ((q >> 1) & 1), xx = 2 * xo + (q & 1);
    s += xc[((int64_t)z * H + yy) * W + xx];
  }
  y[i] = s * 0.125f;
}

// gradient of the pooling: every fine voxel gets 1/8 of its coarse voxel's gradient
__global__ void __launch_bounds__(kThreads) k_pool_bwd(const float *__restrict__ dy, float *__restrict__ dx, int C,
                                                       int D, int H, int W) {
  const int64_t n = (int64_t)C * D * H * W;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const int xx = (int)(i % W), yy = (int)((i / W) % H), z = (int)((i / ((int64_t)W * H)) % D);
  const int64_t c = i / ((int64_t)W * H * D);
  const int d = D / 2, h = H / 2, w = W / 2;
  dx[i] = 0.125f * dy[((c * d + z / 2) * h + yy / 2) * w + xx / 2];
}

// nearest 2x upsampling of [C][d][h][w] -> [C][2d][2h][2w]
__global__ void __launch_bounds__(kThreads) k_up(const float *__restrict__ x, float *__restrict__ y, int C, int d,
                                                 int h, int w) {
  const int D = 2 * d, H = 2 * h, W = 2 * w;
  const int64_t n = (int64_t)C * D * H * W;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const int xx = (int)(i % W), yy = (int)((i / W) % H), z = (int)((i / ((int64_t)W * H)) % D);
  const int64_t c = i / ((int64_t)W * H * D);
  y[i] = x[((c * d + z / 2) * h + yy / 2) * w + xx / 2];
}

// gradient of the upsampling: each coarse voxel sums its 8 fine voxels
__global__ void __launch_bounds__(kThreads) k_up_bwd(const float *__restrict__ dy, float *__restrict__ dx, int C,
                                                     int d, int h, int w) {
  const int D = 2 * d, H = 2 * h, W = 2 * w;
  const int64_t n = (int64_t)C * d * h * w;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const int xo = (int)(i % w), yo = (int)((i / w) % h), zo = (int)((i / ((int64_t)w * h)) % d);
  const int64_t c = i / ((int64_t)w * h * d);
  const float *g = dy + c * D * H * W;
  float s = 0.0f;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int z = 2 * zo + (q >> 2), yy = 2 * yo + ((q >> 1) & 1), xx = 2 * xo + (q & 1);
    s += g[((int64_t)z * H + yy) * W + xx];
  }
  dx[i] = s;
}

__global__ void __launch_bounds__(kThreads) k_add(const float *a, const float *b, float *y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) y[i] = a[i] + b[i];
}

// y += a x
__global__ void __launch_bounds__(kThreads) k_axpy(float a, const float *__restrict__ x, float *__restrict__ y,
                                                   int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) y[i] = fmaf(a, x[i], y[i]);
}

// y = x where mask != 0, else 0 (restricts an image to the object's hull)
__global__ void __launch_bounds__(kThreads) k_mask(const float *x, const uint8_t *__restrict__ mask, float *y,
                                                   int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) y[i] = mask[i] ? x[i] : 0.0f;
}

// mean squared error: dy = 2 (y - t) / n, per-workgroup FP64 sums of (y - t)^2
__global__ void __launch_bounds__(kThreads) k_mse(const float *__restrict__ y, const float *__restrict__ t,
                                                  float *__restrict__ dy, double *__restrict__ part, int64_t n) {
  __shared__ double red[kThreads];
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  double e2 = 0.0;
  if (i < n) {
    const float e = y[i] - t[i];
    if (dy) dy[i] = 2.0f * e / (float)n;
    e2 = (double)e * (double)e;
  }
  red[threadIdx.x] = e2;
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(kThreads) k_mse_final(const double *__restrict__ part, int64_t np, int64_t n,
                                                        double *__restrict__ loss) {
  __shared__ double red[kThreads];
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < np; k += kThreads) s += part[k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] / (double)n;
}

// Adam (Kingma & Ba 2015) with bias correction, step >= 1
__global__ void __launch_bounds__(kThreads) k_adam(float *__restrict__ w, const float *__restrict__ g,
                                                   float *__restrict__ m, float *__restrict__ v, int64_t n, float lr,
                                                   float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---- BF16 matrix-core form of the convolution (cin % 8 == 0, cout % 16 == 0)
//
// Implicit GEMM: y[co][p] = b[co] + sum_k A[co][k] B[k][p] with k = (tap,
// input channel).  One v_mfma_f32_16x16x32_bf16 takes 16 output channels x 16
// voxels (consecutive along W) x 32 values of k: the four lane groups (lane /
// 16) take four consecutive entries q of the list of (tap, group of eight
// input channels) pairs, taps outer, eight channels each.  Lane l supplies
// row l % 16 of A and column l % 16 of B, and receives rows 4 (l / 16) + i of
// column l % 16 of the product (fixed by the instruction; the K order only has
// to be the same in A and B).  Inputs and weights are rounded to bfloat16
// (nearest, ties to even); products are accumulated in FP32.
//
// A workgroup takes a tile of 16 x kMTH x kMTD voxels (W x H x D) and up to
// NMT x 16 output channels; per pass over kMChunk input channels it stages the
// tile's halo in LDS as bfloat16, channels fastest, with a voxel stride of
// 2 * chunk + 16 bytes (so that the 16-byte reads of eight consecutive voxels
// fall in different banks); a lane's B operand is then one 16-byte LDS read.
// Voxels of the halo outside the volume hold 0 (zero padding).  Weights are
// packed beforehand (k_pack_mfma_weights) so that a lane's A operand is one
// 16-byte load.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kMTW = 16, kMTH = 4, kMTD = 2;  // tile (W x H x D): 8 rows of 16 voxels
constexpr int kMWaves = 4;                    // wavefronts per workgroup, two rows each
constexpr int kMRowsPerWave = kMTH * kMTD / kMWaves;
constexpr int kMHW = kMTW + 2, kMHH = kMTH + 2, kMHD = kMTD + 2;
constexpr int kMHalo = kMHW * kMHH * kMHD;  // 432 voxels
constexpr int kMChunk = 32;                 // input channels staged per pass
constexpr int kMStride = 2 * kMChunk + 16;  // bytes per halo voxel in LDS
constexpr int kMStage = 4;                  // staging tasks per thread with their loads in flight together

// float -> bfloat16, round to nearest, ties to even (NaN stays NaN)
__device__ __forceinline__ uint32_t bf16_rne(float f) {
  const uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// wp[(q * cout + co) * 8 + j] = bf16(w[co][8 c8 + j][t]) with q = t * (cin / 8) + c8
__global__ void __launch_bounds__(kThreads) k_pack_mfma_weights(const float *__restrict__ w, uint16_t *__restrict__ wp,
                                                                int cin, int cout) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t n = (int64_t)cin * cout * kTaps;
  if (i >= n) return;
  const int j = (int)(i % 8);
  const int64_t r = i / 8;
  const int co = (int)(r % cout);
  const int64_t q = r / cout;
  const int c8n = cin / 8;
  const int t = (int)(q / c8n), c8 = (int)(q % c8n);
  wp[i] = (uint16_t)bf16_rne(w[((int64_t)co * cin + 8 * c8 + j) * kTaps + t]);
}

template <int NMT>
__global__ void __launch_bounds__(kMWaves * 64) k_conv3d_mfma(const float *__restrict__ x,
                                                              const uint16_t *__restrict__ wp,
                                                              const float *__restrict__ b, float *__restrict__ y,
                                                              int cin, int cout, int D, int H, int W, int tiles_w,
                                                              int tiles_h) {
  __shared__ __attribute__((aligned(16))) unsigned char s_x[kMHalo * kMStride];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int g = lane >> 4, n = lane & 15;
  const int tile = blockIdx.x;
  const int w0 = (tile % tiles_w) * kMTW, h0 = ((tile / tiles_w) % tiles_h) * kMTH, d0 = tile / (tiles_w * tiles_h) * kMTD;
  const int co0 = blockIdx.y * NMT * 16;
  const int64_t V = (int64_t)D * H * W;
  f32x4 acc[NMT][kMRowsPerWave];
#pragma unroll
  for (int m = 0; m < NMT; ++m)
#pragma unroll
    for (int r = 0; r < kMRowsPerWave; ++r) acc[m][r] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int c0 = 0; c0 < cin; c0 += kMChunk) {
    const int c8n = (cin - c0 < kMChunk ? cin - c0 : kMChunk) / 8;
    // stage the halo: task (c8, hv), hv fastest; kMStage tasks per thread
    // at a time, all their loads issued before any store (a task past the
    // end loads task 0's voxels and stores nothing)
    const int ntask = c8n * kMHalo;
    for (int t0 = threadIdx.x; t0 < ntask; t0 += kMStage * kMWaves * 64) {
      float v[kMStage][8];
      bool in[kMStage];
#pragma unroll
      for (int u = 0; u < kMStage; ++u) {
        const int task = t0 + u * kMWaves * 64 < ntask ? t0 + u * kMWaves * 64 : 0;
        const int c8 = task / kMHalo, hv = task % kMHalo;
        const int hx = hv % kMHW, hy = (hv / kMHW) % kMHH, hz = hv / (kMHW * kMHH);
        const int xw = w0 + hx - 1, yh = h0 + hy - 1, zd = d0 + hz - 1;
        in[u] = xw >= 0 && xw < W && yh >= 0 && yh < H && zd >= 0 && zd < D;
        const float *xc = x + (int64_t)(c0 + 8 * c8) * V + (in[u] ? ((int64_t)zd * H + yh) * W + xw : 0);
#pragma unroll
        for (int j = 0; j < 8; ++j) v[u][j] = xc[j * V];
      }
#pragma unroll
      for (int u = 0; u < kMStage; ++u) {
        const int task = t0 + u * kMWaves * 64;
        if (task >= ntask) break;
        const int c8 = task / kMHalo, hv = task % kMHalo;
        u32x4 pk;
#pragma unroll
        for (int j = 0; j < 4; ++j)
          pk[j] = in[u] ? (bf16_rne(v[u][2 * j]) | (bf16_rne(v[u][2 * j + 1]) << 16)) : 0u;
        *reinterpret_cast<u32x4 *>(s_x + hv * kMStride + c8 * 16) = pk;
      }
    }
    __syncthreads();
    const int nq = kTaps * c8n;
    for (int q0 = 0; q0 < nq; q0 += 4) {
      const int q = q0 + g;
      const bool qv = q < nq;
      const int t = qv ? q / c8n : 0, c8 = qv ? q % c8n : 0;
      const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
      bf16x8 bfr[kMRowsPerWave];
#pragma unroll
      for (int r = 0; r < kMRowsPerWave; ++r) {
        const int row = wid * kMRowsPerWave + r, rh = row % kMTH, rd = row / kMTH;
        const int hv = ((rd + 1 + dz) * kMHH + (rh + 1 + dy)) * kMHW + (n + 1 + dx);
        bfr[r] = *reinterpret_cast<const bf16x8 *>(s_x + hv * kMStride + c8 * 16);
      }
      const int64_t kq = (int64_t)t * (cin / 8) + c0 / 8 + c8;  // (tap, channel group) in the packed weights
#pragma unroll
      for (int m = 0; m < NMT; ++m) {
        const int co = co0 + m * 16 + n;
        bf16x8 afr = {};
        if (qv && co < cout) afr = *reinterpret_cast<const bf16x8 *>(wp + (kq * cout + co) * 8);
#pragma unroll
        for (int r = 0; r < kMRowsPerWave; ++r)
          acc[m][r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, bfr[r], acc[m][r], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < kMRowsPerWave; ++r) {
    const int row = wid * kMRowsPerWave + r;
    const int xw = w0 + n, yh = h0 + row % kMTH, zd = d0 + row / kMTH;
    if (xw >= W || yh >= H || zd >= D) continue;
    const int64_t p = ((int64_t)zd * H + yh) * W + xw;
#pragma unroll
    for (int m = 0; m < NMT; ++m)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int co = co0 + m * 16 + 4 * g + i;
        if (co < cout) y[(int64_t)co * V + p] = acc[m][r][i] + (b ? b[co] : 0.0f);
      }
  }
}

// ---- BF16 matrix-core form of the weight gradient (cin % 16 == 0, cout % 16 == 0)
//
// Per tap t, dw[co][ci][t] = sum_p dy[co][p] x[ci][p + off(t)] is a product
// over the voxels p: one v_mfma_f32_16x16x32_bf16 takes 16 output channels
// (rows of A: dy) x 16 input channels (columns of B: x shifted by the tap) x
// the 32 voxels of one row segment along W, lane group g = lane / 16 taking
// voxels 8g .. 8g + 7 of the segment in both operands.  dy and x are rounded
// to bfloat16 (nearest, ties to even); products are accumulated in FP32.
//
// A workgroup takes one 16 x 16 channel tile and the voxel tiles s, s +
// nslab, ... (kGTW x kGTH x kGTD voxels: 8 rows of 32) of its slab s.  Per
// tile it stages in LDS the tile's dy (16 channels x 8 rows, bfloat16 pairs)
// and the halo of x (16 channels x 24 rows x 34 voxels), the latter as
// dwords holding the bfloat16 pair (x[w], x[w + 1]): the eight voxels that a
// lane needs at any shift along W are then four dwords at even distances
// (no alignment constraint).  Each wavefront takes every fourth tap for all
// rows, so its accumulators hold finished sums for the slab: it writes
// part[s][co][ci * 27 + t], the workgroups of channel tile 0 also the bias
// partial part[s][co][cin * 27] (FP32 sums of the unrounded dy), and
// k_wgrad_sum_ranges adds the slabs.
constexpr int kGTW = 32, kGTH = 4, kGTD = 2;
constexpr int kGRows = kGTH * kGTD;               // 8 rows of 32 voxels
constexpr int kGHH = kGTH + 2, kGHD = kGTD + 2;   // halo rows: 6 x 4
constexpr int kGHRows = kGHH * kGHD;              // 24
constexpr int kGHW = kGTW + 2;                    // halo voxels per row (34)
constexpr int kGPairs = kGTW + 1;                 // pair dwords per halo row (33)
constexpr int kGXCh = kGHRows * kGPairs + 1;      // dwords per channel (odd: channels in different banks)
constexpr int kGDyRow = kGTW / 2;                 // dwords per dy row (16)
constexpr int kGDyCh = kGRows * kGDyRow + 4;      // dwords per dy channel (16-byte aligned, banks spread)
constexpr int kGTapsPerWave = (kTaps + kMWaves - 1) / kMWaves;
constexpr int kGStageDy = 16 * kGRows * kGDyRow / (kMWaves * 64);  // dy pairs per thread and tile (8)
static_assert(16 * kGRows * kGDyRow % (kMWaves * 64) == 0, "dy staging must split evenly");
constexpr int kGStageX = 16 * kGHRows * kGHW / (kMWaves * 64);  // x halo values per thread and tile (51)
constexpr int kGXBatch = 17;
static_assert(16 * kGHRows * kGHW % (kMWaves * 64) == 0 && kGStageX % kGXBatch == 0, "x staging must split evenly");
static_assert(kMWaves * 64 / (kGRows * kGDyRow) * kGStageDy == 16, "dy staging: channels per thread");

__global__ void __launch_bounds__(kMWaves * 64) k_wgrad_mfma(const float *__restrict__ x, const float *__restrict__ dy,
                                                             float *__restrict__ part, int cin, int cout, int D,
                                                             int H, int W, int tiles_w, int tiles_h, int64_t ntiles) {
  __shared__ __attribute__((aligned(16))) uint32_t s_x[16 * kGXCh];
  __shared__ __attribute__((aligned(16))) uint32_t s_dy[16 * kGDyCh];
  __shared__ float s_red[kMWaves][kGStageDy];
  const int lane = threadIdx.x & 63, wid = uniform((int)(threadIdx.x >> 6));
  const int g = lane >> 4, n = lane & 15;
  const int64_t slab = blockIdx.x, nslab = gridDim.x;
  const int co0 = blockIdx.y * 16, ci0 = blockIdx.z * 16;
  const int64_t V = (int64_t)D * H * W;
  const bool bias = blockIdx.z == 0;
  uint16_t *s_x16 = reinterpret_cast<uint16_t *>(s_x);
  f32x4 acc[kGTapsPerWave];
#pragma unroll
  for (int m = 0; m < kGTapsPerWave; ++m) acc[m] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  float bsum[kGStageDy];
#pragma unroll
  for (int k = 0; k < kGStageDy; ++k) bsum[k] = 0.0f;
  for (int64_t tile = slab; tile < ntiles; tile += nslab) {
    const int w0 = (int)(tile % tiles_w) * kGTW, h0 = (int)((tile / tiles_w) % tiles_h) * kGTH;
    const int d0 = (int)(tile / ((int64_t)tiles_w * tiles_h)) * kGTD;
    // x halo: value (c, halo row, hw) -> low half of pair hw and high half of
    // pair hw - 1; loads in batches of kGXBatch so that they are in flight
    // together (every lane loads a voxel of the volume, padding then becomes
    // 0: no branch between the loads)
#pragma unroll 1
    for (int k0 = 0; k0 < kGStageX; k0 += kGXBatch) {
      float v[kGXBatch];
#pragma unroll
      for (int u = 0; u < kGXBatch; ++u) {
        const int task = threadIdx.x + (k0 + u) * kMWaves * 64;
        const int c = task / (kGHRows * kGHW), rem = task % (kGHRows * kGHW);
        const int hr = rem / kGHW, hw = rem % kGHW;
        const int zd = d0 + hr / kGHH - 1, yh = h0 + hr % kGHH - 1, xw = w0 + hw - 1;
        const bool in = zd >= 0 && zd < D && yh >= 0 && yh < H && xw >= 0 && xw < W;
        const int zc = min(max(zd, 0), D - 1), yc = min(max(yh, 0), H - 1), xc = min(max(xw, 0), W - 1);
        const float lv = x[(int64_t)(ci0 + c) * V + ((int64_t)zc * H + yc) * W + xc];
        v[u] = in ? lv : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < kGXBatch; ++u) {
        const int task = threadIdx.x + (k0 + u) * kMWaves * 64;
        const int c = task / (kGHRows * kGHW), rem = task % (kGHRows * kGHW);
        const int hr = rem / kGHW, hw = rem % kGHW;
        const uint16_t b = (uint16_t)bf16_rne(v[u]);
        const int base = c * kGXCh + hr * kGPairs;
        if (hw < kGPairs) s_x16[2 * (base + hw)] = b;
        if (hw > 0) s_x16[2 * (base + hw - 1) + 1] = b;
      }
    }
    // dy: pairs of voxels (c, row, 2j .. 2j + 1); thread k-th task: channel 2k + (tid >= 128)
    float dv[kGStageDy][2];
#pragma unroll
    for (int k = 0; k < kGStageDy; ++k) {
      const int task = threadIdx.x + k * kMWaves * 64;
      const int c = task / (kGRows * kGDyRow), rem = task % (kGRows * kGDyRow);
      const int r = rem / kGDyRow, j = rem % kGDyRow;
      const int zd = d0 + r / kGTH, yh = h0 + r % kGTH, xw = w0 + 2 * j;
      const bool row_in = zd < D && yh < H;
      const int64_t rowp = (int64_t)(co0 + c) * V + ((int64_t)min(zd, D - 1) * H + min(yh, H - 1)) * W;
      const float l0 = dy[rowp + min(xw, W - 1)], l1 = dy[rowp + min(xw + 1, W - 1)];
      dv[k][0] = (row_in && xw < W) ? l0 : 0.0f;
      dv[k][1] = (row_in && xw + 1 < W) ? l1 : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < kGStageDy; ++k) {
      const int task = threadIdx.x + k * kMWaves * 64;
      const int c = task / (kGRows * kGDyRow), rem = task % (kGRows * kGDyRow);
      bsum[k] += dv[k][0] + dv[k][1];
      s_dy[c * kGDyCh + rem] = bf16_rne(dv[k][0]) | (bf16_rne(dv[k][1]) << 16);
    }
    __syncthreads();
#pragma unroll 2
    for (int r = 0; r < kGRows; ++r) {
      const bf16x8 afr = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4 *>(s_dy + n * kGDyCh + r * kGDyRow + 4 * g));
      const int rh = r % kGTH, rd = r / kGTH;
#pragma unroll
      for (int m = 0; m < kGTapsPerWave; ++m) {
        // the last wavefront has one tap fewer: it repeats tap 26 into an
        // accumulator it never writes out (no branch in the loop)
        const int t = min(wid + kMWaves * m, kTaps - 1);
        const int dz = t / 9 - 1, dyy = (t / 3) % 3 - 1, dx = t % 3 - 1;
        const int hr = (rd + 1 + dz) * kGHH + (rh + 1 + dyy);
        const uint32_t *q = s_x + n * kGXCh + hr * kGPairs + 8 * g + dx + 1;
        const u32x4 bw = {q[0], q[2], q[4], q[6]};
        acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr, __builtin_bit_cast(bf16x8, bw), acc[m], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  const int64_t stride = (int64_t)cin * kTaps + 1;
#pragma unroll
  for (int m = 0; m < kGTapsPerWave; ++m) {
    const int t = wid + kMWaves * m;
    if (t >= kTaps) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      part[(slab * cout + co0 + 4 * g + i) * stride + (int64_t)(ci0 + n) * kTaps + t] = acc[m][i];
  }
  if (bias) {
#pragma unroll
    for (int k = 0; k < kGStageDy; ++k) {
      const float sw = wave_total(bsum[k]);
      if (lane == 0) s_red[wid][k] = sw;
    }
    __syncthreads();
    if (threadIdx.x < 16) {
      // channel c = 2k + h is held by wavefronts 2h and 2h + 1
      const int c = threadIdx.x, k = c >> 1, h = c & 1;
      part[(slab * cout + co0 + c) * stride + (int64_t)cin * kTaps] = s_red[2 * h][k] + s_red[2 * h + 1][k];
    }
  }
}

static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

hipError_t conv3d(const float *x, const float *w, const float *b, float *y, int cin, int cout, int D, int H, int W,
                  hipStream_t s) {
  const int64_t V = (int64_t)D * H * W;
  if (V <= 0 || cout <= 0) return hipSuccess;
  if (cout >= 16) {
    hipLaunchKernelGGL(k_conv3d<16>, dim3(blocks_for(V), (unsigned)((cout + 15) / 16)), dim3(kThreads), 0, s, x, w,
                       b, y, cin, cout, D, H, W);
  } else if (cout >= 4) {
    hipLaunchKernelGGL(k_conv3d<4>, dim3(blocks_for(V), (unsigned)((cout + 3) / 4)), dim3(kThreads), 0, s, x, w, b,
                       y, cin, cout, D, H, W);
  } else {
    hipLaunchKernelGGL(k_conv3d<1>, dim3(blocks_for(V), (unsigned)cout), dim3(kThreads), 0, s, x, w, b, y, cin, cout,
                       D, H, W);
  }
  return hipGetLastError();
}

bool mfma_shape_ok(int cin, int cout) { return cin > 0 && cout > 0 && cin % 8 == 0 && cout % 16 == 0; }

int64_t mfma_pack_bytes(int cin, int cout) { return (int64_t)cin * cout * kTaps * 2; }

hipError_t conv3d_mfma(const float *x, const float *w, const float *b, float *y, void *wpack, int cin, int cout,
                       int D, int H, int W, hipStream_t s) {
  const int64_t V = (int64_t)D * H * W;
  if (V <= 0) return hipSuccess;
  uint16_t *wp = static_cast<uint16_t *>(wpack);
  const int64_t nw = (int64_t)cin * cout * kTaps;
  hipLaunchKernelGGL(k_pack_mfma_weights, dim3(blocks_for(nw)), dim3(kThreads), 0, s, w, wp, cin, cout);
  const int tw = (W + kMTW - 1) / kMTW, th = (H + kMTH - 1) / kMTH, td = (D + kMTD - 1) / kMTD;
  const unsigned tiles = (unsigned)((int64_t)tw * th * td);
  const int mt = cout / 16;
  if (mt % 4 == 0)
    hipLaunchKernelGGL(k_conv3d_mfma<4>, dim3(tiles, (unsigned)(mt / 4)), dim3(kMWaves * 64), 0, s, x, wp, b, y, cin,
                       cout, D, H, W, tw, th);
  else if (mt % 2 == 0)
    hipLaunchKernelGGL(k_conv3d_mfma<2>, dim3(tiles, (unsigned)(mt / 2)), dim3(kMWaves * 64), 0, s, x, wp, b, y, cin,
                       cout, D, H, W, tw, th);
  else
    hipLaunchKernelGGL(k_conv3d_mfma<1>, dim3(tiles, (unsigned)mt), dim3(kMWaves * 64), 0, s, x, wp, b, y, cin, cout,
                       D, H, W, tw, th);
  return hipGetLastError();
}

hipError_t flip_weights(const float *w, float *wt, int cin, int cout, hipStream_t s) {
  const int64_t n = (int64_t)cin * cout * kTaps;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_flip, dim3(blocks_for(n)), dim3(kThreads), 0, s, w, wt, cin, cout);
  return hipGetLastError();
}

static inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
constexpr int64_t kWgradTargetWgs = 2048;  // workgroups wanted per weight-gradient launch

int64_t wgrad_chunks(int D, int H, int W) {
  return (int64_t)ceil_div(W, 64) * ceil_div(H, kTileY) * ceil_div(D, kTileZ);
}

hipError_t conv3d_wgrad(const float *x, const float *dy, float *dw, float *db, float *part, int cin, int cout, int D,
                        int H, int W, hipStream_t s) {
  const int64_t chunks = wgrad_chunks(D, H, W);
  if (chunks <= 0 || cout <= 0) return hipSuccess;
  const int tx = ceil_div(W, 64), ty = ceil_div(H, kTileY);
  const int64_t wgs = chunks * ceil_div(cout, kWgCob);
  const int splits = (int)std::min<int64_t>(cin, std::max<int64_t>(1, (kWgradTargetWgs + wgs - 1) / wgs));
  const int ci_per = ceil_div(cin, splits);
  hipLaunchKernelGGL(k_wgrad_part, dim3((unsigned)chunks, (unsigned)ceil_div(cout, kWgCob), (unsigned)ceil_div(cin, ci_per)),
                     dim3(kThreads), 0, s, x, dy, part, cin, cout, D, H, W, tx, ty, ci_per);
  const int64_t n = (int64_t)cout * ((int64_t)cin * kTaps + 1);
  hipLaunchKernelGGL(k_wgrad_sum, dim3(blocks_for(n)), dim3(kThreads), 0, s, part, dw, db, chunks, cin, cout);
  return hipGetLastError();
}

// stage 2 of the matrix-core form: element i of the cout x (cin * 27 + 1)
// gradient summed over the slabs in kSumWaves contiguous ranges (one
// wavefront each, slabs in order), the ranges then added in order
constexpr int kSumWaves = 16;
__global__ void __launch_bounds__(kSumWaves * 64) k_wgrad_sum_ranges(const float *__restrict__ part,
                                                                     float *__restrict__ dw, float *__restrict__ db,
                                                                     int64_t chunks, int cin, int cout) {
  __shared__ float red[kSumWaves][64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t stride = (int64_t)cin * kTaps + 1, nout = (int64_t)cout * stride;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const int64_t g0 = chunks * wid / kSumWaves, g1 = chunks * (wid + 1) / kSumWaves;
  float s = 0.0f;
  if (i < nout)
    for (int64_t g = g0; g < g1; ++g) s += part[g * nout + i];
  red[wid][lane] = s;
  __syncthreads();
  if (wid == 0 && i < nout) {
    float t = 0.0f;
    for (int w = 0; w < kSumWaves; ++w) t += red[w][lane];
    const int64_t co = i / stride, j = i % stride;
    if (j < (int64_t)cin * kTaps)
      dw[co * cin * kTaps + j] = t;
    else if (db)
      db[co] = t;
  }
}

bool mfma_wgrad_ok(int cin, int cout) { return cin > 0 && cout > 0 && cin % 16 == 0 && cout % 16 == 0; }

constexpr int64_t kGTargetWgs = 1024;  // workgroups wanted per matrix-core weight-gradient launch

int64_t wgrad_mfma_slabs(int cin, int cout, int D, int H, int W) {
  const int64_t tiles = (int64_t)ceil_div(W, kGTW) * ceil_div(H, kGTH) * ceil_div(D, kGTD);
  const int64_t per = (int64_t)(cout / 16) * (cin / 16);
  if (tiles <= 0 || per <= 0) return 0;
  return std::max<int64_t>(1, std::min<int64_t>(tiles, (kGTargetWgs + per - 1) / per));
}

hipError_t conv3d_wgrad_mfma(const float *x, const float *dy, float *dw, float *db, float *part, int cin, int cout,
                             int D, int H, int W, hipStream_t s) {
  const int64_t nslab = wgrad_mfma_slabs(cin, cout, D, H, W);
  if (nslab <= 0) return hipSuccess;
  const int tw = ceil_div(W, kGTW), th = ceil_div(H, kGTH);
  const int64_t ntiles = (int64_t)tw * th * ceil_div(D, kGTD);
  hipLaunchKernelGGL(k_wgrad_mfma, dim3((unsigned)nslab, (unsigned)(cout / 16), (unsigned)(cin / 16)),
                     dim3(kMWaves * 64), 0, s, x, dy, part, cin, cout, D, H, W, tw, th, ntiles);
  const int64_t n = (int64_t)cout * ((int64_t)cin * kTaps + 1);
  hipLaunchKernelGGL(k_wgrad_sum_ranges, dim3((unsigned)((n + 63) / 64)), dim3(kSumWaves * 64), 0, s, part, dw, db,
                     nslab, cin, cout);
  return hipGetLastError();
}

hipError_t relu(const float *x, float *y, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_relu, dim3(blocks_for(n)), dim3(kThreads), 0, s, x, y, n);
  return hipGetLastError();
}

hipError_t relu_bwd(const float *y, const float *dy, float *dx, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_relu_bwd, dim3(blocks_for(n)), dim3(kThreads), 0, s, y, dy, dx, n);
  return hipGetLastError();
}

hipError_t pool(const float *x, float *y, int C, int D, int H, int W, hipStream_t s) {
  const int64_t n = (int64_t)C * (D / 2) * (H / 2) * (W / 2);
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pool, dim3(blocks_for(n)), dim3(kThreads), 0, s, x, y, C, D, H, W);
  return hipGetLastError();
}

hipError_t pool_bwd(const float *dy, float *dx, int C, int D, int H, int W, hipStream_t s) {
  const int64_t n = (int64_t)C * D * H * W;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pool_bwd, dim3(blocks_for(n)), dim3(kThreads), 0, s, dy, dx, C, D, H, W);
  return hipGetLastError();
}

hipError_t upsample(const float *x, float *y, int C, int d, int h, int w, hipStream_t s) {
  const int64_t n = (int64_t)C * 8 * d * h * w;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_up, dim3(blocks_for(n)), dim3(kThreads), 0, s, x, y, C, d, h, w);
  return hipGetLastError();
}

hipError_t upsample_bwd(const float *dy, float *dx, int C, int d, int h, int w, hipStream_t s) {
  const int64_t n = (int64_t)C * d * h * w;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_up_bwd, dim3(blocks_for(n)), dim3(kThreads), 0, s, dy, dx, C, d, h, w);
  return hipGetLastError();
}

hipError_t add(const float *a, const float *b, float *y, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_add, dim3(blocks_for(n)), dim3(kThreads), 0, s, a, b, y, n);
  return hipGetLastError();
}

hipError_t axpy(float a, const float *x, float *y, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy, dim3(blocks_for(n)), dim3(kThreads), 0, s, a, x, y, n);
  return hipGetLastError();
}

hipError_t mask(const float *x, const uint8_t *m, float *y, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mask, dim3(blocks_for(n)), dim3(kThreads), 0, s, x, m, y, n);
  return hipGetLastError();
}

int64_t mse_parts(int64_t n) { return (n + kThreads - 1) / kThreads; }

hipError_t mse(const float *y, const float *t, float *dy, double *part, double *loss, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t np = mse_parts(n);
  hipLaunchKernelGGL(k_mse, dim3((unsigned)np), dim3(kThreads), 0, s, y, t, dy, part, n);
  hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(kThreads), 0, s, part, np, n, loss);
  return hipGetLastError();
}

hipError_t adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float eps,
                int step, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(n)), dim3(kThreads), 0, s, w, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace cnn
}  // namespace pct
