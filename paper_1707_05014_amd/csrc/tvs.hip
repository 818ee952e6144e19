// Total-variation superiorization (paper Sec. 4.2, the Table 2 discussion:
// both pipelines perturb the image towards lower total variation; DROP does
// it to the image entering every block, CARP once per iteration) and the
// space-carving hull.
//
// TV(x) = sum_v sqrt(dx_v^2 + dy_v^2 + dz_v^2 + eps^2), forward differences
// (0 at the grid's last plane on an axis).  One superiorization step:
// g = dTV/dx (0 outside the mask), then trials z = x - beta g / ||g||,
// beta <- a beta after every trial, the first z with TV(z) <= TV(x) kept,
// at most max_trials trials.  The step size, the running TV and the
// accept decision live in a small device state array, so a step runs as a
// fixed sequence of launches without host synchronisation; kernels of a
// decided step return at once.  TV sums are FP64 with fixed-order
// reductions (per-workgroup partials, then one ordered sum).
#include <hip/hip_runtime.h>

#include "pct_internal.h"

namespace pct {

namespace {

constexpr int kTvBlock = 256;

// state slots (device double[8])
enum { S_BETA = 0, S_TVX = 1, S_GNORM = 2, S_ACCEPTED = 3, S_BETA_ACC = 4, S_N_ACC = 5, S_STOP = 6 };

struct Dims {
  int32_t nx, ny, nz;
  int64_t M;
};

__device__ __forceinline__ double xval(const float *x, int64_t v) { return (double)x[v]; }

// smoothed TV term of voxel (i, j, k) of image f (a functor of the voxel index)
template <typename F>
__device__ __forceinline__ double tv_phi(const Dims &d, F f, int i, int j, int k, double eps, double &dx, double &dy,
                                         double &dz) {
  const int64_t v = ((int64_t)k * d.ny + j) * d.nx + i;
  const double c = f(v);
  dx = (i + 1 < d.nx) ? f(v + 1) - c : 0.0;
  dy = (j + 1 < d.ny) ? f(v + d.nx) - c : 0.0;
  dz = (k + 1 < d.nz) ? f(v + (int64_t)d.nx * d.ny) - c : 0.0;
  return sqrt(dx * dx + dy * dy + dz * dz + eps * eps);
}

__device__ __forceinline__ double block_sum(double v, double *red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = kTvBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  return red[0];
}

__device__ __forceinline__ bool step_done(const double *st) { return st[S_STOP] != 0.0 || st[S_ACCEPTED] != 0.0; }

// g = dTV/dx (masked), per-workgroup partial sums of TV(x) and of g^2
__global__ void __launch_bounds__(kTvBlock) k_tv_grad(Dims d, const float *__restrict__ x,
                                                      const uint8_t *__restrict__ mask, double eps, float *g,
                                                      double *part_tv, double *part_g2, const double *st) {
  __shared__ double red[kTvBlock];
  const int64_t u = (int64_t)blockIdx.x * kTvBlock + threadIdx.x;
  double tv = 0.0, g2 = 0.0;
  const bool live = st[S_STOP] == 0.0;
  if (live && u < d.M) {
    const int i = (int)(u % d.nx), j = (int)((u / d.nx) % d.ny), k = (int)(u / ((int64_t)d.nx * d.ny));
    auto f = [&](int64_t v) { return xval(x, v); };
    double dx, dy, dz;
    const double phi = tv_phi(d, f, i, j, k, eps, dx, dy, dz);
    tv = phi;
    double gu = -(dx + dy + dz) / phi;
    if (i > 0) {
      double a, b, c;
      const double p = tv_phi(d, f, i - 1, j, k, eps, a, b, c);
      gu += a / p;
    }
    if (j > 0) {
      double a, b, c;
      const double p = tv_phi(d, f, i, j - 1, k, eps, a, b, c);
      gu += b / p;
    }
    if (k > 0) {
      double a, b, c;
      const double p = tv_phi(d, f, i, j, k - 1, eps, a, b, c);
      gu += c / p;
    }
    if (mask && !mask[u]) gu = 0.0;
    g[u] = (float)gu;
    g2 = (double)(float)gu * (double)(float)gu;
  }
  const double s_tv = block_sum(tv, red);
  __syncthreads();
  const double s_g2 = block_sum(g2, red);
  if (threadIdx.x == 0) {
    part_tv[blockIdx.x] = s_tv;
    part_g2[blockIdx.x] = s_g2;
  }
}

// per-workgroup partial sums of TV(z), z = x - beta g / ||g|| (the trial)
__global__ void __launch_bounds__(kTvBlock) k_tv_trial(Dims d, const float *__restrict__ x,
                                                       const float *__restrict__ g, double eps, double *part_tv,
                                                       const double *st) {
  __shared__ double red[kTvBlock];
  if (step_done(st)) return;   // uniform over the grid: the step is decided
  const double scale = st[S_BETA] / st[S_GNORM];
  const int64_t u = (int64_t)blockIdx.x * kTvBlock + threadIdx.x;
  double tv = 0.0;
  if (u < d.M) {
    const int i = (int)(u % d.nx), j = (int)((u / d.nx) % d.ny), k = (int)(u / ((int64_t)d.nx * d.ny));
    auto f = [&](int64_t v) { return (double)x[v] - scale * (double)g[v]; };
    double dx, dy, dz;
    tv = tv_phi(d, f, i, j, k, eps, dx, dy, dz);
  }
  const double s = block_sum(tv, red);
  if (threadIdx.x == 0) part_tv[blockIdx.x] = s;
}

// ordered sums of the partials.  mode 0 (after k_tv_grad): TV(x), ||g||,
// clear the step's decision (stop when g = 0); mode 1 (after a trial): keep
// beta if TV(z) <= TV(x), then beta <- a beta
__global__ void __launch_bounds__(kTvBlock) k_tv_reduce(const double *part_a, const double *part_b, int64_t np,
                                                        double a, double *st, int mode) {
  __shared__ double red[kTvBlock];
  if (mode == 1 && step_done(st)) return;
  if (mode == 0 && st[S_STOP] != 0.0) return;
  double sa = 0.0, sb = 0.0;
  for (int64_t q = threadIdx.x; q < np; q += kTvBlock) {
    sa += part_a[q];
    if (mode == 0) sb += part_b[q];
  }
  const double ta = block_sum(sa, red);
  __syncthreads();
  const double tb = mode == 0 ? block_sum(sb, red) : 0.0;
  if (threadIdx.x != 0) return;
  if (mode == 0) {
    st[S_TVX] = ta;
    st[S_GNORM] = sqrt(tb);
    st[S_ACCEPTED] = 0.0;
    if (!(st[S_GNORM] > 0.0)) st[S_STOP] = 1.0;
  } else {
    const double beta = st[S_BETA];
    st[S_BETA] = beta * a;
    if (ta <= st[S_TVX]) {
      st[S_ACCEPTED] = 1.0;
      st[S_BETA_ACC] = beta;
      st[S_N_ACC] += 1.0;
    }
  }
}

// x <- x - beta_acc g / ||g|| when the step kept a trial
__global__ void __launch_bounds__(kTvBlock) k_tv_apply(int64_t M, float *x, const float *__restrict__ g,
                                                       const double *st) {
  if (st[S_STOP] != 0.0 || st[S_ACCEPTED] == 0.0) return;
  const double scale = st[S_BETA_ACC] / st[S_GNORM];
  const int64_t u = (int64_t)blockIdx.x * kTvBlock + threadIdx.x;
  if (u < M) x[u] = (float)((double)x[u] - scale * (double)g[u]);
}

__global__ void k_tv_begin(double *st) {
  if (threadIdx.x == 0) st[S_STOP] = 0.0;
}

// Space carving: one thread per history.  A history with finite values and
// WEPL below wepl_max crossed only air; its straight entry line from u_in to
// u_out is cut at every voxel plane it crosses, the crossing parameters
// (plane - p) / (q - p) taken in increasing order over the three axes (grid
// units, FP64), and every sub-interval longer than min_len mm whose midpoint
// lies in the grid marks that voxel carved (hull[j] = 0).
__global__ void __launch_bounds__(256) k_carve(PathParams P, HistPtrs H, int64_t n, double wepl_max, double min_len,
                                               uint8_t *hull, unsigned long long *used) {
  unsigned long long cnt = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += stride) {
    const float h[10] = {H.phi[q], H.t_in[q], H.v_in[q], H.dt_in[q], H.dv_in[q],
                         H.t_out[q], H.v_out[q], H.dt_out[q], H.dv_out[q], H.wepl[q]};
    bool fin = true;
    for (int f = 0; f < 10; ++f) fin = fin && isfinite(h[f]);
    if (!fin || !((double)h[9] < wepl_max)) continue;
    ++cnt;
    const double phi = h[0], c = cos(phi), s = sin(phi);
    const double u0 = P.u_in, u1 = P.u_out;
    const double t0 = h[1], v0 = h[2], t1 = (double)h[1] + (double)h[3] * (u1 - u0),
                 v1 = (double)h[2] + (double)h[4] * (u1 - u0);
    const double Pw[3] = {u0 * c - t0 * s, u0 * s + t0 * c, v0};
    const double Qw[3] = {u1 * c - t1 * s, u1 * s + t1 * c, v1};
    const double o[3] = {P.ox, P.oy, P.oz}, dd[3] = {P.dx, P.dy, P.dz};
    const int nn[3] = {P.nx, P.ny, P.nz};
    double gp[3], gq[3];
    for (int a = 0; a < 3; ++a) {
      gp[a] = (Pw[a] - o[a]) / dd[a];
      gq[a] = (Qw[a] - o[a]) / dd[a];
    }
    const double ex = Qw[0] - Pw[0], ey = Qw[1] - Pw[1], ez = Qw[2] - Pw[2];
    const double seg = sqrt(ex * ex + ey * ey + ez * ez);
    if (!(seg > 0.0)) continue;
    // next plane per axis (integers strictly between the end coordinates),
    // walked in the direction of travel; alpha = (plane - p) / (q - p)
    double nxt[3], stepd[3], last[3];
    for (int a = 0; a < 3; ++a) {
      if (gq[a] > gp[a]) {
        nxt[a] = floor(gp[a]) + 1.0;
        stepd[a] = 1.0;
        last[a] = gq[a];
      } else if (gq[a] < gp[a]) {
        nxt[a] = ceil(gp[a]) - 1.0;
        stepd[a] = -1.0;
        last[a] = gq[a];
      } else {
        nxt[a] = 0.0;
        stepd[a] = 0.0;
        last[a] = 0.0;
      }
    }
    auto alpha_of = [&](int a) -> double {
      if (stepd[a] == 0.0) return 2.0;
      const bool ok = stepd[a] > 0.0 ? nxt[a] < last[a] : nxt[a] > last[a];
      return ok ? (nxt[a] - gp[a]) / (gq[a] - gp[a]) : 2.0;
    };
    double al[3] = {alpha_of(0), alpha_of(1), alpha_of(2)};
    double a0 = 0.0;
    const int max_iter = 4 * (nn[0] + nn[1] + nn[2]) + 64;
    for (int it = 0; it < max_iter; ++it) {
      int ax = 0;
      if (al[1] < al[ax]) ax = 1;
      if (al[2] < al[ax]) ax = 2;
      const double a1 = al[ax] < 1.0 ? al[ax] : 1.0;
      if (a1 > a0) {
        const double am = 0.5 * (a0 + a1);
        int iv[3];
        bool inside = true;
        for (int a = 0; a < 3; ++a) {
          const double cc = floor(gp[a] + am * (gq[a] - gp[a]));
          if (cc < 0.0 || cc >= (double)nn[a]) inside = false;
          iv[a] = (int)cc;
        }
        if (inside && (a1 - a0) * seg > min_len) {
          const int64_t j = ((int64_t)iv[2] * nn[1] + iv[1]) * nn[0] + iv[0];
          hull[j] = 0;
        }
      }
      if (a1 >= 1.0) break;
      a0 = a1;
      nxt[ax] += stepd[ax];
      al[ax] = alpha_of(ax);
    }
  }
  if (cnt) atomicAdd(used, cnt);
}

}  // namespace

size_t tvs_scratch_bytes(int64_t M) {
  const int64_t np = (M + kTvBlock - 1) / kTvBlock;
  return ((size_t)M * 4 + 255) / 256 * 256 + ((size_t)np * 16 + 255) / 256 * 256;
}

// n_steps superiorization steps of x (see the file comment); scratch of
// tvs_scratch_bytes(M); state: device double[8]
hipError_t launch_tvs(int32_t nx, int32_t ny, int32_t nz, float *x, const uint8_t *mask, int32_t n_steps,
                      int32_t max_trials, double a, double eps, double *state, void *scratch, hipStream_t s) {
  Dims d{nx, ny, nz, (int64_t)nx * ny * nz};
  if (d.M == 0 || n_steps <= 0) return hipSuccess;
  const int64_t np = (d.M + kTvBlock - 1) / kTvBlock;
  char *p = static_cast<char *>(scratch);
  float *g = reinterpret_cast<float *>(p);
  double *part_a = reinterpret_cast<double *>(p + ((size_t)d.M * 4 + 255) / 256 * 256);
  double *part_b = part_a + np;
  const dim3 grid((unsigned)np), blk(kTvBlock);
  hipLaunchKernelGGL(k_tv_begin, dim3(1), dim3(64), 0, s, state);
  for (int st = 0; st < n_steps; ++st) {
    hipLaunchKernelGGL(k_tv_grad, grid, blk, 0, s, d, x, mask, eps, g, part_a, part_b, state);
    hipLaunchKernelGGL(k_tv_reduce, dim3(1), blk, 0, s, part_a, part_b, np, a, state, 0);
    for (int t = 0; t < max_trials; ++t) {
      hipLaunchKernelGGL(k_tv_trial, grid, blk, 0, s, d, x, g, eps, part_a, state);
      hipLaunchKernelGGL(k_tv_reduce, dim3(1), blk, 0, s, part_a, part_b, np, a, state, 1);
    }
    hipLaunchKernelGGL(k_tv_apply, grid, blk, 0, s, d.M, x, g, state);
  }
  return hipGetLastError();
}

hipError_t launch_carve(const PathParams &P, const HistPtrs &H, int64_t n, double wepl_max, double min_len,
                        uint8_t *hull, unsigned long long *used, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + 255) / 256;
  if (g > 16384) g = 16384;
  hipLaunchKernelGGL(k_carve, dim3((unsigned)g), dim3(256), 0, s, P, H, n, wepl_max, min_len, hull, used);
  return hipGetLastError();
}

}  // namespace pct
