/*
 * Seeded synthetic proton histories generated on the GPU (input data only).
 *
 * The same histories as gen.c, produced where they are used: one thread per
 * history, the same Philox4x32-10 counter stream (key = seed, counter =
 * (draw, attempt, proton); Salmon, Moraes, Dror, Shaw, SC 2011), the same
 * FP64 transport through the analytic phantom (Fermi-Eyges Gaussian kicks per
 * step, Bragg-Kleeman energy at the water-equivalent depth reached, Highland
 * factor from the straight entry chord), the same rejection of entry lines
 * that miss the body.  Integer draws are identical to gen.c's; the FP64
 * results differ from the host's only through the device's last-bit
 * differences in sqrt/log/pow/sin/cos, so almost every float32 output is
 * bit-identical.  Like gen.c it holds none of the reconstruction's
 * arithmetic.
 */
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace {

constexpr int kMaxShapes = 16;

struct Shape {   // as pctgen_shape in gen.c (cy, sy filled in on the host)
  int32_t kind;
  double c[3];
  double ax[3];
  double yaw;
  double z0, z1;
  double delta_rsp;
  double bound_r;
  double cy, sy;
};

struct Params {  // as pctgen_params in gen.c
  int32_t n_angles;
  double t_half, v_half;
  double slope_sigma;
  double u_in, u_out;
  double step;
  double E_kin;
  double bk_alpha, bk_p;
  double m_p;
  double E0_hl, X0;
  int32_t highland_log;
  int32_t scatter;
  double wepl_sigma;
  double body_rxy;
};

struct Scene {
  Params p;
  int32_t n_shapes;
  Shape s[kMaxShapes];
};

struct Out {
  float *f[10];
};

__device__ __forceinline__ void philox(const uint32_t ctr[4], uint32_t k0, uint32_t k1, uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

struct Rng {
  uint32_t k0, k1;
  uint32_t ctr[4];
  uint32_t buf[4];
  int left;
  __device__ Rng(uint64_t seed, uint64_t proton, uint32_t attempt) {
    k0 = (uint32_t)seed;
    k1 = (uint32_t)(seed >> 32);
    ctr[0] = 0;
    ctr[1] = attempt;
    ctr[2] = (uint32_t)proton;
    ctr[3] = (uint32_t)(proton >> 32);
    left = 0;
  }
  __device__ uint32_t u32() {
    if (left == 0) {
      philox(ctr, k0, k1, buf);
      ctr[0]++;
      left = 4;
    }
    const int k = 4 - (left--);
    return k == 0 ? buf[0] : (k == 1 ? buf[1] : (k == 2 ? buf[2] : buf[3]));
  }
  __device__ double uniform() {  // (0, 1), 53 random bits
    const uint64_t a = u32() >> 5, b = u32() >> 6;
    return ((double)(a * 67108864u + b) + 0.5) / 9007199254740992.0;
  }
  __device__ void normal2(double &z0, double &z1) {
    const double u1 = uniform(), u2 = uniform();
    const double rad = sqrt(-2.0 * log(u1));
    z0 = rad * cos(2.0 * M_PI * u2);
    z1 = rad * sin(2.0 * M_PI * u2);
  }
};

__device__ bool shape_interval(const Shape &sh, const double P[3], const double D[3], double &s0, double &s1) {
  const double cs = sh.cy, sn = sh.sy;
  const double px = P[0] - sh.c[0], py = P[1] - sh.c[1], pz = P[2] - sh.c[2];
  const double lx = cs * px + sn * py, ly = -sn * px + cs * py;
  const double dx = cs * D[0] + sn * D[1], dy = -sn * D[0] + cs * D[1], dz = D[2];
  double lo = -INFINITY, hi = INFINITY;
  double A, B, C;
  if (sh.kind == 0) {
    const double ia = 1.0 / sh.ax[0], ib = 1.0 / sh.ax[1], ic = 1.0 / sh.ax[2];
    const double qx = lx * ia, qy = ly * ib, qz = pz * ic;
    const double ex = dx * ia, ey = dy * ib, ez = dz * ic;
    A = ex * ex + ey * ey + ez * ez;
    B = 2.0 * (qx * ex + qy * ey + qz * ez);
    C = qx * qx + qy * qy + qz * qz - 1.0;
  } else {
    const double ia = 1.0 / sh.ax[0], ib = 1.0 / sh.ax[1];
    const double qx = lx * ia, qy = ly * ib;
    const double ex = dx * ia, ey = dy * ib;
    A = ex * ex + ey * ey;
    B = 2.0 * (qx * ex + qy * ey);
    C = qx * qx + qy * qy - 1.0;
    const double zp = P[2];
    if (fabs(dz) < 1e-300) {
      if (zp < sh.z0 || zp > sh.z1) return false;
    } else {
      double a0 = (sh.z0 - zp) / dz, a1 = (sh.z1 - zp) / dz;
      if (a0 > a1) { const double t = a0; a0 = a1; a1 = t; }
      lo = a0;
      hi = a1;
    }
  }
  if (A < 1e-300) {
    if (C > 0.0) return false;
  } else {
    const double disc = B * B - 4.0 * A * C;
    if (disc <= 0.0) return false;
    const double sq = sqrt(disc);
    const double q = -0.5 * (B + (B >= 0 ? sq : -sq));
    double r0 = q / A, r1 = (q != 0.0) ? C / q : r0;
    if (r0 > r1) { const double t = r0; r0 = r1; r1 = t; }
    if (r0 > lo) lo = r0;
    if (r1 < hi) hi = r1;
  }
  if (hi <= lo) return false;
  s0 = lo;
  s1 = hi;
  return true;
}

__device__ double segment_wepl(const Scene &S, const double P[3], const double Q[3]) {
  const double D[3] = {Q[0] - P[0], Q[1] - P[1], Q[2] - P[2]};
  const double len = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
  if (len <= 0.0) return 0.0;
  const double M[3] = {0.5 * (P[0] + Q[0]), 0.5 * (P[1] + Q[1]), 0.5 * (P[2] + Q[2])};
  double acc = 0.0;
  for (int s = 0; s < S.n_shapes; ++s) {
    const Shape &sh = S.s[s];
    const double ddx = M[0] - sh.c[0], ddy = M[1] - sh.c[1], ddz = M[2] - sh.c[2];
    const double reach = sh.bound_r + 0.5 * len;
    if (ddx * ddx + ddy * ddy + ddz * ddz > reach * reach) continue;
    double a, b;
    if (!shape_interval(sh, P, D, a, b)) continue;
    if (a < 0.0) a = 0.0;
    if (b > 1.0) b = 1.0;
    if (b > a) acc += sh.delta_rsp * (b - a) * len;
  }
  return acc;
}

__device__ __forceinline__ void beam_point(double pc, double ps, double u, double t, double v, double out[3]) {
  out[0] = u * pc - t * ps;
  out[1] = u * ps + t * pc;
  out[2] = v;
}

__global__ void __launch_bounds__(256) k_histories(Scene S, uint64_t seed, int64_t i0, int64_t n, Out o,
                                                   unsigned long long *failures) {
  const Params &p = S.p;
  const Shape &body = S.s[0];
  const double R0 = p.bk_alpha * pow(p.E_kin, p.bk_p);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t ii = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; ii < n; ii += stride) {
    const int64_t i = i0 + ii;
    const int32_t a_idx = (int32_t)(i % p.n_angles);
    const double phi = 2.0 * M_PI * (double)a_idx / (double)p.n_angles;
    const double pc = cos(phi), ps = sin(phi);
    bool done = false;
    for (uint32_t attempt = 0; attempt < 1000 && !done; ++attempt) {
      Rng rg(seed, (uint64_t)i, attempt);
      const double t0 = (2.0 * rg.uniform() - 1.0) * p.t_half;
      const double v0 = (2.0 * rg.uniform() - 1.0) * p.v_half;
      double z0, z1;
      rg.normal2(z0, z1);
      const double st = z0 * p.slope_sigma, sv = z1 * p.slope_sigma;
      double P[3], Q[3];
      const double ua = p.u_in, ub = p.u_out;
      beam_point(pc, ps, ua, t0, v0, P);
      beam_point(pc, ps, ub, t0 + st * (ub - ua), v0 + sv * (ub - ua), Q);
      const double Dl[3] = {Q[0] - P[0], Q[1] - P[1], Q[2] - P[2]};
      double s_a, s_b;
      if (!shape_interval(body, P, Dl, s_a, s_b)) continue;
      if (s_b <= 0.0 || s_a >= 1.0) continue;
      const double u_enter = ua + s_a * (ub - ua);
      double kappa = 1.0;
      if (p.highland_log) {
        double Lwe = segment_wepl(S, P, Q);
        if (Lwe < 1e-3) Lwe = 1e-3;
        const double g = 1.0 + 0.038 * log(Lwe / p.X0);
        kappa = g * g;
      }
      double u = u_enter;
      double t = t0 + st * (u - ua), v = v0 + sv * (u - ua);
      double th_t = st, th_v = sv;
      double wdepth = 0.0, rsp_prev = -1.0;
      bool stopped = false;
      const double h = p.step;
      const double u_end = p.body_rxy + h;
      while (u < u_end) {
        const double hh = h;
        double T = 0.0;
        if (p.scatter) {
          double rsp_here = rsp_prev;
          if (rsp_here < 0.0) {
            double A0[3], A1[3];
            beam_point(pc, ps, u, t, v, A0);
            beam_point(pc, ps, u + hh, t + th_t * hh, v + th_v * hh, A1);
            const double sl = sqrt((A1[0] - A0[0]) * (A1[0] - A0[0]) + (A1[1] - A0[1]) * (A1[1] - A0[1]) +
                                   (A1[2] - A0[2]) * (A1[2] - A0[2]));
            rsp_here = segment_wepl(S, A0, A1) / sl;
          }
          if (rsp_here > 0.0) {
            const double rem = R0 - wdepth;
            if (rem <= 1e-6) { stopped = true; break; }
            const double E = pow(rem / p.bk_alpha, 1.0 / p.bk_p);
            const double bp = (E * E + 2.0 * E * p.m_p) / (E + p.m_p);
            T = (p.E0_hl / bp) * (p.E0_hl / bp) * rsp_here / p.X0 * kappa;
          }
        }
        double dt_kick = 0.0, dth_t = 0.0, dv_kick = 0.0, dth_v = 0.0;
        if (T > 0.0) {
          double za, zb, zc, zd;
          rg.normal2(za, zb);
          rg.normal2(zc, zd);
          const double sth = sqrt(T * hh);
          const double sres = sqrt(T * hh * hh * hh / 12.0);
          dth_t = sth * za;
          dt_kick = 0.5 * hh * dth_t + sres * zb;
          dth_v = sth * zc;
          dv_kick = 0.5 * hh * dth_v + sres * zd;
        }
        const double un = u + hh;
        const double tn = t + th_t * hh + dt_kick;
        const double vn = v + th_v * hh + dv_kick;
        double A0[3], A1[3];
        beam_point(pc, ps, u, t, v, A0);
        beam_point(pc, ps, un, tn, vn, A1);
        const double w = segment_wepl(S, A0, A1);
        const double sl = sqrt((A1[0] - A0[0]) * (A1[0] - A0[0]) + (A1[1] - A0[1]) * (A1[1] - A0[1]) +
                               (A1[2] - A0[2]) * (A1[2] - A0[2]));
        wdepth += w;
        rsp_prev = (sl > 0.0) ? w / sl : 0.0;
        u = un;
        t = tn;
        v = vn;
        th_t += dth_t;
        th_v += dth_v;
      }
      if (stopped) continue;
      const double t_out = t + th_t * (p.u_out - u);
      const double v_out = v + th_v * (p.u_out - u);
      double zn0, zn1;
      rg.normal2(zn0, zn1);
      const double wepl = wdepth + p.wepl_sigma * zn0;
      o.f[0][ii] = (float)phi;
      o.f[1][ii] = (float)t0;
      o.f[2][ii] = (float)v0;
      o.f[3][ii] = (float)st;
      o.f[4][ii] = (float)sv;
      o.f[5][ii] = (float)t_out;
      o.f[6][ii] = (float)v_out;
      o.f[7][ii] = (float)th_t;
      o.f[8][ii] = (float)th_v;
      o.f[9][ii] = (float)wepl;
      done = true;
    }
    if (!done) {
      for (int q = 0; q < 10; ++q) o.f[q][ii] = __builtin_nanf("");
      atomicAdd(failures, 1ull);
    }
  }
}

}  // namespace

extern "C" {

/* Histories [i0, i0 + n) of the seeded sequence into ten device float32
 * arrays (phi, t_in, v_in, dt_in, dv_in, t_out, v_out, dt_out, dv_out, wepl),
 * on `stream`.  params / shapes: host structs laid out as gen.c's
 * pctgen_params / pctgen_shape (at most 16 shapes, shape 0 the body).
 * failures: device uint64 counter, incremented for each history that needed
 * more than 1000 attempts (written as NaN); the caller zeroes it.  Returns 0,
 * or -1 for bad arguments, -2 if the launch failed. */
int pctgen_gpu_histories(const void *params, const void *shapes, int32_t n_shapes, uint64_t seed, int64_t i0,
                         int64_t n, float *const *out, unsigned long long *failures, void *stream) {
  if (!params || !shapes || n_shapes < 1 || n_shapes > kMaxShapes || n < 0 || i0 < 0 || !out || !failures) return -1;
  if (n == 0) return 0;
  Scene S;
  S.p = *static_cast<const Params *>(params);
  S.n_shapes = n_shapes;
  const Shape *sh = static_cast<const Shape *>(shapes);
  for (int s = 0; s < n_shapes; ++s) {
    S.s[s] = sh[s];
    S.s[s].cy = cos(sh[s].yaw);
    S.s[s].sy = sin(sh[s].yaw);
  }
  Out o;
  for (int q = 0; q < 10; ++q) {
    if (!out[q]) return -1;
    o.f[q] = out[q];
  }
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_histories, dim3((unsigned)g), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), S, seed,
                     i0, n, o, failures);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // extern "C"
