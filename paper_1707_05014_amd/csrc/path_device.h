// Device-side construction of one proton's row of A by one wavefront:
// hull entry/exit, most-likely path samples, voxel walk, row assembly in LDS.
//
// Paper Sec. 2: each proton's MLP is estimated from the entry and exit
// positions and angles; its row of A holds the path length in every voxel the
// path touches.  The MLP is the Bayesian most-likely path the paper cites
// (Schulte et al. 2008) written in Kalman-gain form, which stays well
// conditioned at both ends of the path; the covariance integrals use closed
// forms of the polynomial prior.  The voxel walk is Amanatides-Woo, one path
// segment per lane, on sub-voxel local coordinates.
//
// The template parameter R is the precision of path positions, of the gain
// and of the voxel walk's crossing parameters: double gives lengths good to
// ~1e-12 mm except on near-tangent crossings; float is the reduced precision
// variant (coordinates good to ~1e-5 mm at 100 mm from the isocentre).  The
// walk runs on coordinates relative to the segment's first voxel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pct_internal.h"

namespace pct {

__device__ __forceinline__ int wave_lane() { return __lane_id(); }

// Cross-lane moves with DPP (GFX9 data-parallel primitives; no LDS traffic).
// Row shifts move data within rows of 16 lanes, row broadcasts carry lane 15
// of a row into the next row(s); wave shifts move data by one lane across the
// whole wavefront.  Lanes without a source lane read 0.
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;
constexpr int kDppWaveShl1 = 0x130, kDppWaveShr1 = 0x138;

// Orders this wavefront's LDS accesses across lanes (a write by one lane,
// then a read by another) without waiting for its outstanding global loads.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
}

// inclusive prefix sum over the 64 lanes
__device__ __forceinline__ int wave_incl_scan_i32(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, kDppRowShr1, 0xf, 0xf, false);
  x += __builtin_amdgcn_update_dpp(0, x, kDppRowShr2, 0xf, 0xf, false);
  x += __builtin_amdgcn_update_dpp(0, x, kDppRowShr4, 0xf, 0xf, false);
  x += __builtin_amdgcn_update_dpp(0, x, kDppRowShr8, 0xf, 0xf, false);
  x += __builtin_amdgcn_update_dpp(0, x, kDppRowBcast15, 0xa, 0xf, false);
  x += __builtin_amdgcn_update_dpp(0, x, kDppRowBcast31, 0xc, 0xf, false);
  return x;
}

__device__ __forceinline__ float wave_incl_scan_dpp(float x) {
  x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), kDppRowShr1, 0xf, 0xf, false));
  x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), kDppRowShr2, 0xf, 0xf, false));
  x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), kDppRowShr4, 0xf, 0xf, false));
  x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), kDppRowShr8, 0xf, 0xf, false));
  x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), kDppRowBcast15, 0xa, 0xf, false));
  x += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), kDppRowBcast31, 0xc, 0xf, false));
  return x;
}

// exclusive prefix sum over the 64 lanes
__device__ __forceinline__ int wave_excl_scan(int v) { return wave_incl_scan_i32(v) - v; }

// the value held by lane + 1 (lane 63 reads 0) / lane - 1 (lane 0 reads 0)
__device__ __forceinline__ int lane_next(int v) {
  return __builtin_amdgcn_update_dpp(0, v, kDppWaveShl1, 0xf, 0xf, true);
}
__device__ __forceinline__ int lane_prev(int v) {
  return __builtin_amdgcn_update_dpp(0, v, kDppWaveShr1, 0xf, 0xf, true);
}
__device__ __forceinline__ float lane_next(float v) {
  return __builtin_bit_cast(float, lane_next(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double lane_next(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)lane_next((int)(uint32_t)u);
  const uint32_t hi = (uint32_t)lane_next((int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ float wave_sum_f32(float v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// move a wave-uniform value into scalar registers
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uniform(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double uniform(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// 1/a for finite nonzero a: the hardware estimate refined by two Newton steps
// (within an ulp or two of the quotient; a fraction of the IEEE division's
// instruction count)
__device__ __forceinline__ double recip(double a) {
  double y = __builtin_amdgcn_rcp(a);
  double e = fma(-a, y, 1.0);
  y = fma(y, e, y);
  e = fma(-a, y, 1.0);
  return fma(y, e, y);
}
__device__ __forceinline__ float recip(float a) { return 1.0f / a; }

template <typename R> __device__ __forceinline__ R rsqrt_(R v);
template <> __device__ __forceinline__ float rsqrt_(float v) { return sqrtf(v); }
template <> __device__ __forceinline__ double rsqrt_(double v) { return sqrt(v); }

// The prior's antiderivative tables cF[p][n] (3 x 8), staged per workgroup in
// LDS so that they do not occupy scalar registers for the whole kernel.
template <typename R> struct Tables;
template <> struct Tables<double> {
  __device__ static const double *cF(const PathParams &P) { return &P.cF_d[0][0]; }
};
template <> struct Tables<float> {
  __device__ static const float *cF(const PathParams &P) { return &P.cF_f[0][0]; }
};

// copy the tables into s_cF[24] (all threads of the workgroup call it; it
// ends with a workgroup barrier)
template <typename R>
__device__ __forceinline__ void stage_prior(const PathParams &P, R *s_cF) {
  if (threadIdx.x < 24) s_cF[threadIdx.x] = Tables<R>::cF(P)[threadIdx.x];
  __syncthreads();
}

// Interval [lo, hi] of u on which the line t(u) = t_ref + st (u - u_ref),
// v(u) = v_ref + sv (u - u_ref) lies in the elliptic-cylinder hull.
template <typename R>
__device__ __forceinline__ bool hull_interval(const PathParams &P, R c, R s, R u_ref, R t_ref, R v_ref, R st, R sv,
                                              R &lo, R &hi) {
  const R ia2 = (R)P.hull_ia2, ib2 = (R)P.hull_ib2;
  const R T = t_ref - st * u_ref;
  const R V = v_ref - sv * u_ref;
  const R px = c - st * s, qx = -T * s;
  const R py = s + st * c, qy = T * c;
  const R A = px * px * ia2 + py * py * ib2;
  const R B = (R)2 * (px * qx * ia2 + py * qy * ib2);
  const R C = qx * qx * ia2 + qy * qy * ib2 - (R)1;
  const R disc = B * B - (R)4 * A * C;
  if (!(disc > (R)0)) return false;
  const R sq = rsqrt_<R>(disc);
  const R q = (R)(-0.5) * (B + (B >= (R)0 ? sq : -sq));
  R r0 = q / A, r1 = (q != (R)0) ? C / q : r0;
  lo = r0 < r1 ? r0 : r1;
  hi = r0 < r1 ? r1 : r0;
  if (sv != (R)0) {
    R z0 = ((R)P.hull_zmin - V) / sv, z1 = ((R)P.hull_zmax - V) / sv;
    R zl = z0 < z1 ? z0 : z1, zh = z0 < z1 ? z1 : z0;
    lo = lo > zl ? lo : zl;
    hi = hi < zh ? hi : zh;
  } else if (V < (R)P.hull_zmin || V > (R)P.hull_zmax) {
    return false;
  }
  return hi > lo;
}

template <typename R>
struct ProtonPath {
  bool valid;
  int K;                 // segments
  R u0, L, c, s;         // hull entry, path length along u, cos/sin phi
  R t0, st0, v0, sv0;    // entry state
  R dtt, dts, dvt, dvs;  // innovations y2 - R(L) y0 per plane
  R FL[3];               // F_p(L), p = 0, 1, 2 (see mlp_point)
};

// The per-proton set-up as stored by k_path_setup (one thread per proton)
// and read by the path kernels (one wavefront per proton, scalar loads):
// the fifteen ProtonPath values, the segment count (0: no path) and b_i.
template <typename R>
struct PathRec {
  R v[15];   // u0, L, c, s, t0, st0, v0, sv0, dtt, dts, dvt, dvs, FL0, FL1, FL2
  int32_t K;
  float b;
};
static_assert(sizeof(PathRec<double>) <= kPathRecBytes, "path record larger than its workspace slot");

template <typename T>
__device__ __forceinline__ const T *uniform_ptr(const T *p) {
  const uint64_t u = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
  return reinterpret_cast<const T *>(((uint64_t)hi << 32) | lo);
}

// Horner: d^(M+1) * sum_n c[n] d^n
template <typename R, int M>
__device__ __forceinline__ R moment(const R *c, R d) {
  R acc = (R)0;
#pragma unroll
  for (int q = 7; q >= 0; --q) acc = acc * d + c[q];
  R dp = d;
#pragma unroll
  for (int m = 0; m < M; ++m) dp *= d;
  return acc * dp;
}

// Per-proton set-up, computed by one thread (k_path_setup).  The hull
// intersections and end states are found in double for both path precisions:
// they are per proton, and near-tangent lines are ill-conditioned.
template <typename R>
__device__ __forceinline__ void setup_path(const PathParams &P, const R *cF, const float h[10], ProtonPath<R> &pp) {
  pp.valid = false;
  pp.K = 0;
  bool fin = true;
#pragma unroll
  for (int q = 0; q < 10; ++q) fin = fin && isfinite(h[q]);
  if (!fin) return;
  double c, s;
  sincos((double)h[0], &s, &c);
  double a0, b0, a2, b2;
  const double u_in = P.u_in, u_out = P.u_out;
  if (!hull_interval<double>(P, c, s, u_in, h[1], h[2], h[3], h[4], a0, b0)) return;
  if (!hull_interval<double>(P, c, s, u_out, h[5], h[6], h[7], h[8], a2, b2)) return;
  const double u0 = a0, u2 = b2;
  const double L = u2 - u0;
  if (!(L > 0.0)) return;
  int K = (int)ceil(L * (double)P.inv_step - 1e-9);
  if (K < 1) K = 1;
  const double st0 = h[3], sv0 = h[4];
  const double t0 = (double)h[1] + st0 * (u0 - u_in);
  const double v0 = (double)h[2] + sv0 * (u0 - u_in);
  const double t2 = (double)h[5] + (double)h[7] * (u2 - u_out);
  const double v2 = (double)h[6] + (double)h[8] * (u2 - u_out);
  pp.K = K;
  pp.c = (R)c;
  pp.s = (R)s;
  pp.u0 = (R)u0;
  pp.L = (R)L;
  pp.st0 = (R)st0;
  pp.sv0 = (R)sv0;
  pp.t0 = (R)t0;
  pp.v0 = (R)v0;
  pp.dtt = (R)(t2 - (t0 + st0 * L));
  pp.dts = (R)((double)h[7] - st0);
  pp.dvt = (R)(v2 - (v0 + sv0 * L));
  pp.dvs = (R)((double)h[8] - sv0);
  pp.FL[0] = moment<R, 0>(cF, pp.L);
  pp.FL[1] = moment<R, 1>(cF + 8, pp.L);
  pp.FL[2] = moment<R, 2>(cF + 16, pp.L);
  pp.valid = true;
}

template <typename R>
__device__ __forceinline__ void store_record(const ProtonPath<R> &pp, float b, PathRec<R> *rec) {
  PathRec<R> r;
  const R vals[15] = {pp.u0, pp.L, pp.c, pp.s, pp.t0, pp.st0, pp.v0, pp.sv0,
                      pp.dtt, pp.dts, pp.dvt, pp.dvs, pp.FL[0], pp.FL[1], pp.FL[2]};
#pragma unroll
  for (int q = 0; q < 15; ++q) r.v[q] = pp.valid ? vals[q] : (R)0;
  r.K = pp.valid ? pp.K : 0;
  r.b = b;
  *rec = r;
}

// the record of the wavefront's proton, in scalar registers
template <typename R>
__device__ __forceinline__ void load_record(const PathRec<R> *rec, ProtonPath<R> &pp, float &b) {
  const PathRec<R> *r = uniform_ptr(rec);
  pp.K = uniform(r->K);
  pp.valid = pp.K > 0;
  pp.u0 = uniform(r->v[0]); pp.L = uniform(r->v[1]); pp.c = uniform(r->v[2]); pp.s = uniform(r->v[3]);
  pp.t0 = uniform(r->v[4]); pp.st0 = uniform(r->v[5]); pp.v0 = uniform(r->v[6]); pp.sv0 = uniform(r->v[7]);
  pp.dtt = uniform(r->v[8]); pp.dts = uniform(r->v[9]); pp.dvt = uniform(r->v[10]); pp.dvs = uniform(r->v[11]);
  pp.FL[0] = uniform(r->v[12]); pp.FL[1] = uniform(r->v[13]); pp.FL[2] = uniform(r->v[14]);
  b = uniform(r->b);
}

// MLP lateral offsets (t, v) at depth d1 from the hull entry, 0 < d1 < L.
//   S1 ~ [I2 I1; I1 I0],  I_m = int_0^d1 f(s) (d1 - s)^m ds
//   S2 ~ [J2 J1; J1 J0],  J_m = int_d1^L f(s) (L - s)^m ds
// Both from the three antiderivative moments F_p(x) = int_0^x f(s) s^p ds by
// the binomial expansions of (d1 - s)^m and (L - s)^m (the common factor
// E0^2/X0 cancels in the gain).
template <typename R>
__device__ __forceinline__ void mlp_point(const PathParams &P, const R *cF, const ProtonPath<R> &pp, R d1, R &t,
                                          R &v) {
  const R L = pp.L;
  const R d2 = L - d1;
  const R F0 = moment<R, 0>(cF, d1);
  const R F1 = moment<R, 1>(cF + 8, d1);
  const R F2 = moment<R, 2>(cF + 16, d1);
  R I0 = F0;
  R I1 = d1 * F0 - F1;
  R I2 = d1 * (d1 * F0 - (R)2 * F1) + F2;
  const R e0 = pp.FL[0] - F0;
  const R e1 = pp.FL[1] - F1;
  const R e2 = pp.FL[2] - F2;
  R J0 = e0;
  R J1 = L * e0 - e1;
  R J2 = L * (L * e0 - (R)2 * e1) + e2;
  if (P.highland) {
    // the logarithmic factor only scales the two covariances; float keeps its
    // relative error near 1e-7 (a ~1e-7 mm change of the path) at a fraction
    // of the cost of a double logarithm
    const float ix0 = (float)P.inv_X0;
    const float f1 = fmaf(0.038f, __logf((float)d1 * ix0), 1.0f);
    const float f2 = fmaf(0.038f, __logf((float)d2 * ix0), 1.0f);
    const R g1 = (R)(f1 * f1);
    const R g2 = (R)(f2 * f2);
    I0 *= g1; I1 *= g1; I2 *= g1;
    J0 *= g2; J1 *= g2; J2 *= g2;
  }
  // C = R1 S1 R1^T + S2 with R1 = [1 d2; 0 1]
  const R C00 = d2 * d2 * I0 + (R)2 * d2 * I1 + I2 + J2;
  const R C01 = d2 * I0 + I1 + J1;
  const R C11 = I0 + J0;
  const R det = C00 * C11 - C01 * C01;
  // first row of S1 R1^T C^-1
  const R A0 = d2 * I1 + I2, A1 = I1;
  const R inv = recip(det);
  const R G0 = (A0 * C11 - A1 * C01) * inv;
  const R G1 = (A1 * C00 - A0 * C01) * inv;
  t = pp.t0 + pp.st0 * d1 + (G0 * pp.dtt + G1 * pp.dts);
  v = pp.v0 + pp.sv0 * d1 + (G0 * pp.dvt + G1 * pp.dvs);
}

// index of voxel (ix, iy, iz) in the rows' numbering (P.brick)
__device__ __forceinline__ int voxel_id(const PathParams &P, int ix, int iy, int iz) {
  if (!P.brick) return (iz * P.ny + iy) * P.nx + ix;
  return ((((iz >> 2) * P.nby + (iy >> 2)) * P.nbx + (ix >> 2)) << 6) | ((iz & 3) << 4) | ((iy & 3) << 2) | (ix & 3);
}

// Voxel walk of one segment given in local coordinates: (px,py,pz) in [0,1]^3
// relative to voxel (bx,by,bz), end point (qx,qy,qz) in the same frame,
// physical length seg.  Emits up to kMaxPieces (voxel, length) pieces;
// returns the count, or kMaxPieces + 1 on overflow.  W is the precision of
// the crossing parameters.
template <typename W>
__device__ __forceinline__ int walk_segment(const PathParams &P, int bx, int by, int bz, W px, W py, W pz, W qx,
                                            W qy, W qz, W seg, int vox[kMaxPieces], float len[kMaxPieces]) {
  const W dx = qx - px, dy = qy - py, dz = qz - pz;
  int ix = bx, iy = by, iz = bz;
  const W INF = (W)3.0e38f;
  int sx = 0, sy = 0, sz = 0;
  W tx = INF, ty = INF, tz = INF, ddx = INF, ddy = INF, ddz = INF;
  // crossing parameters along the segment: next face per axis, then per voxel
  if (dx > (W)0) { sx = 1; ddx = recip(dx); tx = ((W)1 - px) * ddx; }
  else if (dx < (W)0) { sx = -1; ddx = -recip(dx); tx = px * ddx; }
  if (dy > (W)0) { sy = 1; ddy = recip(dy); ty = ((W)1 - py) * ddy; }
  else if (dy < (W)0) { sy = -1; ddy = -recip(dy); ty = py * ddy; }
  if (dz > (W)0) { sz = 1; ddz = recip(dz); tz = ((W)1 - pz) * ddz; }
  else if (dz < (W)0) { sz = -1; ddz = -recip(dz); tz = pz * ddz; }
  W tc = (W)0;
  int np = 0;
  const W eps = (W)P.eps_len;
  // Straight-line body (selects, no branches inside): a lane that has
  // reached the segment's end keeps its state and emits nothing; the loop
  // ends when every lane has.
  bool done = false, over = false;
  for (int it = 0; it < 3 * kMaxPieces; ++it) {
    W tn = tx < ty ? tx : ty;
    tn = tn < tz ? tn : tz;
    tn = tn < (W)1 ? tn : (W)1;
    const W l = (tn - tc) * seg;
    const bool keep = !done && l > eps && ix >= 0 && iy >= 0 && iz >= 0 && ix < P.nx && iy < P.ny && iz < P.nz;
    over = over || (keep && np == kMaxPieces);
    const int j = voxel_id(P, ix, iy, iz);
#pragma unroll
    for (int q = 0; q < kMaxPieces; ++q) {
      const bool w = keep && q == np;
      vox[q] = w ? j : vox[q];
      len[q] = w ? (float)l : len[q];
    }
    np += keep ? 1 : 0;
    done = done || tn >= (W)1;
    if (!__any(!done)) break;
    tc = done ? tc : tn;
    const bool ax = !done && tx <= ty && tx <= tz;
    const bool ay = !done && !ax && ty <= tz;
    const bool az = !done && !ax && !ay;
    ix += ax ? sx : 0;
    iy += ay ? sy : 0;
    iz += az ? sz : 0;
    tx = ax ? tx + ddx : tx;
    ty = ay ? ty + ddy : ty;
    tz = az ? tz + ddz : tz;
  }
  return (over || !done) ? kMaxPieces + 1 : (np > kMaxPieces ? kMaxPieces + 1 : np);
}

// the row buffer of wavefront wid in the dynamic LDS area (see row_buf_bytes)
struct RowBuf {
  int *vox;
  float *len;
  int16_t *aux;
};
__device__ __forceinline__ RowBuf row_buf(void *smem, int wid, int emax) {
  char *base = static_cast<char *>(smem) + (size_t)wid * row_buf_bytes(emax);
  return {reinterpret_cast<int *>(base), reinterpret_cast<float *>(base + 4 * (size_t)emax),
          reinterpret_cast<int16_t *>(base + 8 * (size_t)emax)};
}

// Build the row of one proton (set-up pp, wave-uniform) in the wavefront's
// LDS slice (s_vox, s_len, s_aux of P.emax entries each); cF = the staged
// prior tables.  Returns the entry count (wave-uniform); on a bound violation
// sets `status` bits and returns 0.
template <typename R>
__device__ int build_row(const PathParams &P, const R *cF, const ProtonPath<R> &pp, int *s_vox, float *s_len,
                         int16_t *s_aux, uint32_t *status) {
  const int lane = wave_lane();
  if (!pp.valid) return 0;
  if (pp.K > P.kmax) {
    if (lane == 0) atomicOr(status, kStOverflow);
    return 0;
  }
  const int K = pp.K;
  const R du = pp.L / (R)K;
  const R gox = (R)P.ox, goy = (R)P.oy, goz = (R)P.oz;
  const R gix = (R)P.idx, giy = (R)P.idy, giz = (R)P.idz;
  int count = 0;
  int carry_vox = -1;
  int lane_dirs = 0;  // directions in which the voxel indices of this lane's segments change (below)
  for (int base = 0; base < K; base += kSegPerRound) {
    const int k = base + lane;
    R wx = 0, wy = 0, wz = 0;
    if (k <= K) {
      R t, v, d1;
      if (k == 0) {
        t = pp.t0; v = pp.v0; d1 = 0;
      } else if (k == K) {
        t = pp.t0 + pp.st0 * pp.L + pp.dtt;
        v = pp.v0 + pp.sv0 * pp.L + pp.dvt;
        d1 = pp.L;
      } else {
        d1 = (R)k * du;
        mlp_point<R>(P, cF, pp, d1, t, v);
      }
      const R u = pp.u0 + d1;
      wx = u * pp.c - t * pp.s;
      wy = u * pp.s + t * pp.c;
      wz = v;
    }
    const R gx = (wx - gox) * gix, gy = (wy - goy) * giy, gz = (wz - goz) * giz;
    const R ngx = lane_next(gx), ngy = lane_next(gy), ngz = lane_next(gz);
    const R nwx = lane_next(wx), nwy = lane_next(wy), nwz = lane_next(wz);
    int vox[kMaxPieces];
    float len[kMaxPieces];
    int np = 0;
    int dirs = 0;
    if (lane < kSegPerRound && k < K) {
      const R ex = nwx - wx, ey = nwy - wy, ez = nwz - wz;
      const R seg = rsqrt_<R>(ex * ex + ey * ey + ez * ez);
      const R fx = floor(gx), fy = floor(gy), fz = floor(gz);
      np = walk_segment<R>(P, (int)fx, (int)fy, (int)fz, gx - fx, gy - fy, gz - fz, ngx - fx, ngy - fy,
                           ngz - fz, seg, vox, len);
      // the segment's voxel-index changes per axis: bit a for up along axis
      // a (x, y, z), bit a + 3 for down (a path ending exactly on a face
      // enters the next voxel with the next segment; counted here)
      const R nfx = floor(ngx), nfy = floor(ngy), nfz = floor(ngz);
      dirs = (nfx > fx ? 1 : 0) | (nfy > fy ? 2 : 0) | (nfz > fz ? 4 : 0) | (nfx < fx ? 8 : 0) |
             (nfy < fy ? 16 : 0) | (nfz < fz ? 32 : 0);
    }
    lane_dirs |= dirs;
    const bool bad = np > kMaxPieces;
    if (__ballot(bad)) {
      if (lane == 0) atomicOr(status, kStOverflow);
      return 0;
    }
    int first = -1, last = -1;
    float first_len = 0.0f;
#pragma unroll
    for (int q = 0; q < kMaxPieces; ++q) {
      if (q == 0 && np > 0) { first = vox[0]; first_len = len[0]; }
      if (q == np - 1) last = vox[q];
    }
    int prev_last = lane_prev(last);
    if (lane == 0) prev_last = carry_vox;
    const bool merge = np > 0 && prev_last >= 0 && first == prev_last;
    const int ne = np - (merge ? 1 : 0);
    const int pos = wave_excl_scan(ne);
    const int total = __shfl(pos + ne, kWave - 1, kWave);
    if (count + total > P.emax) {
      if (lane == 0) atomicOr(status, kStOverflow);
      return 0;
    }
    // new entries
    const int at = count + pos - (merge ? 1 : 0);
#pragma unroll
    for (int q = 0; q < kMaxPieces; ++q) {
      if (q < np && !(q == 0 && merge)) {
        s_vox[at + q] = vox[q];
        s_len[at + q] = len[q];
      }
    }
    wave_lds_sync();
    // a first piece in the same voxel as the previous piece extends that entry
    if (merge) atomicAdd(&s_len[count + pos - 1], first_len);
    count += total;
    wave_lds_sync();
    carry_vox = count > 0 ? s_vox[count - 1] : -1;
  }
  // voxels revisited after a short excursion: fold into the first visit.
  // A path returns to a voxel only if it crosses faces of one axis in both
  // directions, so rows that never do skip the search.
  int row_dirs = 0;
#pragma unroll
  for (int b = 0; b < 6; ++b)
    if (__ballot(lane_dirs & (1 << b))) row_dirs |= 1 << b;
  if ((row_dirs & (row_dirs >> 3) & 7) == 0) return count;
  bool any = false;
  for (int e0 = 0; e0 < count; e0 += kWave) {
    const int e = e0 + lane;
    int m = -1;
    if (e < count) {
      const int v = s_vox[e];
      const int lo = e - kDedupWindow > 0 ? e - kDedupWindow : 0;
      for (int f = lo; f <= e - 2; ++f)
        if (s_vox[f] == v) { m = f; break; }
      s_aux[e] = (int16_t)m;
    }
    any = any || (__ballot(m >= 0) != 0);
  }
  wave_lds_sync();
  if (any) {
    if (lane == 0) {
      for (int e = 0; e < count; ++e) {
        int r = s_aux[e];
        if (r < 0) continue;
        while (s_aux[r] >= 0) r = s_aux[r];
        s_len[r] += s_len[e];
        s_vox[e] = -1;
      }
    }
    wave_lds_sync();
    int out = 0;
    for (int e0 = 0; e0 < count; e0 += kWave) {
      const int e = e0 + lane;
      int v = -1;
      float l = 0.f;
      if (e < count) { v = s_vox[e]; l = s_len[e]; }
      const int keep = v >= 0 ? 1 : 0;
      const int p = wave_excl_scan(keep);
      const int tot = __shfl(p + keep, kWave - 1, kWave);
      wave_lds_sync();
      if (keep) { s_vox[out + p] = v; s_len[out + p] = l; }
      wave_lds_sync();
      out += tot;
    }
    count = out;
  }
  return count;
}

__device__ __forceinline__ void load_history(const HistPtrs &H, int64_t i, float h[10]) {
  h[0] = H.phi[i]; h[1] = H.t_in[i]; h[2] = H.v_in[i]; h[3] = H.dt_in[i]; h[4] = H.dv_in[i];
  h[5] = H.t_out[i]; h[6] = H.v_out[i]; h[7] = H.dt_out[i]; h[8] = H.dv_out[i]; h[9] = H.wepl[i];
}

}  // namespace pct
