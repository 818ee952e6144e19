/*
 * Seeded synthetic proton-history generator (input data only).
 *
 * This module stands in for the scanner data that the paper reconstructs
 * (Sec. 3: a head-sized phantom imaged with 200 MeV protons by two tracker
 * pairs and a range detector, Sec. 2).  It produces, per proton, the entry
 * and exit positions and slopes at the two tracker planes and a WEPL value,
 * by transporting the proton through an analytic phantom with Gaussian
 * multiple Coulomb scattering.  It holds none of the reconstruction's
 * arithmetic: no most-likely path, no voxel traversal, no projection.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC 2011), keyed by the seed and counted by
 * (proton, attempt, draw), so every history is reproducible on its own and
 * the output does not depend on the thread count.
 *
 * Physics (FP64):
 *   - beam frame for gantry angle phi: u along (cos phi, sin phi, 0),
 *     t along (-sin phi, cos phi, 0), v along z;
 *   - straight flight in air from the entry tracker plane to the phantom;
 *   - inside: steps of h along u; per step the lateral (offset, slope) pair of
 *     each plane receives a correlated Gaussian kick with covariance
 *     T * [[h^3/3, h^2/2], [h^2/2, h]] (Fermi-Eyges), T = (E0/(beta p))^2 *
 *     rsp / X0 * kappa, beta*p from the Bragg-Kleeman range-energy relation
 *     at the water-equivalent depth reached, kappa = (1 + 0.038 ln(L/X0))^2
 *     from the straight entry chord's water-equivalent length L;
 *   - WEPL = exact integral of RSP along the resulting polyline through the
 *     analytic shapes, plus Gaussian noise.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- Philox */
static inline void mulhilo32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo) {
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

void pctgen_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo32(0xD2511F53u, c0, &hi0, &lo0);
        mulhilo32(0xCD9E8D57u, c2, &hi1, &lo1);
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

typedef struct {
    uint32_t key[2];
    uint32_t ctr[4];
    uint32_t buf[4];
    int left;
} rng_t;

static void rng_init(rng_t *r, uint64_t seed, uint64_t proton, uint32_t attempt) {
    r->key[0] = (uint32_t)seed;
    r->key[1] = (uint32_t)(seed >> 32);
    r->ctr[0] = 0;                      /* draw counter */
    r->ctr[1] = attempt;
    r->ctr[2] = (uint32_t)proton;
    r->ctr[3] = (uint32_t)(proton >> 32);
    r->left = 0;
}

static uint32_t rng_u32(rng_t *r) {
    if (r->left == 0) {
        pctgen_philox4x32_10(r->ctr, r->key, r->buf);
        r->ctr[0]++;
        r->left = 4;
    }
    return r->buf[4 - (r->left--)];
}

/* uniform in (0, 1), 53 random bits */
static double rng_uniform(rng_t *r) {
    uint64_t a = rng_u32(r) >> 5, b = rng_u32(r) >> 6;
    return ((double)(a * 67108864u + b) + 0.5) / 9007199254740992.0;
}

static void rng_normal2(rng_t *r, double *z0, double *z1) {
    double u1 = rng_uniform(r), u2 = rng_uniform(r);
    double rad = sqrt(-2.0 * log(u1));
    *z0 = rad * cos(2.0 * M_PI * u2);
    *z1 = rad * sin(2.0 * M_PI * u2);
}

/* ---------------------------------------------------------------- shapes */
/* kind 0: ellipsoid (cx,cy,cz, ax,ay,az, yaw);
 * kind 1: elliptic cylinder along z (cx,cy, ax,ay, yaw, z0..z1).
 * RSP composition: rsp(p) = sum over shapes containing p of delta_rsp. */
typedef struct {
    int32_t kind;
    double c[3];
    double ax[3];
    double yaw;
    double z0, z1;
    double delta_rsp;
    double bound_r;     /* radius of a bounding sphere about c (for culling) */
    double cy, sy;      /* cos/sin of yaw, filled in by the generator */
} pctgen_shape;

typedef struct {
    int32_t n_angles;
    double t_half, v_half;          /* entry field half-widths (uniform) */
    double slope_sigma;             /* entry slope std, rad */
    double u_in, u_out;             /* tracker planes */
    double step;                    /* transport step along u, mm */
    double E_kin;                   /* MeV */
    double bk_alpha, bk_p;          /* Bragg-Kleeman R = alpha E^p (mm, MeV) */
    double m_p;                     /* proton rest energy, MeV */
    double E0_hl, X0;               /* Highland constant (MeV) and X0 of water (mm) */
    int32_t highland_log;
    int32_t scatter;                /* 0 = straight lines (no scattering) */
    double wepl_sigma;              /* mm */
    /* hull = shape 0 (must be kind 1, the body) */
    double body_rxy;                /* max lateral extent of the body */
} pctgen_params;

/* interval of s in [0,1] for which P + s*D lies inside shape; returns length fraction */
static int shape_interval(const pctgen_shape *sh, const double P[3], const double D[3],
                          double *s0, double *s1) {
    double cs = sh->cy, sn = sh->sy;
    double px = P[0] - sh->c[0], py = P[1] - sh->c[1], pz = P[2] - sh->c[2];
    double lx = cs * px + sn * py, ly = -sn * px + cs * py;
    double dx = cs * D[0] + sn * D[1], dy = -sn * D[0] + cs * D[1], dz = D[2];
    double lo = -INFINITY, hi = INFINITY;
    double A, B, C;
    if (sh->kind == 0) {
        double ia = 1.0 / sh->ax[0], ib = 1.0 / sh->ax[1], ic = 1.0 / sh->ax[2];
        double qx = lx * ia, qy = ly * ib, qz = pz * ic;
        double ex = dx * ia, ey = dy * ib, ez = dz * ic;
        A = ex * ex + ey * ey + ez * ez;
        B = 2.0 * (qx * ex + qy * ey + qz * ez);
        C = qx * qx + qy * qy + qz * qz - 1.0;
    } else {
        double ia = 1.0 / sh->ax[0], ib = 1.0 / sh->ax[1];
        double qx = lx * ia, qy = ly * ib;
        double ex = dx * ia, ey = dy * ib;
        A = ex * ex + ey * ey;
        B = 2.0 * (qx * ex + qy * ey);
        C = qx * qx + qy * qy - 1.0;
        /* slab in absolute z */
        double zp = P[2];
        if (fabs(dz) < 1e-300) {
            if (zp < sh->z0 || zp > sh->z1) return 0;
        } else {
            double a0 = (sh->z0 - zp) / dz, a1 = (sh->z1 - zp) / dz;
            if (a0 > a1) { double t = a0; a0 = a1; a1 = t; }
            lo = a0; hi = a1;
        }
    }
    if (A < 1e-300) {
        if (C > 0.0) return 0;
    } else {
        double disc = B * B - 4.0 * A * C;
        if (disc <= 0.0) return 0;
        double sq = sqrt(disc);
        double q = -0.5 * (B + (B >= 0 ? sq : -sq));
        double r0 = q / A, r1 = (q != 0.0) ? C / q : r0;
        if (r0 > r1) { double t = r0; r0 = r1; r1 = t; }
        if (r0 > lo) lo = r0;
        if (r1 < hi) hi = r1;
    }
    if (hi <= lo) return 0;
    *s0 = lo; *s1 = hi;
    return 1;
}

/* integral of rsp along segment P -> Q */
static double segment_wepl(const pctgen_shape *shapes, int ns, const double P[3], const double Q[3]) {
    double D[3] = {Q[0] - P[0], Q[1] - P[1], Q[2] - P[2]};
    double len = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
    if (len <= 0.0) return 0.0;
    double M[3] = {0.5 * (P[0] + Q[0]), 0.5 * (P[1] + Q[1]), 0.5 * (P[2] + Q[2])};
    double acc = 0.0;
    for (int s = 0; s < ns; ++s) {
        const pctgen_shape *sh = &shapes[s];
        double ddx = M[0] - sh->c[0], ddy = M[1] - sh->c[1], ddz = M[2] - sh->c[2];
        double reach = sh->bound_r + 0.5 * len;
        if (ddx * ddx + ddy * ddy + ddz * ddz > reach * reach) continue;
        double a, b;
        if (!shape_interval(sh, P, D, &a, &b)) continue;
        if (a < 0.0) a = 0.0;
        if (b > 1.0) b = 1.0;
        if (b > a) acc += sh->delta_rsp * (b - a) * len;
    }
    return acc;
}

static void beam_point(double phi_c, double phi_s, double u, double t, double v, double out[3]) {
    out[0] = u * phi_c - t * phi_s;
    out[1] = u * phi_s + t * phi_c;
    out[2] = v;
}

/* beta*p (MeV) of a proton of kinetic energy E */
static double beta_p(double E, double m) {
    double pc2 = E * E + 2.0 * E * m;
    return pc2 / (E + m);
}

/*
 * Generate histories [i0, i0+n) of the seeded sequence.  Output arrays are
 * float32, length n.  Returns the number of histories that needed more than
 * 1000 attempts (they are written as NaN), normally 0.
 */
static pctgen_shape *with_trig(const pctgen_shape *in, int32_t n) {
    pctgen_shape *o = (pctgen_shape *)malloc((size_t)(n > 0 ? n : 1) * sizeof(pctgen_shape));
    for (int32_t s = 0; s < n; ++s) {
        o[s] = in[s];
        o[s].cy = cos(in[s].yaw);
        o[s].sy = sin(in[s].yaw);
    }
    return o;
}

static int64_t histories_impl(const pctgen_params *p, const pctgen_shape *shapes, int32_t n_shapes,
                         uint64_t seed, int64_t i0, int64_t n,
                         float *phi_o, float *t_in_o, float *v_in_o, float *dt_in_o, float *dv_in_o,
                         float *t_out_o, float *v_out_o, float *dt_out_o, float *dv_out_o,
                         float *wepl_o, int32_t nthreads) {
    const pctgen_shape *body = &shapes[0];
    const double R0 = p->bk_alpha * pow(p->E_kin, p->bk_p);
    int64_t failures = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : failures)
#endif
    for (int64_t ii = 0; ii < n; ++ii) {
        int64_t i = i0 + ii;
        int32_t a_idx = (int32_t)(i % p->n_angles);
        double phi = 2.0 * M_PI * (double)a_idx / (double)p->n_angles;
        double pc = cos(phi), ps = sin(phi);
        int done = 0;
        for (uint32_t attempt = 0; attempt < 1000 && !done; ++attempt) {
            rng_t rg;
            rng_init(&rg, seed, (uint64_t)i, attempt);
            double t0 = (2.0 * rng_uniform(&rg) - 1.0) * p->t_half;
            double v0 = (2.0 * rng_uniform(&rg) - 1.0) * p->v_half;
            double z0, z1;
            rng_normal2(&rg, &z0, &z1);
            double st = z0 * p->slope_sigma, sv = z1 * p->slope_sigma;
            /* entry line: does it meet the body? */
            double P[3], Q[3];
            double ua = p->u_in, ub = p->u_out;
            beam_point(pc, ps, ua, t0, v0, P);
            beam_point(pc, ps, ub, t0 + st * (ub - ua), v0 + sv * (ub - ua), Q);
            double Dl[3] = {Q[0] - P[0], Q[1] - P[1], Q[2] - P[2]};
            double s_a, s_b;
            if (!shape_interval(body, P, Dl, &s_a, &s_b)) continue;
            if (s_b <= 0.0 || s_a >= 1.0) continue;
            double u_enter = ua + s_a * (ub - ua);
            /* Highland factor from the straight entry chord's water-equivalent length */
            double kappa = 1.0;
            if (p->highland_log) {
                double Lwe = segment_wepl(shapes, n_shapes, P, Q);
                if (Lwe < 1e-3) Lwe = 1e-3;
                double g = 1.0 + 0.038 * log(Lwe / p->X0);
                kappa = g * g;
            }
            /* transport */
            double u = u_enter;
            double t = t0 + st * (u - ua), v = v0 + sv * (u - ua);
            double th_t = st, th_v = sv;
            double wdepth = 0.0, rsp_prev = -1.0;
            int stopped = 0;
            const double h = p->step;
            const double u_end = p->body_rxy + h;
            while (u < u_end) {
                double hh = h;
                double T = 0.0;
                if (p->scatter) {
                    double rsp_here = rsp_prev;
                    if (rsp_here < 0.0) {
                        /* first step: material on the straight step ahead */
                        double A0[3], A1[3];
                        beam_point(pc, ps, u, t, v, A0);
                        beam_point(pc, ps, u + hh, t + th_t * hh, v + th_v * hh, A1);
                        double sl = sqrt((A1[0] - A0[0]) * (A1[0] - A0[0]) + (A1[1] - A0[1]) * (A1[1] - A0[1]) +
                                         (A1[2] - A0[2]) * (A1[2] - A0[2]));
                        rsp_here = segment_wepl(shapes, n_shapes, A0, A1) / sl;
                    }
                    if (rsp_here > 0.0) {
                        double rem = R0 - wdepth;
                        if (rem <= 1e-6) { stopped = 1; break; }
                        double E = pow(rem / p->bk_alpha, 1.0 / p->bk_p);
                        double bp = beta_p(E, p->m_p);
                        T = (p->E0_hl / bp) * (p->E0_hl / bp) * rsp_here / p->X0 * kappa;
                    }
                }
                double dt_kick = 0.0, dth_t = 0.0, dv_kick = 0.0, dth_v = 0.0;
                if (T > 0.0) {
                    /* correlated pair: th ~ sqrt(T h) z_a ; x = T h^2/2 / (T h) th + sqrt(T h^3/12) z_b */
                    double za, zb, zc, zd;
                    rng_normal2(&rg, &za, &zb);
                    rng_normal2(&rg, &zc, &zd);
                    double sth = sqrt(T * hh);
                    double sres = sqrt(T * hh * hh * hh / 12.0);
                    dth_t = sth * za;
                    dt_kick = 0.5 * hh * dth_t + sres * zb;
                    dth_v = sth * zc;
                    dv_kick = 0.5 * hh * dth_v + sres * zd;
                }
                double un = u + hh;
                double tn = t + th_t * hh + dt_kick;
                double vn = v + th_v * hh + dv_kick;
                double A0[3], A1[3];
                beam_point(pc, ps, u, t, v, A0);
                beam_point(pc, ps, un, tn, vn, A1);
                double w = segment_wepl(shapes, n_shapes, A0, A1);
                double sl = sqrt((A1[0] - A0[0]) * (A1[0] - A0[0]) + (A1[1] - A0[1]) * (A1[1] - A0[1]) +
                                 (A1[2] - A0[2]) * (A1[2] - A0[2]));
                wdepth += w;
                rsp_prev = (sl > 0.0) ? w / sl : 0.0;
                u = un; t = tn; v = vn;
                th_t += dth_t; th_v += dth_v;
            }
            if (stopped) continue;
            /* straight in air to the exit tracker plane */
            double t_out = t + th_t * (p->u_out - u);
            double v_out = v + th_v * (p->u_out - u);
            double zn0, zn1;
            rng_normal2(&rg, &zn0, &zn1);
            double wepl = wdepth + p->wepl_sigma * zn0;
            phi_o[ii] = (float)phi;
            t_in_o[ii] = (float)t0;
            v_in_o[ii] = (float)v0;
            dt_in_o[ii] = (float)st;
            dv_in_o[ii] = (float)sv;
            t_out_o[ii] = (float)t_out;
            v_out_o[ii] = (float)v_out;
            dt_out_o[ii] = (float)th_t;
            dv_out_o[ii] = (float)th_v;
            wepl_o[ii] = (float)wepl;
            done = 1;
        }
        if (!done) {
            float nanv = NAN;
            phi_o[ii] = t_in_o[ii] = v_in_o[ii] = dt_in_o[ii] = dv_in_o[ii] = nanv;
            t_out_o[ii] = v_out_o[ii] = dt_out_o[ii] = dv_out_o[ii] = wepl_o[ii] = nanv;
            failures += 1;
        }
    }
    return failures;
}

int64_t pctgen_histories(const pctgen_params *p, const pctgen_shape *shapes, int32_t n_shapes,
                         uint64_t seed, int64_t i0, int64_t n,
                         float *phi_o, float *t_in_o, float *v_in_o, float *dt_in_o, float *dv_in_o,
                         float *t_out_o, float *v_out_o, float *dt_out_o, float *dv_out_o,
                         float *wepl_o, int32_t nthreads) {
    pctgen_shape *sh = with_trig(shapes, n_shapes);
    int64_t r = histories_impl(p, sh, n_shapes, seed, i0, n, phi_o, t_in_o, v_in_o, dt_in_o, dv_in_o, t_out_o,
                               v_out_o, dt_out_o, dv_out_o, wepl_o, nthreads);
    free(sh);
    return r;
}

/*
 * Histories [i0, i0+n) of a second seeded stream: protons whose straight
 * line misses the body, as a scanner records them passing through air
 * beside the object (input of the space-carving hull).  Same beam and field
 * as pctgen_histories, counters (seed, proton, 0x40000000 + attempt, draw),
 * so the stream is disjoint from the object histories; the line is kept
 * when it misses the body between the tracker planes.  Exit state = the
 * straight extrapolation, WEPL = Gaussian noise only.  Returns the number
 * of failures (NaN rows), normally 0.
 */
int64_t pctgen_miss_histories(const pctgen_params *p, const pctgen_shape *shapes_in, int32_t n_shapes,
                              uint64_t seed, int64_t i0, int64_t n,
                              float *phi_o, float *t_in_o, float *v_in_o, float *dt_in_o, float *dv_in_o,
                              float *t_out_o, float *v_out_o, float *dt_out_o, float *dv_out_o,
                              float *wepl_o, int32_t nthreads) {
    pctgen_shape *shapes = with_trig(shapes_in, n_shapes);
    const pctgen_shape *body = &shapes[0];
    int64_t failures = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : failures)
#endif
    for (int64_t ii = 0; ii < n; ++ii) {
        int64_t i = i0 + ii;
        int32_t a_idx = (int32_t)(i % p->n_angles);
        double phi = 2.0 * M_PI * (double)a_idx / (double)p->n_angles;
        double pc = cos(phi), ps = sin(phi);
        int done = 0;
        for (uint32_t attempt = 0; attempt < 1000 && !done; ++attempt) {
            rng_t rg;
            rng_init(&rg, seed, (uint64_t)i, 0x40000000u + attempt);
            double t0 = (2.0 * rng_uniform(&rg) - 1.0) * p->t_half;
            double v0 = (2.0 * rng_uniform(&rg) - 1.0) * p->v_half;
            double z0, z1;
            rng_normal2(&rg, &z0, &z1);
            double st = z0 * p->slope_sigma, sv = z1 * p->slope_sigma;
            double P[3], Q[3];
            double ua = p->u_in, ub = p->u_out;
            beam_point(pc, ps, ua, t0, v0, P);
            beam_point(pc, ps, ub, t0 + st * (ub - ua), v0 + sv * (ub - ua), Q);
            double Dl[3] = {Q[0] - P[0], Q[1] - P[1], Q[2] - P[2]};
            double s_a, s_b;
            if (shape_interval(body, P, Dl, &s_a, &s_b) && s_b > 0.0 && s_a < 1.0) continue;
            double zn0, zn1;
            rng_normal2(&rg, &zn0, &zn1);
            phi_o[ii] = (float)phi;
            t_in_o[ii] = (float)t0;
            v_in_o[ii] = (float)v0;
            dt_in_o[ii] = (float)st;
            dv_in_o[ii] = (float)sv;
            t_out_o[ii] = (float)(t0 + st * (ub - ua));
            v_out_o[ii] = (float)(v0 + sv * (ub - ua));
            dt_out_o[ii] = (float)st;
            dv_out_o[ii] = (float)sv;
            wepl_o[ii] = (float)(p->wepl_sigma * zn0);
            done = 1;
        }
        if (!done) {
            float nanv = NAN;
            phi_o[ii] = t_in_o[ii] = v_in_o[ii] = dt_in_o[ii] = dv_in_o[ii] = nanv;
            t_out_o[ii] = v_out_o[ii] = dt_out_o[ii] = dv_out_o[ii] = wepl_o[ii] = nanv;
            failures += 1;
        }
    }
    free(shapes);
    return failures;
}

/* Exact RSP line integral of the analytic phantom along a segment (test hook). */
double pctgen_segment_wepl(const pctgen_shape *shapes, int32_t n_shapes, const double P[3], const double Q[3]) {
    pctgen_shape *sh = with_trig(shapes, n_shapes);
    double r = segment_wepl(sh, n_shapes, P, Q);
    free(sh);
    return r;
}

static double point_rsp(const pctgen_shape *shapes, int32_t n_shapes, const double X[3]);

/* Point RSP of the analytic phantom. */
double pctgen_point_rsp(const pctgen_shape *shapes, int32_t n_shapes, const double X[3]) {
    pctgen_shape *sh = with_trig(shapes, n_shapes);
    double r = point_rsp(sh, n_shapes, X);
    free(sh);
    return r;
}

static double point_rsp(const pctgen_shape *shapes, int32_t n_shapes, const double X[3]) {
    double acc = 0.0;
    for (int s = 0; s < n_shapes; ++s) {
        const pctgen_shape *sh = &shapes[s];
        double cs = sh->cy, sn = sh->sy;
        double px = X[0] - sh->c[0], py = X[1] - sh->c[1];
        double lx = cs * px + sn * py, ly = -sn * px + cs * py;
        double q;
        if (sh->kind == 0) {
            double pz = X[2] - sh->c[2];
            q = (lx / sh->ax[0]) * (lx / sh->ax[0]) + (ly / sh->ax[1]) * (ly / sh->ax[1]) +
                (pz / sh->ax[2]) * (pz / sh->ax[2]);
            if (q <= 1.0) acc += sh->delta_rsp;
        } else {
            q = (lx / sh->ax[0]) * (lx / sh->ax[0]) + (ly / sh->ax[1]) * (ly / sh->ax[1]);
            if (q <= 1.0 && X[2] >= sh->z0 && X[2] <= sh->z1) acc += sh->delta_rsp;
        }
    }
    return acc;
}

/* Voxel-average RSP on a grid by ss^3 point supersampling (truth image). */
void pctgen_truth_image(const pctgen_shape *shapes, int32_t n_shapes, int32_t nx, int32_t ny, int32_t nz,
                        double dx, double dy, double dz, double ox, double oy, double oz, int32_t ss,
                        float *out, int32_t nthreads) {
    pctgen_shape *sh = with_trig(shapes, n_shapes);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (int64_t j = 0; j < (int64_t)nx * ny * nz; ++j) {
        int i = (int)(j % nx), jj = (int)((j / nx) % ny), k = (int)(j / ((int64_t)nx * ny));
        double acc = 0.0;
        for (int a = 0; a < ss; ++a)
            for (int b = 0; b < ss; ++b)
                for (int c = 0; c < ss; ++c) {
                    double X[3] = {ox + (i + (a + 0.5) / ss) * dx, oy + (jj + (b + 0.5) / ss) * dy,
                                   oz + (k + (c + 0.5) / ss) * dz};
                    acc += point_rsp(sh, n_shapes, X);
                }
        out[j] = (float)(acc / ((double)ss * ss * ss));
    }
    free(sh);
}

/* splitmix64 (Steele, Lea, Flood 2014) */
static inline uint64_t splitmix64_next(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Seeded Fisher-Yates permutation of 0..n-1 (block composition order). */
void pctgen_permutation(int64_t n, uint64_t seed, int64_t *out) {
    for (int64_t i = 0; i < n; ++i) out[i] = i;
    uint64_t s = seed;
    for (int64_t i = n - 1; i > 0; --i) {
        /* unbiased bounded draw in [0, i] by rejection */
        uint64_t bound = (uint64_t)i + 1;
        uint64_t lim = UINT64_MAX - (UINT64_MAX % bound);
        uint64_t r;
        do { r = splitmix64_next(&s); } while (r >= lim);
        int64_t j = (int64_t)(r % bound);
        int64_t tmp = out[i]; out[i] = out[j]; out[j] = tmp;
    }
}
