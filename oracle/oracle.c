/*
 * FP64 CPU oracle of event-by-event pCT reconstruction.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline use it.  It is written for clarity, not speed, and shares no code
 * with the GPU library.
 *
 * What it computes (paper Sec. 2, "Image Reconstruction"):
 *   - for each proton history (entry and exit position and direction from the
 *     two tracker pairs, and its WEPL), the most-likely path through the
 *     object, sampled as a polyline;
 *   - the proton's row of A: the lengths of that path inside each voxel it
 *     touches (the paper's A has one column per proton; here A is N x M with
 *     one row per proton, so that Ax = b has b of length N and x of length M);
 *   - the block-iterative solution of Ax = b: DROP (Sec. 2.1: the data split
 *     into blocks, each block's solution seeds the next, a fixed number of
 *     sweeps), with ART (Kaczmarz) as the block-size-one case.
 *
 * The most-likely path follows the Bayesian formulation the paper cites
 * (Schulte et al. 2008), applied independently in the two lateral planes,
 * with a scattering prior built from a polynomial in depth for 1/(beta p)^2
 * and the Highland logarithmic factor.  The voxel traversal follows Siddon's
 * parametric method (all plane crossings sorted, midpoint classification).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t nx, ny, nz;
    double dx, dy, dz;
    double ox, oy, oz;
} orc_grid;

typedef struct {
    double u_in, u_out;                        /* tracker planes along the beam axis, mm */
    double hull_a, hull_b, hull_zmin, hull_zmax;  /* elliptic cylinder about the isocentre */
    double step;                               /* path sample spacing, mm */
    int32_t highland_log;                      /* 1: (1 + 0.038 ln(d/X0))^2 factor */
    int32_t n_poly;                            /* coefficients of 1/(beta p)^2 in depth (mm) */
    double poly[8];
    double E0, X0;                             /* MeV, mm */
} orc_geom;

/* history fields, in this order, as float32 arrays */
enum { H_PHI, H_TIN, H_VIN, H_DTIN, H_DVIN, H_TOUT, H_VOUT, H_DTOUT, H_DVOUT, H_WEPL, H_NF };

/* ------------------------------------------------------------------ hull */
/* Interval [ua, ub] of beam-axis coordinate u over which the straight line
 * t(u) = t_ref + st (u - u_ref), v(u) = v_ref + sv (u - u_ref) lies inside the
 * elliptic cylinder (x/a)^2 + (y/b)^2 <= 1, zmin <= z <= zmax.  Returns 0 on a
 * miss. */
static int hull_interval(const orc_geom *g, double phi, double u_ref, double t_ref, double v_ref,
                         double st, double sv, double *ua, double *ub) {
    double c = cos(phi), s = sin(phi);
    double T = t_ref - st * u_ref;  /* t at u = 0 */
    double V = v_ref - sv * u_ref;
    /* x(u) = px u + qx, y(u) = py u + qy */
    double px = c - st * s, qx = -T * s;
    double py = s + st * c, qy = T * c;
    double ia2 = 1.0 / (g->hull_a * g->hull_a), ib2 = 1.0 / (g->hull_b * g->hull_b);
    double A = px * px * ia2 + py * py * ib2;
    double B = 2.0 * (px * qx * ia2 + py * qy * ib2);
    double C = qx * qx * ia2 + qy * qy * ib2 - 1.0;
    double disc = B * B - 4.0 * A * C;
    if (A <= 0.0 || disc <= 0.0) return 0;
    double sq = sqrt(disc);
    double lo = (-B - sq) / (2.0 * A), hi = (-B + sq) / (2.0 * A);
    /* z slab */
    if (sv != 0.0) {
        double z0 = (g->hull_zmin - V) / sv, z1 = (g->hull_zmax - V) / sv;
        if (z0 > z1) { double tmp = z0; z0 = z1; z1 = tmp; }
        if (z0 > lo) lo = z0;
        if (z1 < hi) hi = z1;
    } else if (V < g->hull_zmin || V > g->hull_zmax) {
        return 0;
    }
    if (hi <= lo) return 0;
    *ua = lo;
    *ub = hi;
    return 1;
}

/* --------------------------------------------------------- scattering prior */
/* 8-point Gauss-Legendre rule on [-1, 1] (exact for polynomials of degree 15). */
static const double GL_X[8] = {-0.9602898564975363, -0.7966664774136267, -0.5255324099163290, -0.1834346424956498,
                               0.1834346424956498, 0.5255324099163290, 0.7966664774136267, 0.9602898564975363};
static const double GL_W[8] = {0.1012285362903763, 0.2223810344533745, 0.3137066458778873, 0.3626837833783620,
                               0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763};

static double prior_f(const orc_geom *g, double s) {
    double acc = 0.0, p = 1.0;
    for (int n = 0; n < g->n_poly; ++n) {
        acc += g->poly[n] * p;
        p *= s;
    }
    return acc;
}

/* out[m] = integral over s in [a, b] of f(s) (e - s)^m, m = 0, 1, 2 */
static void prior_moments(const orc_geom *g, double a, double b, double e, double out[3]) {
    double half = 0.5 * (b - a), mid = 0.5 * (a + b);
    out[0] = out[1] = out[2] = 0.0;
    for (int q = 0; q < 8; ++q) {
        double s = mid + half * GL_X[q];
        double w = GL_W[q] * half * prior_f(g, s);
        double r = e - s;
        out[0] += w;
        out[1] += w * r;
        out[2] += w * r * r;
    }
}

static double highland_g(const orc_geom *g, double d) {
    if (!g->highland_log) return 1.0;
    double h = 1.0 + 0.038 * log(d / g->X0);
    return h * h;
}

/* 2x2 helpers, row-major [a b; c d] */
static void inv2(const double m[4], double o[4]) {
    double det = m[0] * m[3] - m[1] * m[2];
    o[0] = m[3] / det;
    o[1] = -m[1] / det;
    o[2] = -m[2] / det;
    o[3] = m[0] / det;
}
static void mul2(const double a[4], const double b[4], double o[4]) {
    double r0 = a[0] * b[0] + a[1] * b[2], r1 = a[0] * b[1] + a[1] * b[3];
    double r2 = a[2] * b[0] + a[3] * b[2], r3 = a[2] * b[1] + a[3] * b[3];
    o[0] = r0; o[1] = r1; o[2] = r2; o[3] = r3;
}
static void mv2(const double a[4], const double v[2], double o[2]) {
    double r0 = a[0] * v[0] + a[1] * v[1], r1 = a[2] * v[0] + a[3] * v[1];
    o[0] = r0; o[1] = r1;
}

/* ------------------------------------------------------------------- MLP */
/*
 * Most-likely path of one history, sampled at u_k = u0 + k L / K, k = 0..K,
 * L = u2 - u0, K = max(1, ceil(L / step - 1e-9)), where u0 is where the entry
 * line meets the hull first and u2 where the exit line leaves it last.
 * At interior samples, per lateral plane with state y = (offset, slope):
 *   y = (S1^-1 + R1^T S2^-1 R1)^-1 (S1^-1 R0 y0 + R1^T S2^-1 y2),
 *   R0 = [1 d1; 0 1], R1 = [1 L-d1; 0 1], d1 = u - u0,
 *   S1 = E0^2/X0 g(d1)   * [I2 I1; I1 I0],  Im = int_0^d1  f(s) (d1 - s)^m ds,
 *   S2 = E0^2/X0 g(L-d1) * [J2 J1; J1 J0],  Jm = int_d1^L  f(s) (L - s)^m ds,
 * f = 1/(beta p)^2 as a polynomial in depth s from u0.  The end samples are
 * the hull states y0 and y2 themselves.
 * Returns the number of samples K+1, 0 for an empty path, or -(K+1) when cap
 * is too small.
 */
int orc_mlp_path(const orc_geom *g, const double h[H_NF], int cap, double *uo, double *to, double *vo) {
    double phi = h[H_PHI];
    double u0a, u0b, u2a, u2b;
    for (int f = 0; f < H_NF; ++f)
        if (!isfinite(h[f])) return 0;
    if (!hull_interval(g, phi, g->u_in, h[H_TIN], h[H_VIN], h[H_DTIN], h[H_DVIN], &u0a, &u0b)) return 0;
    if (!hull_interval(g, phi, g->u_out, h[H_TOUT], h[H_VOUT], h[H_DTOUT], h[H_DVOUT], &u2a, &u2b)) return 0;
    double u0 = u0a, u2 = u2b;
    double L = u2 - u0;
    if (!(L > 0.0)) return 0;
    int K = (int)ceil(L / g->step - 1e-9);
    if (K < 1) K = 1;
    if (K + 1 > cap) return -(K + 1);
    double y0t[2] = {h[H_TIN] + h[H_DTIN] * (u0 - g->u_in), h[H_DTIN]};
    double y0v[2] = {h[H_VIN] + h[H_DVIN] * (u0 - g->u_in), h[H_DVIN]};
    double y2t[2] = {h[H_TOUT] + h[H_DTOUT] * (u2 - g->u_out), h[H_DTOUT]};
    double y2v[2] = {h[H_VOUT] + h[H_DVOUT] * (u2 - g->u_out), h[H_DVOUT]};
    double csc = g->E0 * g->E0 / g->X0;
    for (int k = 0; k <= K; ++k) {
        double u = u0 + (double)k * L / (double)K;
        uo[k] = u;
        if (k == 0) { to[k] = y0t[0]; vo[k] = y0v[0]; continue; }
        if (k == K) { uo[k] = u2; to[k] = y2t[0]; vo[k] = y2v[0]; continue; }
        double d1 = u - u0;
        double I[3], J[3];
        prior_moments(g, 0.0, d1, d1, I);
        prior_moments(g, d1, L, L, J);
        double g1 = csc * highland_g(g, d1), g2 = csc * highland_g(g, L - d1);
        double S1[4] = {g1 * I[2], g1 * I[1], g1 * I[1], g1 * I[0]};
        double S2[4] = {g2 * J[2], g2 * J[1], g2 * J[1], g2 * J[0]};
        double R0[4] = {1.0, d1, 0.0, 1.0};
        double R1[4] = {1.0, L - d1, 0.0, 1.0};
        double R1T[4] = {1.0, 0.0, L - d1, 1.0};
        double S1i[4], S2i[4], tmp[4], Mm[4], Mi[4];
        inv2(S1, S1i);
        inv2(S2, S2i);
        mul2(R1T, S2i, tmp);      /* R1^T S2^-1 */
        mul2(tmp, R1, Mm);        /* R1^T S2^-1 R1 */
        for (int q = 0; q < 4; ++q) Mm[q] += S1i[q];
        inv2(Mm, Mi);
        double A1[4];
        mul2(S1i, R0, A1);        /* S1^-1 R0 */
        /* t plane */
        double a[2], b[2], r[2], y[2];
        mv2(A1, y0t, a);
        mv2(tmp, y2t, b);
        r[0] = a[0] + b[0]; r[1] = a[1] + b[1];
        mv2(Mi, r, y);
        to[k] = y[0];
        /* v plane */
        mv2(A1, y0v, a);
        mv2(tmp, y2v, b);
        r[0] = a[0] + b[0]; r[1] = a[1] + b[1];
        mv2(Mi, r, y);
        vo[k] = y[0];
    }
    return K + 1;
}

/* ------------------------------------------------------------- traversal */
typedef struct { int32_t j; double l; } piece_t;

static int cmp_double(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}
static int cmp_piece(const void *a, const void *b) {
    const piece_t *x = (const piece_t *)a, *y = (const piece_t *)b;
    return (x->j > y->j) - (x->j < y->j);
}

typedef struct { piece_t *p; int64_t n, cap; } pbuf_t;
static void pb_push(pbuf_t *b, int32_t j, double l) {
    if (b->n == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 1024;
        b->p = (piece_t *)realloc(b->p, (size_t)b->cap * sizeof(piece_t));
    }
    b->p[b->n].j = j;
    b->p[b->n].l = l;
    b->n++;
}

/* Siddon: exact intersection lengths of segment P->Q with the voxels. */
static void siddon_segment(const orc_grid *gr, const double P[3], const double Q[3], pbuf_t *out) {
    double gp[3] = {(P[0] - gr->ox) / gr->dx, (P[1] - gr->oy) / gr->dy, (P[2] - gr->oz) / gr->dz};
    double gq[3] = {(Q[0] - gr->ox) / gr->dx, (Q[1] - gr->oy) / gr->dy, (Q[2] - gr->oz) / gr->dz};
    double seg = sqrt((Q[0] - P[0]) * (Q[0] - P[0]) + (Q[1] - P[1]) * (Q[1] - P[1]) + (Q[2] - P[2]) * (Q[2] - P[2]));
    if (!(seg > 0.0)) return;
    int total = 2;
    for (int a = 0; a < 3; ++a) total += (int)fabs(ceil(gq[a]) - floor(gp[a])) + 2;
    double *alphas = (double *)malloc((size_t)total * sizeof(double));
    int na = 0;
    alphas[na++] = 0.0;
    alphas[na++] = 1.0;
    for (int a = 0; a < 3; ++a) {
        double lo = gp[a] < gq[a] ? gp[a] : gq[a];
        double hi = gp[a] < gq[a] ? gq[a] : gp[a];
        if (hi == lo) continue;
        for (double pl = floor(lo) + 1.0; pl < hi; pl += 1.0) {
            double al = (pl - gp[a]) / (gq[a] - gp[a]);
            if (al > 0.0 && al < 1.0 && na < total) alphas[na++] = al;
        }
    }
    qsort(alphas, (size_t)na, sizeof(double), cmp_double);
    int n[3] = {gr->nx, gr->ny, gr->nz};
    for (int q = 0; q + 1 < na; ++q) {
        double a0 = alphas[q], a1 = alphas[q + 1];
        if (!(a1 > a0)) continue;
        double am = 0.5 * (a0 + a1);
        int iv[3];
        int inside = 1;
        for (int a = 0; a < 3; ++a) {
            double c = gp[a] + am * (gq[a] - gp[a]);
            double fl = floor(c);
            if (fl < 0.0 || fl >= (double)n[a]) { inside = 0; break; }
            iv[a] = (int)fl;
        }
        if (!inside) continue;
        int32_t j = (int32_t)(((int64_t)iv[2] * gr->ny + iv[1]) * gr->nx + iv[0]);
        pb_push(out, j, (a1 - a0) * seg);
    }
    free(alphas);
}

/* Merge pieces per voxel (ascending index), drop sums below 1e-9 mm.
 * Returns the entry count; writes at most cap entries when idx != NULL. */
static int64_t merge_pieces(pbuf_t *b, int32_t *idx, double *len, int64_t cap, double *norm2) {
    if (b->n == 0) { if (norm2) *norm2 = 0.0; return 0; }
    qsort(b->p, (size_t)b->n, sizeof(piece_t), cmp_piece);
    int64_t cnt = 0;
    double n2 = 0.0;
    int64_t q = 0;
    while (q < b->n) {
        int32_t j = b->p[q].j;
        double s = 0.0;
        while (q < b->n && b->p[q].j == j) s += b->p[q++].l;
        if (s < 1e-9) continue;
        if (idx && cnt < cap) { idx[cnt] = j; len[cnt] = s; }
        n2 += s * s;
        cnt++;
    }
    if (norm2) *norm2 = n2;
    return cnt;
}

static void beam_to_object(double phi, double u, double t, double v, double P[3]) {
    double c = cos(phi), s = sin(phi);
    P[0] = u * c - t * s;
    P[1] = u * s + t * c;
    P[2] = v;
}

/* Row of an arbitrary polyline (object frame, npts x 3). */
int64_t orc_polyline_row(const orc_grid *gr, int32_t npts, const double *xyz, int32_t *idx, double *len,
                         int64_t cap, double *norm2) {
    pbuf_t b = {0, 0, 0};
    for (int k = 0; k + 1 < npts; ++k) siddon_segment(gr, &xyz[3 * k], &xyz[3 * (k + 1)], &b);
    int64_t c = merge_pieces(&b, idx, len, cap, norm2);
    free(b.p);
    return c;
}

static int64_t trace_one(const orc_grid *gr, const orc_geom *g, const double h[H_NF], int32_t *idx, double *len,
                         int64_t cap, double *norm2, double **wk, int *wcap) {
    int np;
    for (;;) {
        np = orc_mlp_path(g, h, *wcap, wk[0], wk[1], wk[2]);
        if (np >= 0) break;
        *wcap = -np + 16;
        for (int q = 0; q < 3; ++q) wk[q] = (double *)realloc(wk[q], (size_t)(*wcap) * sizeof(double));
    }
    if (np == 0) { if (norm2) *norm2 = 0.0; return 0; }
    pbuf_t b = {0, 0, 0};
    double P[3], Q[3];
    beam_to_object(h[H_PHI], wk[0][0], wk[1][0], wk[2][0], P);
    for (int k = 1; k < np; ++k) {
        beam_to_object(h[H_PHI], wk[0][k], wk[1][k], wk[2][k], Q);
        siddon_segment(gr, P, Q, &b);
        P[0] = Q[0]; P[1] = Q[1]; P[2] = Q[2];
    }
    int64_t c = merge_pieces(&b, idx, len, cap, norm2);
    free(b.p);
    return c;
}

/*
 * Rows of A for n histories (float32 SoA, field order phi, t_in, v_in,
 * dt_in, dv_in, t_out, v_out, dt_out, dv_out, wepl).
 * Count mode (idx == NULL): fills row_ptr[0..n] and returns the total.
 * Fill mode: row_ptr must hold the counts from count mode; writes idx, len
 * (voxel index ascending) and norm2.  Rows are independent, so the OpenMP
 * loop does not change any result.
 */
int64_t orc_trace(const orc_grid *gr, const orc_geom *g, int64_t n, const float *const *hist, int64_t *row_ptr,
                  int32_t *idx, double *len, double *norm2, int32_t nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    if (idx == NULL) {
#ifdef _OPENMP
#pragma omp parallel
#endif
        {
            int wcap = 512;
            double *wk[3];
            for (int q = 0; q < 3; ++q) wk[q] = (double *)malloc((size_t)wcap * sizeof(double));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
            for (int64_t i = 0; i < n; ++i) {
                double h[H_NF];
                for (int f = 0; f < H_NF; ++f) h[f] = (double)hist[f][i];
                row_ptr[i + 1] = trace_one(gr, g, h, NULL, NULL, 0, NULL, wk, &wcap);
            }
            for (int q = 0; q < 3; ++q) free(wk[q]);
        }
        row_ptr[0] = 0;
        for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] += row_ptr[i];
        return row_ptr[n];
    }
#ifdef _OPENMP
#pragma omp parallel
#endif
    {
        int wcap = 512;
        double *wk[3];
        for (int q = 0; q < 3; ++q) wk[q] = (double *)malloc((size_t)wcap * sizeof(double));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
        for (int64_t i = 0; i < n; ++i) {
            double h[H_NF];
            for (int f = 0; f < H_NF; ++f) h[f] = (double)hist[f][i];
            int64_t cap = row_ptr[i + 1] - row_ptr[i];
            trace_one(gr, g, h, idx + row_ptr[i], len + row_ptr[i], cap, &norm2[i], wk, &wcap);
        }
        for (int q = 0; q < 3; ++q) free(wk[q]);
    }
    return row_ptr[n];
}

/* ------------------------------------------- total-variation superiorization */
/*
 * TVS (Sec. 4.2, the Table 2 discussion: both pipelines perturb the image
 * towards lower total variation; DROP does it to the image entering every
 * block, CARP once at the start of every iteration).  The paper gives no
 * formula; this follows the superiorization scheme of the pCT literature it
 * builds on (Penfold et al. 2010), in 3D:
 *   TV(x)  = sum over voxels v of sqrt(dx_v^2 + dy_v^2 + dz_v^2 + eps^2),
 *            d*_v = x(v + e_*) - x(v) (forward difference; 0 at the grid's
 *            last plane on that axis);
 *   g      = dTV/dx (zeroed outside the mask), v = -g / ||g||_2;
 *   one step: try z = x + beta v, then beta <- a beta; accept z if
 *            TV(z) <= TV(x), else try again with the smaller beta, at most
 *            max_trials times.  beta keeps shrinking from call to call, so
 *            the perturbations are summable.
 */
typedef struct {
    int32_t n_steps;      /* perturbation steps per call */
    int32_t max_trials;   /* step sizes tried per step */
    double a;             /* beta factor per trial, 0 < a < 1 */
    double eps;           /* smoothing of the TV norm */
} orc_tvs;

static double tv_term(const orc_grid *gr, const double *x, int64_t i, int64_t j, int64_t k, double eps) {
    int64_t nx = gr->nx, ny = gr->ny, nz = gr->nz;
    int64_t v = (k * ny + j) * nx + i;
    double dx = (i + 1 < nx) ? x[v + 1] - x[v] : 0.0;
    double dy = (j + 1 < ny) ? x[v + nx] - x[v] : 0.0;
    double dz = (k + 1 < nz) ? x[v + nx * ny] - x[v] : 0.0;
    return sqrt(dx * dx + dy * dy + dz * dz + eps * eps);
}

double orc_tv(const orc_grid *gr, const double *x, double eps) {
    double acc = 0.0;
    for (int64_t k = 0; k < gr->nz; ++k)
        for (int64_t j = 0; j < gr->ny; ++j)
            for (int64_t i = 0; i < gr->nx; ++i) acc += tv_term(gr, x, i, j, k, eps);
    return acc;
}

/* g = dTV/dx: voxel u enters its own term (as -d*_u) and the terms of its
 * three lower neighbours (as +d*_{u - e_*}) */
void orc_tv_grad(const orc_grid *gr, const double *x, double eps, double *g) {
    int64_t nx = gr->nx, ny = gr->ny, nz = gr->nz;
    int64_t M = nx * ny * nz;
    for (int64_t u = 0; u < M; ++u) g[u] = 0.0;
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t v = (k * ny + j) * nx + i;
                double dx = (i + 1 < nx) ? x[v + 1] - x[v] : 0.0;
                double dy = (j + 1 < ny) ? x[v + nx] - x[v] : 0.0;
                double dz = (k + 1 < nz) ? x[v + nx * ny] - x[v] : 0.0;
                double phi = sqrt(dx * dx + dy * dy + dz * dz + eps * eps);
                g[v] -= (dx + dy + dz) / phi;
                if (i + 1 < nx) g[v + 1] += dx / phi;
                if (j + 1 < ny) g[v + nx] += dy / phi;
                if (k + 1 < nz) g[v + nx * ny] += dz / phi;
            }
}

/* TVS steps on x (mask: voxels that may change; NULL = all).  *beta is the
 * current step size, updated in place.  Returns the number of accepted steps. */
int orc_tvs_apply(const orc_grid *gr, const orc_tvs *t, const uint8_t *mask, double *x, double *beta) {
    int64_t M = (int64_t)gr->nx * gr->ny * gr->nz;
    double *g = (double *)malloc((size_t)M * sizeof(double));
    double *z = (double *)malloc((size_t)M * sizeof(double));
    int accepted = 0;
    for (int s = 0; s < t->n_steps; ++s) {
        orc_tv_grad(gr, x, t->eps, g);
        double nrm = 0.0;
        for (int64_t u = 0; u < M; ++u) {
            if (mask && !mask[u]) g[u] = 0.0;
            nrm += g[u] * g[u];
        }
        nrm = sqrt(nrm);
        if (!(nrm > 0.0)) break;
        double tvx = orc_tv(gr, x, t->eps);
        for (int trial = 0; trial < t->max_trials; ++trial) {
            double bt = *beta;
            *beta *= t->a;
            for (int64_t u = 0; u < M; ++u) z[u] = x[u] - bt * g[u] / nrm;
            if (orc_tv(gr, z, t->eps) <= tvx) {
                memcpy(x, z, (size_t)M * sizeof(double));
                accepted++;
                break;
            }
        }
    }
    free(g);
    free(z);
    return accepted;
}

/* --------------------------------------------------------------- solvers */
/*
 * Block-iterative row projection (DROP, paper Sec. 2.1).  The rows are taken
 * in the order `order`, in consecutive blocks of `block` rows (the last block
 * may be short).  For each block, with x fixed at its value at block start:
 *   r_i   = (b_i - a_i . x) / ||a_i||^2           for every row i of the block,
 *   num_j = sum_i r_i a_ij,   s_j = #{i in block : a_ij > 0},
 *   x_j  += lambda num_j / s_j                     for s_j > 0 and mask_j = 1;
 * voxels with mask_j = 0 are held at zero.  The next block starts from the
 * result; after the last block a new sweep starts from the same order.
 * block = 1 is ART (Kaczmarz).  Empty rows are skipped.  If resid is given,
 * ||Ax - b||_2 over the non-empty rows is stored after every sweep.
 */
static double residual_norm(int64_t n, const int64_t *row_ptr, const int32_t *idx, const double *len,
                            const double *b, const double *x) {
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (row_ptr[i + 1] == row_ptr[i]) continue;
        double d = 0.0;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) d += len[e] * x[idx[e]];
        acc += (d - b[i]) * (d - b[i]);
    }
    return sqrt(acc);
}

double orc_residual(int64_t n, const int64_t *row_ptr, const int32_t *idx, const double *len, const double *b,
                    const double *x) {
    return residual_norm(n, row_ptr, idx, len, b, x);
}

/*
 * The update of one block of nb rows (entries by ascending voxel):
 *   num_j = sum_q r_q a_qj,  s_j = #{q : a_qj > 0},  x_j += lambda num_j / s_j
 * for s_j > 0 and mask_j = 1; num and cnt are left at zero.  Threads own
 * disjoint voxel ranges and each walks the rows in block order, so every
 * voxel's sums run in block order whatever the thread count (the result is
 * that of the plain sequential loop).
 */
static void scatter_apply(int64_t nb, int32_t *const *ridx, double *const *rlen, const int64_t *rcnt,
                          const double *r, double lambda, const uint8_t *mask, int64_t M, double *x, double *num,
                          int64_t *cnt, uint8_t *touched) {
#ifdef _OPENMP
#pragma omp parallel
#endif
    {
        int T = 1, t = 0;
#ifdef _OPENMP
        T = omp_get_num_threads();
        t = omp_get_thread_num();
#endif
        int64_t j0 = M * t / T, j1 = M * (t + 1) / T;
        for (int64_t q = 0; q < nb; ++q) {
            const int32_t *ix = ridx[q];
            int64_t lo = 0, hi = rcnt[q];
            while (lo < hi) {   /* first entry with voxel >= j0 */
                int64_t mid = (lo + hi) / 2;
                if (ix[mid] < j0) lo = mid + 1; else hi = mid;
            }
            for (int64_t e = lo; e < rcnt[q] && ix[e] < j1; ++e) {
                num[ix[e]] += r[q] * rlen[q][e];
                cnt[ix[e]] += 1;
            }
        }
        for (int64_t j = j0; j < j1; ++j) {
            if (cnt[j] == 0) continue;
            if (touched) touched[j] = 1;
            if (!mask || mask[j]) x[j] += lambda * num[j] / (double)cnt[j];
            num[j] = 0.0;
            cnt[j] = 0;
        }
    }
}

/* ||Ax - b||_2 over the non-empty rows: squares per row (in parallel), summed
 * by row index */
static double residual_norm_par(int64_t n, const int64_t *row_ptr, const int32_t *idx, const double *len,
                                const double *b, const double *x) {
    double *sq = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int64_t i = 0; i < n; ++i) {
        sq[i] = -1.0;
        if (row_ptr[i + 1] == row_ptr[i]) continue;
        double d = 0.0;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) d += len[e] * x[idx[e]];
        sq[i] = (d - b[i]) * (d - b[i]);
    }
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i)
        if (sq[i] >= 0.0) acc += sq[i];
    free(sq);
    return sqrt(acc);
}

/* scratch of a stored-row DROP sweep */
typedef struct {
    double *num, *r;
    int64_t *cnt;
    int32_t **ridx;
    double **rlen;
    int64_t *rcnt;
} drop_work;

static drop_work drop_work_alloc(int64_t M, int64_t block) {
    drop_work w;
    w.num = (double *)calloc((size_t)M, sizeof(double));
    w.cnt = (int64_t *)calloc((size_t)M, sizeof(int64_t));
    w.r = (double *)malloc((size_t)block * sizeof(double));
    w.ridx = (int32_t **)malloc((size_t)block * sizeof(int32_t *));
    w.rlen = (double **)malloc((size_t)block * sizeof(double *));
    w.rcnt = (int64_t *)malloc((size_t)block * sizeof(int64_t));
    return w;
}

static void drop_work_free(drop_work *w) {
    free(w->num);
    free(w->cnt);
    free(w->r);
    free(w->ridx);
    free(w->rlen);
    free(w->rcnt);
}

/*
 * One DROP sweep over the rows at positions [p0, p1) of `order`, in
 * consecutive blocks of `block` positions from p0.  With tvs given, the TVS
 * steps are applied to the image that enters each block.  touched (or NULL):
 * set to 1 for every voxel some row of the range touches.
 */
static void drop_sweep_range(const int64_t *row_ptr, const int32_t *idx, const double *len, const double *norm2,
                             const double *b, const int64_t *order, int64_t p0, int64_t p1, int64_t block,
                             double lambda, const uint8_t *mask, int64_t M, double *x, drop_work *w,
                             const orc_grid *gr, const orc_tvs *tvs, double *beta, uint8_t *touched) {
    for (int64_t b0 = p0; b0 < p1; b0 += block) {
        int64_t nb = (p1 - b0 < block) ? p1 - b0 : block;
        if (tvs) orc_tvs_apply(gr, tvs, mask, x, beta);
        /* projections against x at block start */
#ifdef _OPENMP
#pragma omp parallel for schedule(static) if (nb > 4096)
#endif
        for (int64_t q = 0; q < nb; ++q) {
            int64_t i = order[b0 + q];
            w->ridx[q] = (int32_t *)idx + row_ptr[i];
            w->rlen[q] = (double *)len + row_ptr[i];
            w->rcnt[q] = row_ptr[i + 1] - row_ptr[i];
            if (w->rcnt[q] == 0) { w->r[q] = 0.0; continue; }
            double d = 0.0;
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) d += len[e] * x[idx[e]];
            w->r[q] = (b[i] - d) / norm2[i];
        }
        scatter_apply(nb, w->ridx, w->rlen, w->rcnt, w->r, lambda, mask, M, x, w->num, w->cnt, touched);
    }
}

int orc_drop(int64_t n, const int64_t *row_ptr, const int32_t *idx, const double *len, const double *norm2,
             const double *b, const int64_t *order, int64_t block, double lambda, const uint8_t *mask, int64_t M,
             int32_t sweeps, double *x, double *resid, int32_t nthreads) {
    if (block < 1) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    drop_work w = drop_work_alloc(M, block);
    if (mask)
        for (int64_t j = 0; j < M; ++j)
            if (!mask[j]) x[j] = 0.0;
    for (int32_t sw = 0; sw < sweeps; ++sw) {
        drop_sweep_range(row_ptr, idx, len, norm2, b, order, 0, n, block, lambda, mask, M, x, &w, NULL, NULL, NULL,
                         NULL);
        if (resid) resid[sw] = residual_norm_par(n, row_ptr, idx, len, b, x);
    }
    drop_work_free(&w);
    return 0;
}

/* DROP with the TVS steps before every block (Sec. 4.2); *beta as in
 * orc_tvs_apply, carried across blocks and sweeps. */
int orc_drop_tvs(const orc_grid *gr, int64_t n, const int64_t *row_ptr, const int32_t *idx, const double *len,
                 const double *norm2, const double *b, const int64_t *order, int64_t block, double lambda,
                 const uint8_t *mask, int32_t sweeps, const orc_tvs *tvs, double *beta, double *x, double *resid,
                 int32_t nthreads) {
    if (block < 1 || !tvs) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int64_t M = (int64_t)gr->nx * gr->ny * gr->nz;
    drop_work w = drop_work_alloc(M, block);
    if (mask)
        for (int64_t j = 0; j < M; ++j)
            if (!mask[j]) x[j] = 0.0;
    for (int32_t sw = 0; sw < sweeps; ++sw) {
        drop_sweep_range(row_ptr, idx, len, norm2, b, order, 0, n, block, lambda, mask, M, x, &w, gr, tvs, beta,
                         NULL);
        if (resid) resid[sw] = residual_norm_par(n, row_ptr, idx, len, b, x);
    }
    drop_work_free(&w);
    return 0;
}

/*
 * CARP (Sec. 2.2, component-averaged row projections; Gordon & Gordon
 * 2005): the positions of `order` are split into n_strings consecutive
 * strings, string s = [n s / S, n (s+1) / S).  Every iteration each string
 * starts from the same x and runs one DROP sweep over its own rows (blocks
 * of `block` positions from the string's start) into its own image x_s;
 * then every voxel becomes the mean of x_s over the strings whose rows touch
 * it (voxels no string touches keep their value).  With tvs given, the TVS
 * steps are applied once to x at the start of every iteration.
 */
int orc_carp(const orc_grid *gr, int64_t n, const int64_t *row_ptr, const int32_t *idx, const double *len,
             const double *norm2, const double *b, const int64_t *order, int32_t n_strings, int64_t block,
             double lambda, const uint8_t *mask, int32_t iters, const orc_tvs *tvs, double *beta, double *x,
             double *resid, int32_t nthreads) {
    if (block < 1 || n_strings < 1) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int64_t M = (int64_t)gr->nx * gr->ny * gr->nz;
    drop_work w = drop_work_alloc(M, block);
    double *xs = (double *)malloc((size_t)M * sizeof(double));
    double *acc = (double *)malloc((size_t)M * sizeof(double));
    int32_t *tc = (int32_t *)malloc((size_t)M * sizeof(int32_t));
    uint8_t *touched = (uint8_t *)malloc((size_t)M);
    if (mask)
        for (int64_t j = 0; j < M; ++j)
            if (!mask[j]) x[j] = 0.0;
    for (int32_t it = 0; it < iters; ++it) {
        if (tvs) orc_tvs_apply(gr, tvs, mask, x, beta);
        memset(acc, 0, (size_t)M * sizeof(double));
        memset(tc, 0, (size_t)M * sizeof(int32_t));
        for (int32_t s = 0; s < n_strings; ++s) {
            int64_t p0 = n * s / n_strings, p1 = n * (s + 1) / n_strings;
            memcpy(xs, x, (size_t)M * sizeof(double));
            memset(touched, 0, (size_t)M);
            drop_sweep_range(row_ptr, idx, len, norm2, b, order, p0, p1, block, lambda, mask, M, xs, &w, NULL, NULL,
                             NULL, touched);
            for (int64_t j = 0; j < M; ++j)
                if (touched[j]) {
                    acc[j] += xs[j];
                    tc[j] += 1;
                }
        }
        for (int64_t j = 0; j < M; ++j)
            if (tc[j] > 0) x[j] = acc[j] / (double)tc[j];
        if (resid) resid[it] = residual_norm_par(n, row_ptr, idx, len, b, x);
    }
    drop_work_free(&w);
    free(xs);
    free(acc);
    free(tc);
    free(touched);
    return 0;
}

/* --------------------------------------------------- DROP without stored A */
/*
 * The same block-iterative projections as orc_drop, for the case the paper
 * raises in Sec. 2 and Sec. 4.1 (A of 10^8-10^9 rows too large to keep): each
 * block's rows are traced from the histories just before the block is
 * projected and then discarded, and the residual after a sweep traces every
 * row once more.  Every row is the same as orc_trace makes it and every sum
 * runs in the same order as orc_drop's (entries by ascending voxel, rows in
 * block order for the scatter, rows by index for the residual), so given the
 * same histories the result equals orc_drop on orc_trace's rows.
 */
typedef struct { int32_t *idx; double *len; int64_t cnt; double n2; } orc_row_t;

/* row of history i, in freshly allocated arrays (caller frees) */
static void trace_owned(const orc_grid *gr, const orc_geom *g, const float *const *hist, int64_t i, orc_row_t *r,
                        double **wk, int *wcap) {
    double h[H_NF];
    for (int f = 0; f < H_NF; ++f) h[f] = (double)hist[f][i];
    int64_t cap = 512;
    for (;;) {
        r->idx = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
        r->len = (double *)malloc((size_t)cap * sizeof(double));
        r->cnt = trace_one(gr, g, h, r->idx, r->len, cap, &r->n2, wk, wcap);
        if (r->cnt <= cap) return;
        free(r->idx);
        free(r->len);
        cap = r->cnt;
    }
}

int orc_drop_recompute(const orc_grid *gr, const orc_geom *g, int64_t n, const float *const *hist,
                       const int64_t *order, int64_t block, double lambda, const uint8_t *mask, int64_t M,
                       int32_t sweeps, double *x, double *resid, int32_t nthreads) {
    if (block < 1) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    double *num = (double *)calloc((size_t)M, sizeof(double));
    int64_t *cnt = (int64_t *)calloc((size_t)M, sizeof(int64_t));
    double *r = (double *)malloc((size_t)block * sizeof(double));
    int32_t **ridx = (int32_t **)malloc((size_t)block * sizeof(int32_t *));
    double **rlen = (double **)malloc((size_t)block * sizeof(double *));
    int64_t *rcnt = (int64_t *)malloc((size_t)block * sizeof(int64_t));
    orc_row_t *rows = (orc_row_t *)calloc((size_t)block, sizeof(orc_row_t));
    if (mask)
        for (int64_t j = 0; j < M; ++j)
            if (!mask[j]) x[j] = 0.0;
    for (int32_t sw = 0; sw < sweeps; ++sw) {
        for (int64_t b0 = 0; b0 < n; b0 += block) {
            int64_t nb = (n - b0 < block) ? n - b0 : block;
            /* trace the block's rows, then project them against x at block start */
#ifdef _OPENMP
#pragma omp parallel
#endif
            {
                int wcap = 512;
                double *wk[3];
                for (int q = 0; q < 3; ++q) wk[q] = (double *)malloc((size_t)wcap * sizeof(double));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
                for (int64_t q = 0; q < nb; ++q) {
                    int64_t i = order[b0 + q];
                    trace_owned(gr, g, hist, i, &rows[q], wk, &wcap);
                    if (rows[q].cnt == 0) { r[q] = 0.0; continue; }
                    double d = 0.0;
                    for (int64_t e = 0; e < rows[q].cnt; ++e) d += rows[q].len[e] * x[rows[q].idx[e]];
                    r[q] = ((double)hist[H_WEPL][i] - d) / rows[q].n2;
                }
                for (int q = 0; q < 3; ++q) free(wk[q]);
            }
            /* accumulate in block order, then update */
            for (int64_t q = 0; q < nb; ++q) {
                ridx[q] = rows[q].idx;
                rlen[q] = rows[q].len;
                rcnt[q] = rows[q].cnt;
            }
            scatter_apply(nb, ridx, rlen, rcnt, r, lambda, mask, M, x, num, cnt, NULL);
            for (int64_t q = 0; q < nb; ++q) {
                free(rows[q].idx);
                free(rows[q].len);
                rows[q].idx = NULL;
                rows[q].len = NULL;
            }
        }
        if (resid) {
            /* (a_i . x - b_i)^2 per row with its row traced again, summed by row index */
            double *sq = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
#ifdef _OPENMP
#pragma omp parallel
#endif
            {
                int wcap = 512;
                double *wk[3];
                for (int q = 0; q < 3; ++q) wk[q] = (double *)malloc((size_t)wcap * sizeof(double));
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
                for (int64_t i = 0; i < n; ++i) {
                    orc_row_t rw;
                    trace_owned(gr, g, hist, i, &rw, wk, &wcap);
                    sq[i] = -1.0;
                    if (rw.cnt > 0) {
                        double d = 0.0;
                        for (int64_t e = 0; e < rw.cnt; ++e) d += rw.len[e] * x[rw.idx[e]];
                        double dd = d - (double)hist[H_WEPL][i];
                        sq[i] = dd * dd;
                    }
                    free(rw.idx);
                    free(rw.len);
                }
                for (int q = 0; q < 3; ++q) free(wk[q]);
            }
            double acc = 0.0;
            for (int64_t i = 0; i < n; ++i)
                if (sq[i] >= 0.0) acc += sq[i];
            resid[sw] = sqrt(acc);
            free(sq);
        }
    }
    free(rows);
    free(num);
    free(cnt);
    free(r);
    free(ridx);
    free(rlen);
    free(rcnt);
    return 0;
}


/* ------------------------------------------------------ space-carving hull */
/*
 * Hull from the data (the configurations' "hull" when no analytic outline is
 * known): a proton whose WEPL is below wepl_max crossed only air, so every
 * voxel its straight line (the entry tracker's position and slope, from
 * u_in to u_out) passes through for more than min_len mm lies outside the
 * object and is carved (carved[j] = 1; the caller zeroes the array).  The
 * line is cut into voxel pieces by Siddon's method, as for the rows.
 * Returns the number of histories used.
 */
int64_t orc_carve(const orc_grid *gr, const orc_geom *g, int64_t n, const float *const *hist, double wepl_max,
                  double min_len, uint8_t *carved, int32_t nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int64_t used = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : used)
#endif
    for (int64_t i = 0; i < n; ++i) {
        double h[H_NF];
        int fin = 1;
        for (int f = 0; f < H_NF; ++f) {
            h[f] = (double)hist[f][i];
            fin = fin && isfinite(h[f]);
        }
        if (!fin || !(h[H_WEPL] < wepl_max)) continue;
        used++;
        double P[3], Q[3];
        double u0 = g->u_in, u1 = g->u_out;
        beam_to_object(h[H_PHI], u0, h[H_TIN], h[H_VIN], P);
        beam_to_object(h[H_PHI], u1, h[H_TIN] + h[H_DTIN] * (u1 - u0), h[H_VIN] + h[H_DVIN] * (u1 - u0), Q);
        pbuf_t b = {0, 0, 0};
        siddon_segment(gr, P, Q, &b);
        for (int64_t q = 0; q < b.n; ++q)
            if (b.p[q].l > min_len) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
                carved[b.p[q].j] = 1;
            }
        free(b.p);
    }
    return used;
}
