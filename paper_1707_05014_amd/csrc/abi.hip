// C ABI of libpct.so: argument validation, workspace carving, kernel order.
// The operations are defined in include/pct.h; see there for ownership,
// layouts and error behaviour.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pct_internal.h"

namespace {

thread_local std::string g_err;

// ---- optional kernel timing (pct_profile_enable / pct_profile_read)
struct ProfRec {
  int kind;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_prof_pool;

hipEvent_t prof_event() {
  if (!g_prof_pool.empty()) {
    hipEvent_t e = g_prof_pool.back();
    g_prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// brackets one launch: records a start event now and a stop event at stop()
struct ProfScope {
  int kind;
  hipStream_t s;
  hipEvent_t a = nullptr;
  ProfScope(int k, hipStream_t st) : kind(k), s(st) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (!g_prof_on) return;
    a = prof_event();
    if (a) hipEventRecord(a, s);
  }
  void stop() {
    if (!a) return;
    std::lock_guard<std::mutex> g(g_prof_mu);
    hipEvent_t b = prof_event();
    if (!b) return;
    hipEventRecord(b, s);
    g_prof.push_back({kind, a, b});
    a = nullptr;
  }
};

#define PROF(kind, expr)                  \
  do {                                    \
    ProfScope ps_((kind), c.s);           \
    hipError_t pe_ = (expr);              \
    ps_.stop();                           \
    HIPCHECK(pe_);                        \
  } while (0)

pct_status fail(pct_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
pct_status fail(pct_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHECK(expr)                                                                         \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return fail(PCT_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));    \
  } while (0)

inline size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

int64_t grid_voxels(const pct_grid *g) { return (int64_t)g->nx * g->ny * g->nz; }

pct_status check_grid(const pct_grid *g) {
  if (!g) return fail(PCT_EINVAL, "grid is NULL");
  if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0) return fail(PCT_EINVAL, "grid dimensions must be positive");
  if (!(g->dx > 0.f && g->dy > 0.f && g->dz > 0.f)) return fail(PCT_EINVAL, "voxel sizes must be positive");
  if (!(std::isfinite(g->ox) && std::isfinite(g->oy) && std::isfinite(g->oz)))
    return fail(PCT_EINVAL, "grid origin must be finite");
  if (grid_voxels(g) > 0x7fffffffLL) return fail(PCT_EINVAL, "grid has more than 2^31-1 voxels");
  return PCT_OK;
}

pct_status check_hist(const pct_histories *h) {
  if (!h) return fail(PCT_EINVAL, "histories are NULL");
  if (h->n < 0) return fail(PCT_EINVAL, "history count is negative");
  if (h->n > 0 && (!h->phi || !h->t_in || !h->v_in || !h->dt_in || !h->dv_in || !h->t_out || !h->v_out ||
                   !h->dt_out || !h->dv_out || !h->wepl))
    return fail(PCT_EINVAL, "a history array is NULL");
  return PCT_OK;
}

pct_status make_params(const pct_grid *g, const pct_geom *G, pct::PathParams &P) {
  if (!G) return fail(PCT_EINVAL, "geometry is NULL");
  const float dmin = std::min(g->dx, std::min(g->dy, g->dz));
  if (!(G->step_mm > 0.f) || G->step_mm > dmin * (1.0f + 1e-6f))
    return fail(PCT_EINVAL, "step_mm must be in (0, min voxel size]");
  if (!(G->hull_a > 0.f && G->hull_b > 0.f) || !(G->hull_zmax > G->hull_zmin))
    return fail(PCT_EINVAL, "hull must have positive semi-axes and zmax > zmin");
  if (!(G->u_out > G->u_in)) return fail(PCT_EINVAL, "u_out must exceed u_in");
  if (G->n_poly < 1 || G->n_poly > 8) return fail(PCT_EINVAL, "n_poly must be 1..8");
  if (G->highland_log && !(G->X0_mm > 0.0)) return fail(PCT_EINVAL, "X0_mm must be positive");
  std::memset(&P, 0, sizeof P);
  P.u_in = G->u_in;
  P.u_out = G->u_out;
  P.hull_ia2 = 1.0 / ((double)G->hull_a * (double)G->hull_a);
  P.hull_ib2 = 1.0 / ((double)G->hull_b * (double)G->hull_b);
  P.hull_zmin = G->hull_zmin;
  P.hull_zmax = G->hull_zmax;
  P.step = G->step_mm;
  P.inv_step = 1.0f / G->step_mm;
  P.highland = G->highland_log ? 1 : 0;
  P.inv_X0 = G->highland_log ? (float)(1.0 / G->X0_mm) : 0.f;
  for (int n = 0; n < 8; ++n) {
    if (n < G->n_poly && !std::isfinite(G->poly[n])) return fail(PCT_EINVAL, "prior coefficient %d is not finite", n);
    const double an = n < G->n_poly ? G->poly[n] : 0.0;
    const double n1 = n + 1.0, n2 = n + 2.0, n3 = n + 3.0;
    const double ci[3] = {an / n1, an / (n1 * n2), 2.0 * an / (n1 * n2 * n3)};
    for (int m = 0; m < 3; ++m) {
      P.cI_d[m][n] = ci[m];
      P.cF_d[m][n] = an / (n + m + 1.0);
      P.cI_f[m][n] = (float)P.cI_d[m][n];
      P.cF_f[m][n] = (float)P.cF_d[m][n];
    }
  }
  if (G->path_fp32 != 0 && G->path_fp32 != 1) return fail(PCT_EINVAL, "path_fp32 must be 0 or 1");
  P.path_fp32 = G->path_fp32;
  P.nx = g->nx;
  P.ny = g->ny;
  P.nz = g->nz;
  P.dx = g->dx;
  P.dy = g->dy;
  P.dz = g->dz;
  P.idx = 1.0 / (double)g->dx;
  P.idy = 1.0 / (double)g->dy;
  P.idz = 1.0 / (double)g->dz;
  P.ox = g->ox;
  P.oy = g->oy;
  P.oz = g->oz;
  P.eps_len = 1e-6f * dmin;
  const double reach = 2.0 * std::max(G->hull_a, G->hull_b);
  P.kmax = (int32_t)std::ceil(reach / G->step_mm) + 2;
  P.emax = 4 * (P.kmax + 1) + 16;
  const size_t per_wave = (size_t)P.emax * 3 * sizeof(int);
  P.waves_per_block = (int32_t)std::min<size_t>(4, 65536 / per_wave);
  if (P.waves_per_block < 1)
    return fail(PCT_EINVAL, "hull too long for the sample step (row buffer exceeds the LDS budget)");
  return PCT_OK;
}

pct::HistPtrs hist_ptrs(const pct_histories *h) {
  return {h->phi, h->t_in, h->v_in, h->dt_in, h->dv_in, h->t_out, h->v_out, h->dt_out, h->dv_out, h->wepl};
}

pct_status check_rows(const pct_rows *r, int64_t n, bool need_data) {
  if (!r) return fail(PCT_EINVAL, "rows are NULL");
  if (r->n_rows != n) return fail(PCT_EINVAL, "rows.n_rows (%lld) != history count (%lld)", (long long)r->n_rows,
                                  (long long)n);
  if (!r->row_ptr) return fail(PCT_EINVAL, "rows.row_ptr is NULL");
  if (r->len_dtype != 0 && r->len_dtype != 1) return fail(PCT_EINVAL, "rows.len_dtype must be 0 or 1");
  if (need_data && (!r->idx || !r->len || !r->norm2)) return fail(PCT_EINVAL, "rows arrays are NULL");
  if (r->cap_nnz < 0) return fail(PCT_EINVAL, "rows.cap_nnz is negative");
  return PCT_OK;
}

pct_status check_params(const pct_sweep_params *p, bool cached) {
  if (!p) return fail(PCT_EINVAL, "params are NULL");
  if (p->algo != 0 && p->algo != 1) return fail(PCT_EINVAL, "algo must be 0 (ART) or 1 (DROP)");
  if (p->algo == 0 && !cached) return fail(PCT_EINVAL, "ART needs cached rows");
  if (p->algo == 1 && p->block_size < 1) return fail(PCT_EINVAL, "block_size must be >= 1");
  if (!(p->lambda > 0.f && p->lambda < 2.f)) return fail(PCT_EINVAL, "lambda must be in (0, 2)");
  if (p->n_sweeps < 0) return fail(PCT_EINVAL, "n_sweeps must be >= 0");
  return PCT_OK;
}

struct Ctx {
  pct::PathParams P;
  pct::HistPtrs H;
  pct::Workspace W;
  int64_t M, n;
  hipStream_t s;
};

pct_status check_ws(void *ws, size_t ws_bytes, int64_t M, int64_t n) {
  const size_t need = pct::workspace_bytes(M, n);
  if (!ws || ws_bytes < need)
    return fail(PCT_ENOMEM, "workspace of %zu bytes given, %zu needed", ws ? ws_bytes : (size_t)0, need);
  return PCT_OK;
}

pct_status read_status(Ctx &c, uint32_t *out) {
  HIPCHECK(hipMemcpyAsync(out, c.W.status, sizeof(uint32_t), hipMemcpyDeviceToHost, c.s));
  HIPCHECK(hipStreamSynchronize(c.s));
  return PCT_OK;
}

pct_status status_to_code(uint32_t st) {
  if (st & pct::kStOverflow) return fail(PCT_EDEVICE, "a row exceeded its device-side bound");
  if (st & pct::kStRowMismatch) return fail(PCT_EDEVICE, "fill pass disagreed with the count pass");
  if (st & pct::kStBadIndex) return fail(PCT_EINVAL, "order holds an entry outside [0, n) or rows hold a voxel outside [0, M)");
  if (st & pct::kStNonFinite) return fail(PCT_ENONFINITE, "histories with NaN/Inf were given empty rows");
  return PCT_OK;
}

pct_status do_trace(Ctx &c, pct_rows *rows) {
  HIPCHECK(pct::launch_fill_u32(c.W.status, 4, 0u, c.s));
  PROF(PCT_K_TRACE_COUNT,
       pct::launch_trace(c.P, c.H, c.n, 0, rows->row_ptr, nullptr, nullptr, 0, nullptr, c.W.status, c.s));
  HIPCHECK(pct::launch_scan_rows(rows->row_ptr, c.n, c.W.scan, c.s));
  int64_t total = 0;
  HIPCHECK(hipMemcpyAsync(&total, rows->row_ptr + c.n, sizeof total, hipMemcpyDeviceToHost, c.s));
  uint32_t st = 0;
  pct_status r = read_status(c, &st);
  if (r != PCT_OK) return r;
  rows->nnz = total;
  if (st & (pct::kStOverflow | pct::kStRowMismatch)) return status_to_code(st);
  if (!rows->idx) return status_to_code(st);
  if (total > rows->cap_nnz)
    return fail(PCT_EROWCAP, "rows need %lld entries, capacity is %lld", (long long)total,
                (long long)rows->cap_nnz);
  PROF(PCT_K_TRACE_FILL, pct::launch_trace(c.P, c.H, c.n, 1, rows->row_ptr, rows->idx, rows->len, rows->len_dtype,
                                            rows->norm2, c.W.status, c.s));
  r = read_status(c, &st);
  if (r != PCT_OK) return r;
  return status_to_code(st);
}

float len_unit(const pct_grid *g) { return std::min(g->dx, std::min(g->dy, g->dz)); }

pct_status do_sweep(Ctx &c, const pct_grid *g, const pct_rows *rows, float *x, const pct_sweep_params *p) {
  HIPCHECK(pct::launch_mask(x, p->hull_mask, c.M, c.s));
  const float unit = len_unit(g);
  if (p->algo == 0) {
    PROF(PCT_K_ART, pct::launch_art(rows->row_ptr, rows->idx, rows->len, rows->len_dtype, unit, rows->norm2,
                                    c.H.wepl, p->order, c.n, c.M, x, p->hull_mask, p->lambda, c.W.status, c.s));
    return PCT_OK;
  }
  HIPCHECK(pct::launch_fill_f32(c.W.num, c.M, 0.f, c.s));
  HIPCHECK(pct::launch_fill_u32(c.W.cnt, c.M, 0u, c.s));
  for (int64_t first = 0; first < c.n; first += p->block_size) {
    const int64_t count = std::min<int64_t>(p->block_size, c.n - first);
    if (rows)
      PROF(PCT_K_PROJECT, pct::launch_project_cached(rows->row_ptr, rows->idx, rows->len, rows->len_dtype, unit,
                                                     rows->norm2, c.H.wepl, p->order, first, count, c.n, c.M, x,
                                                     c.W.num, c.W.cnt, c.W.status, c.s));
    else
      PROF(PCT_K_PROJECT, pct::launch_project_fused(c.P, c.H, p->order, first, count, c.n, x, c.W.num, c.W.cnt,
                                                    c.W.status, c.s));
    PROF(PCT_K_APPLY, pct::launch_apply(x, c.W.num, c.W.cnt, p->hull_mask, c.M, p->lambda, c.s));
  }
  return PCT_OK;
}

pct_status do_residual(Ctx &c, const pct_grid *g, const pct_rows *rows, const float *x, double *out) {
  if (rows)
    PROF(PCT_K_RESIDUAL, pct::launch_residual_cached(rows->row_ptr, rows->idx, rows->len, rows->len_dtype,
                                                     len_unit(g), c.H.wepl, c.n, c.M, x, c.W.partials, out, c.s));
  else
    PROF(PCT_K_RESIDUAL, pct::launch_residual_fused(c.P, c.H, c.n, x, c.W.partials, c.W.status, out, c.s));
  return PCT_OK;
}

pct_status setup(Ctx &c, const pct_grid *grid, const pct_geom *geom, const pct_histories *hist, void *ws,
                  size_t ws_bytes, void *stream) {
  pct_status r;
  if ((r = check_grid(grid)) != PCT_OK) return r;
  if ((r = check_hist(hist)) != PCT_OK) return r;
  if ((r = make_params(grid, geom, c.P)) != PCT_OK) return r;
  c.M = grid_voxels(grid);
  c.n = hist->n;
  if ((r = check_ws(ws, ws_bytes, c.M, c.n)) != PCT_OK) return r;
  c.H = hist_ptrs(hist);
  c.W = pct::carve_workspace(ws, c.M, c.n);
  c.s = reinterpret_cast<hipStream_t>(stream);
  return PCT_OK;
}

}  // namespace

namespace pct {

size_t workspace_bytes(int64_t M, int64_t n_hist) {
  size_t b = align_up(4 * sizeof(uint32_t));
  b += align_up((size_t)M * sizeof(float));
  b += align_up((size_t)M * sizeof(uint32_t));
  b += align_up((size_t)kMaxPartials * sizeof(double));
  b += align_up((size_t)((n_hist + kScanChunk - 1) / kScanChunk + 2) * sizeof(int64_t));
  return b;
}

Workspace carve_workspace(void *base, int64_t M, int64_t n_hist) {
  char *p = static_cast<char *>(base);
  Workspace w;
  w.status = reinterpret_cast<uint32_t *>(p);
  p += align_up(4 * sizeof(uint32_t));
  w.num = reinterpret_cast<float *>(p);
  p += align_up((size_t)M * sizeof(float));
  w.cnt = reinterpret_cast<uint32_t *>(p);
  p += align_up((size_t)M * sizeof(uint32_t));
  w.partials = reinterpret_cast<double *>(p);
  p += align_up((size_t)kMaxPartials * sizeof(double));
  w.scan = reinterpret_cast<int64_t *>(p);
  (void)n_hist;
  return w;
}

}  // namespace pct

extern "C" {

size_t pct_workspace_size(const pct_grid *grid, const pct_geom *geom, const pct_sweep_params *params,
                          int64_t n_hist, int32_t fused) {
  (void)geom;
  (void)params;
  (void)fused;
  if (!grid || grid->nx <= 0 || grid->ny <= 0 || grid->nz <= 0 || n_hist < 0) return 0;
  return pct::workspace_bytes(grid_voxels(grid), n_hist);
}

pct_status pct_mlp_trace(const pct_grid *grid, const pct_geom *geom, const pct_histories *hist, pct_rows *rows,
                         void *workspace, size_t ws_bytes, void *stream) {
  g_err.clear();
  Ctx c;
  pct_status r = setup(c, grid, geom, hist, workspace, ws_bytes, stream);
  if (r != PCT_OK) return r;
  if ((r = check_rows(rows, c.n, false)) != PCT_OK) return r;
  if (rows->idx && (!rows->len || !rows->norm2)) return fail(PCT_EINVAL, "rows.len / rows.norm2 are NULL");
  return do_trace(c, rows);
}

pct_status pct_project_sweep(const pct_grid *grid, const pct_geom *geom, const pct_histories *hist,
                             const pct_rows *rows, float *x, const pct_sweep_params *params, double *resid_out,
                             void *workspace, size_t ws_bytes, void *stream) {
  g_err.clear();
  Ctx c;
  pct_status r = setup(c, grid, geom, hist, workspace, ws_bytes, stream);
  if (r != PCT_OK) return r;
  if (rows && (r = check_rows(rows, c.n, true)) != PCT_OK) return r;
  if ((r = check_params(params, rows != nullptr)) != PCT_OK) return r;
  if (!x) return fail(PCT_EINVAL, "x is NULL");
  HIPCHECK(pct::launch_fill_u32(c.W.status, 4, 0u, c.s));
  if ((r = do_sweep(c, grid, rows, x, params)) != PCT_OK) return r;
  if (resid_out) {
    if ((r = do_residual(c, grid, rows, x, resid_out)) != PCT_OK) return r;
    HIPCHECK(pct::launch_poison_on_status(resid_out, c.W.status, c.s));
  }
  return PCT_OK;
}

pct_status pct_reconstruct(const pct_grid *grid, const pct_geom *geom, const pct_histories *hist,
                           const pct_sweep_params *params, pct_rows *rows, float *x_inout, double *resid_host,
                           void *workspace, size_t ws_bytes, void *stream) {
  g_err.clear();
  Ctx c;
  pct_status r = setup(c, grid, geom, hist, workspace, ws_bytes, stream);
  if (r != PCT_OK) return r;
  if (rows && (r = check_rows(rows, c.n, true)) != PCT_OK) return r;
  if ((r = check_params(params, rows != nullptr)) != PCT_OK) return r;
  if (!x_inout) return fail(PCT_EINVAL, "x is NULL");
  pct_status trace_st = PCT_OK;
  if (rows) {
    trace_st = do_trace(c, rows);
    if (trace_st != PCT_OK && trace_st != PCT_ENONFINITE) return trace_st;
  } else {
    HIPCHECK(pct::launch_fill_u32(c.W.status, 4, 0u, c.s));
  }
  double *dres = c.W.partials + (pct::kMaxPartials - 1);
  for (int32_t sw = 0; sw < params->n_sweeps; ++sw) {
    if ((r = do_sweep(c, grid, rows, x_inout, params)) != PCT_OK) return r;
    if (resid_host) {
      // partial sums use the front of the array; the result sits in its last slot
      if ((r = do_residual(c, grid, rows, x_inout, dres)) != PCT_OK) return r;
      HIPCHECK(hipMemcpyAsync(&resid_host[sw], dres, sizeof(double), hipMemcpyDeviceToHost, c.s));
    }
  }
  uint32_t st = 0;
  if ((r = read_status(c, &st)) != PCT_OK) return r;
  r = status_to_code(st);
  if (r != PCT_OK) return r;
  return trace_st;
}

pct_status pct_residual(const pct_grid *grid, const pct_geom *geom, const pct_histories *hist,
                        const pct_rows *rows, const float *x, double *out, void *workspace, size_t ws_bytes,
                        void *stream) {
  g_err.clear();
  Ctx c;
  pct_status r = setup(c, grid, geom, hist, workspace, ws_bytes, stream);
  if (r != PCT_OK) return r;
  if (rows && (r = check_rows(rows, c.n, true)) != PCT_OK) return r;
  if (!x || !out) return fail(PCT_EINVAL, "x / out is NULL");
  return do_residual(c, grid, rows, x, out);
}

pct_status pct_roi_stats(const float *x, const uint8_t *labels, int64_t M, int32_t n_labels, double *sums,
                         int64_t *counts, void *stream) {
  g_err.clear();
  if (M < 0 || n_labels < 1 || n_labels > 255) return fail(PCT_EINVAL, "need M >= 0 and 1 <= n_labels <= 255");
  if ((M > 0 && (!x || !labels)) || !sums || !counts) return fail(PCT_EINVAL, "NULL array");
  HIPCHECK(pct::launch_roi(x, labels, M, n_labels, sums, counts, reinterpret_cast<hipStream_t>(stream)));
  return PCT_OK;
}

pct_status pct_profile_enable(int32_t on) {
  g_err.clear();
  std::lock_guard<std::mutex> g(g_prof_mu);
  if (on) {
    for (auto &r : g_prof) {
      hipEventSynchronize(r.b);
      g_prof_pool.push_back(r.a);
      g_prof_pool.push_back(r.b);
    }
    g_prof.clear();
  }
  g_prof_on = on != 0;
  return PCT_OK;
}

pct_status pct_profile_read(int64_t *launches, double *ms) {
  g_err.clear();
  if (!launches || !ms) return fail(PCT_EINVAL, "NULL output array");
  std::lock_guard<std::mutex> g(g_prof_mu);
  for (int k = 0; k < PCT_K_COUNT; ++k) {
    launches[k] = 0;
    ms[k] = 0.0;
  }
  for (auto &r : g_prof) {
    if (hipEventSynchronize(r.b) != hipSuccess) return fail(PCT_EDEVICE, "event synchronisation failed");
    float t = 0.f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return fail(PCT_EDEVICE, "event timing failed");
    launches[r.kind] += 1;
    ms[r.kind] += t;
  }
  return PCT_OK;
}

const char *pct_last_error(void) { return g_err.c_str(); }

}  // extern "C"
