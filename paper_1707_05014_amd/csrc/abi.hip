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

#include "cnn_internal.h"
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
    if (a && hipEventRecord(a, s) != hipSuccess) {  // no timing for this launch
      g_prof_pool.push_back(a);
      a = nullptr;
    }
  }
  void stop() {
    if (!a) return;
    std::lock_guard<std::mutex> g(g_prof_mu);
    hipEvent_t b = prof_event();
    if (b && hipEventRecord(b, s) == hipSuccess) {
      g_prof.push_back({kind, a, b});
    } else {
      g_prof_pool.push_back(a);
      if (b) g_prof_pool.push_back(b);
    }
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

// voxels of the grid rounded up to whole 4 x 4 x 4 bricks: the length of the
// workspace's per-voxel arrays, which the rebuilt-row sweeps index in brick
// order
int64_t brick_voxels(const pct_grid *g) {
  return (int64_t)((g->nx + 3) / 4) * ((g->ny + 3) / 4) * ((g->nz + 3) / 4) * 64;
}

pct::PathParams brick_params(const pct::PathParams &P) {
  pct::PathParams b = P;
  b.brick = 1;
  return b;
}

pct_status check_grid(const pct_grid *g) {
  if (!g) return fail(PCT_EINVAL, "grid is NULL");
  if (g->nx <= 0 || g->ny <= 0 || g->nz <= 0) return fail(PCT_EINVAL, "grid dimensions must be positive");
  if (!(g->dx > 0.f && g->dy > 0.f && g->dz > 0.f)) return fail(PCT_EINVAL, "voxel sizes must be positive");
  if (!(std::isfinite(g->ox) && std::isfinite(g->oy) && std::isfinite(g->oz)))
    return fail(PCT_EINVAL, "grid origin must be finite");
  if (brick_voxels(g) > 0x7fffffffLL) return fail(PCT_EINVAL, "grid has more than 2^31-1 voxels in whole 4x4x4 bricks");
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
    for (int m = 0; m < 3; ++m) {
      P.cF_d[m][n] = an / (n + m + 1.0);
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
  P.brick = 0;
  P.nbx = (g->nx + 3) / 4;
  P.nby = (g->ny + 3) / 4;
  const double reach = 2.0 * std::max(G->hull_a, G->hull_b);
  P.kmax = (int32_t)std::ceil(reach / G->step_mm) + 2;
  // Entries of a row: at most one more than the voxel faces its path crosses.
  // A smooth path of arc length s crosses at most sqrt(3) s / dmin faces plus
  // a few per turning point of each coordinate; s is at most the sample
  // spacing (<= dmin, checked above) times the segment count, stretched a
  // little by the lateral offsets, so 2 entries per sample bound it with room
  // to spare.  A row that still does not fit is reported (kStOverflow).
  P.emax = 2 * (P.kmax + 1) + 16;
  const size_t per_wave = pct::row_buf_bytes(P.emax);
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

pct_status check_tvs_params(const pct_sweep_params *p);

pct_status check_params(const pct_sweep_params *p, bool cached) {
  if (!p) return fail(PCT_EINVAL, "params are NULL");
  if (p->algo != 0 && p->algo != 1) return fail(PCT_EINVAL, "algo must be 0 (ART) or 1 (DROP)");
  if (p->algo == 0 && !cached) return fail(PCT_EINVAL, "ART needs cached rows");
  if (p->algo == 1 && p->block_size < 1) return fail(PCT_EINVAL, "block_size must be >= 1");
  if (!(p->lambda > 0.f && p->lambda < 2.f)) return fail(PCT_EINVAL, "lambda must be in (0, 2)");
  if (p->n_sweeps < 0) return fail(PCT_EINVAL, "n_sweeps must be >= 0");
  return check_tvs_params(p);
}

struct Ctx {
  pct::PathParams P;
  pct::HistPtrs H;
  pct::Workspace W;
  int64_t M, n;
  int64_t Mw = 0;           // voxels of the workspace's accumulators (M rounded up to whole bricks)
  hipStream_t s;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  bool recs_ready = false;  // W.recs holds every history's path record
  int extra = 0;            // optional workspace regions (kWsTvs, kWsCarp)
};

bool tvs_on(const pct_sweep_params *p) { return p && p->tvs && p->tvs->n_steps > 0; }

pct_status check_tvs(const pct_tvs *t);
pct_status check_tvs_params(const pct_sweep_params *p) {
  if (!p->tvs) return PCT_OK;
  if (p->tvs->n_steps > 0 && p->algo == 0) return fail(PCT_EINVAL, "TV superiorization runs with DROP (algo 1)");
  return check_tvs(p->tvs);
}

pct_status check_tvs(const pct_tvs *t) {
  if (!t || t->n_steps == 0) return PCT_OK;
  if (t->n_steps < 0) return fail(PCT_EINVAL, "tvs.n_steps must be >= 0");
  if (t->max_trials < 1 || t->max_trials > 16) return fail(PCT_EINVAL, "tvs.max_trials must be 1..16");
  if (!(t->a > 0.0 && t->a < 1.0)) return fail(PCT_EINVAL, "tvs.a must be in (0, 1)");
  if (!(t->eps > 0.0) || !std::isfinite(t->eps)) return fail(PCT_EINVAL, "tvs.eps must be positive");
  if (!t->state) return fail(PCT_EINVAL, "tvs.state is NULL");
  return PCT_OK;
}

// the TVS steps on x (the image entering a block, or a CARP iteration)
hipError_t run_tvs(const Ctx &c, int32_t nx, int32_t ny, int32_t nz, float *x, const uint8_t *mask,
                   const pct_tvs *t) {
  return pct::launch_tvs(nx, ny, nz, x, mask, t->n_steps, t->max_trials, t->a, t->eps, t->state, c.W.tvs, c.s);
}

pct_status check_ws(void *ws, size_t ws_bytes, int64_t M, int64_t n, int64_t plan_bt = 0, int extra = 0) {
  const size_t need = pct::workspace_bytes(M, n, plan_bt, 0, 0, false, extra);
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

float len_unit(const pct_grid *g) { return std::min(g->dx, std::min(g->dy, g->dz)); }

// One path pass per proton: chunks of rows are traced into staging slots of
// P.emax entries per row, their counts scanned into row_ptr, then compacted
// into the CSR arrays.  Without rows->idx only the counts are produced (sizing).
pct_status do_trace(Ctx &c, const pct_grid *g, pct_rows *rows) {
  const bool fill = rows->idx != nullptr;
  int64_t st_rows = std::min<int64_t>(c.n, pct::kStageRows);
  if (fill) {
    while (st_rows > 1 && pct::workspace_bytes(c.Mw, c.n, 0, st_rows * c.P.emax, 0, false, c.extra) > c.ws_bytes)
      st_rows /= 2;
    const size_t need = pct::workspace_bytes(c.Mw, c.n, 0, std::max<int64_t>(st_rows, 1) * c.P.emax, 0, false, c.extra);
    if (need > c.ws_bytes)
      return fail(PCT_ENOMEM, "workspace of %zu bytes given, %zu needed to stage rows", c.ws_bytes, need);
  }
  st_rows = std::max<int64_t>(st_rows, 1);
  c.W = pct::carve_workspace(c.ws, c.Mw, c.n, 0, fill ? st_rows * c.P.emax : 0, 0, false, c.extra);
  const float scale = 1.0f / len_unit(g);
  HIPCHECK(pct::launch_fill_u32(c.W.status, 4, 0u, c.s));
  if (c.n == 0) HIPCHECK(pct::launch_scan_rows(rows->row_ptr, 0, 0, c.W.scan, c.s));
  for (int64_t i0 = 0; i0 < c.n; i0 += st_rows) {
    const int64_t nr = std::min<int64_t>(st_rows, c.n - i0);
    PROF(PCT_K_PATH_SETUP, pct::launch_path_setup(c.P, c.H, nullptr, i0, nr, c.n, c.W.recs, c.W.status, true, c.s));
    PROF(PCT_K_TRACE_PATH, pct::launch_trace_stage(c.P, c.W.recs, i0, nr, rows->row_ptr + i0 + 1,
                                                   fill ? c.W.st_idx : nullptr, c.W.st_len, rows->norm2,
                                                   c.W.status, c.s));
    HIPCHECK(pct::launch_scan_rows(rows->row_ptr, i0, nr, c.W.scan, c.s));
    if (fill)
      PROF(PCT_K_TRACE_COMPACT, pct::launch_trace_compact(i0, nr, rows->row_ptr, c.W.st_idx, c.W.st_len, c.P.emax,
                                                          rows->idx, rows->len, rows->len_dtype, scale,
                                                          rows->cap_nnz, c.W.status, c.s));
  }
  int64_t total = 0;
  HIPCHECK(hipMemcpyAsync(&total, rows->row_ptr + c.n, sizeof total, hipMemcpyDeviceToHost, c.s));
  uint32_t st = 0;
  pct_status r = read_status(c, &st);
  if (r != PCT_OK) return r;
  rows->nnz = total;
  if (st & pct::kStOverflow) return status_to_code(st);
  if (fill && (st & pct::kStRowCap))
    return fail(PCT_EROWCAP, "rows need %lld entries, capacity is %lld", (long long)total,
                (long long)rows->cap_nnz);
  return status_to_code(st);
}

// Elements of the per-block voxel counts that a fused DROP reconstruction of
// several sweeps keeps (the block composition, hence s_j, is the same every
// sweep): n_blocks x M, or 0 when not worth it or too large.
int64_t fused_count_elems(int64_t M, int64_t n, const pct_sweep_params *p) {
  if (!p || p->algo != 1 || p->block_size < 1 || p->n_sweeps < 2 || n <= 0) return 0;
  const int64_t nb = (n + p->block_size - 1) / p->block_size;
  if (nb > pct::kMaxBlkCntBytes / 2 / std::max<int64_t>(M, 1)) return 0;
  return nb * M;
}

// Fused calls: when the workspace holds one path record per history, carve
// it so (keeping the per-block counts when blk > 0 and they fit too).
bool carve_fused(Ctx &c, int64_t blk) {
  const int x = c.extra;
  if (blk > 0 && pct::workspace_bytes(c.Mw, c.n, 0, 0, blk, true, x) <= c.ws_bytes) {
    c.W = pct::carve_workspace(c.ws, c.Mw, c.n, 0, 0, blk, true, x);
    return true;
  }
  if (pct::workspace_bytes(c.Mw, c.n, 0, 0, 0, true, x) <= c.ws_bytes) {
    c.W = pct::carve_workspace(c.ws, c.Mw, c.n, 0, 0, 0, true, x);
    return true;
  }
  if (blk > 0 && pct::workspace_bytes(c.Mw, c.n, 0, 0, blk, false, x) <= c.ws_bytes)
    c.W = pct::carve_workspace(c.ws, c.Mw, c.n, 0, 0, blk, false, x);
  return false;
}

// every history's path set-up, once per call (the records do not depend on x)
pct_status prepare_records(Ctx &c) {
  if (c.recs_ready || c.W.rec_rows < c.n || c.n == 0) return PCT_OK;
  PROF(PCT_K_PATH_SETUP, pct::launch_path_setup(c.P, c.H, nullptr, 0, c.n, c.n, c.W.recs, c.W.status, false, c.s));
  c.recs_ready = true;
  return PCT_OK;
}

// count_mode 0: s_j formed with atomics in every block; 1: formed and stored
// per block; 2: read from the stored counts.  The sweep covers the positions
// [p0, p1) of the order (p1 < 0: all), in blocks from p0; with p->tvs the
// TVS steps run on x before every block; touched (CARP) marks the voxels
// the rows touch.
pct_status do_sweep(Ctx &c, const pct_grid *g, const pct_rows *rows, float *x, const pct_sweep_params *p,
                    int count_mode = 0, int64_t p0 = 0, int64_t p1 = -1, uint8_t *touched = nullptr) {
  HIPCHECK(pct::launch_mask(x, p->hull_mask, c.M, c.s));
  const float unit = len_unit(g);
  if (p->algo == 0) {
    PROF(PCT_K_ART, pct::launch_art(rows->row_ptr, rows->idx, rows->len, rows->len_dtype, unit, rows->norm2,
                                    c.H.wepl, p->order, c.n, c.M, x, p->hull_mask, p->lambda, c.W.status, c.s));
    return PCT_OK;
  }
  const bool tv = tvs_on(p);
  if (tv && !c.W.tvs) return fail(PCT_ENOMEM, "workspace carved without the TV superiorization scratch");
  if (p1 < 0) p1 = c.n;
  HIPCHECK(pct::launch_fill_f32(c.W.num, c.Mw, 0.f, c.s));
  HIPCHECK(pct::launch_fill_u32(c.W.cnt, c.Mw, 0u, c.s));
  if (rows || !c.W.blk_cnt || touched) count_mode = 0;
  // rebuilt rows: voxels numbered in bricks (accumulators and a copy of x
  // in that order), so that each wavefront's atomics and gathers along a
  // path touch few cache lines
  const pct::PathParams Pb = brick_params(c.P);
  if (!rows) HIPCHECK(pct::launch_to_bricks(Pb, x, c.W.xb, c.Mw, c.s));
  const int kproj = count_mode == 2 ? PCT_K_PROJECT : PCT_K_PROJECT_COUNTING;
  // rebuilt rows: a sweep that forms the block counts adds numerator and
  // count with one packed 64-bit atomic
  int pk_bits = 0, pk_k = 0;
  unsigned long long *pk = nullptr;
  if (count_mode != 2 && !rows && c.W.pk && pct::packed_counts(p->block_size, pk_bits, pk_k)) {
    pk = c.W.pk;
    HIPCHECK(pct::launch_fill_u32(reinterpret_cast<uint32_t *>(pk), 2 * c.Mw, 0u, c.s));
  }
  for (int64_t first = p0, blk = 0; first < p1; first += p->block_size, ++blk) {
    const int64_t count = std::min<int64_t>(p->block_size, p1 - first);
    if (tv) {
      PROF(PCT_K_TVS, run_tvs(c, g->nx, g->ny, g->nz, x, p->hull_mask, p->tvs));
      if (!rows) HIPCHECK(pct::launch_to_bricks(Pb, x, c.W.xb, c.Mw, c.s));
    }
    if (rows)
      PROF(PCT_K_PROJECT, pct::launch_project_cached(rows->row_ptr, rows->idx, rows->len, rows->len_dtype, unit,
                                                     rows->norm2, c.H.wepl, p->order, first, count, c.n, c.M, x,
                                                     c.W.num, c.W.cnt, c.W.status, c.s));
    else if (c.recs_ready)
      PROF(kproj, pct::launch_project_fused(Pb, c.W.recs, p->order, first, c.n, true, count, c.W.xb, c.W.num,
                                            count_mode == 2 ? nullptr : c.W.cnt, c.W.status, c.s, pk, pk_bits, pk_k));
    else
      for (int64_t s0 = 0; s0 < count; s0 += c.W.rec_rows) {
        const int64_t cs = std::min<int64_t>(c.W.rec_rows, count - s0);
        PROF(PCT_K_PATH_SETUP, pct::launch_path_setup(c.P, c.H, p->order, first + s0, cs, c.n, c.W.recs,
                                                      c.W.status, false, c.s));
        PROF(kproj, pct::launch_project_fused(Pb, c.W.recs, nullptr, 0, c.n, false, cs, c.W.xb, c.W.num,
                                              count_mode == 2 ? nullptr : c.W.cnt, c.W.status, c.s, pk, pk_bits,
                                              pk_k));
      }
    PROF(PCT_K_APPLY, pct::launch_apply_counts(x, c.W.num, c.W.cnt, count_mode ? c.W.blk_cnt + blk * c.Mw : nullptr,
                                               count_mode, p->hull_mask, c.M, p->lambda, c.W.status, c.s, touched,
                                               rows ? nullptr : &Pb, c.W.xb, c.Mw, pk, pk_bits, pk_k));
  }
  return PCT_OK;
}

pct_status do_residual(Ctx &c, const pct_grid *g, const pct_rows *rows, const float *x, double *out) {
  if (rows) {
    PROF(PCT_K_RESIDUAL, pct::launch_residual_cached(rows->row_ptr, rows->idx, rows->len, rows->len_dtype,
                                                     len_unit(g), c.H.wepl, c.n, c.M, x, c.W.partials, out, c.s));
    return PCT_OK;
  }
  const pct::PathParams Pb = brick_params(c.P);
  HIPCHECK(pct::launch_to_bricks(Pb, x, c.W.xb, c.Mw, c.s));
  if (c.recs_ready) {
    PROF(PCT_K_RESIDUAL, pct::launch_residual_fused(Pb, c.W.recs, c.n, c.W.xb, c.W.partials, c.W.status, false, c.s));
    HIPCHECK(pct::launch_residual_final(c.W.partials, pct::kResidFusedGrid, out, c.s));
  } else {
    for (int64_t i0 = 0; i0 < c.n; i0 += c.W.rec_rows) {
      const int64_t cs = std::min<int64_t>(c.W.rec_rows, c.n - i0);
      PROF(PCT_K_PATH_SETUP, pct::launch_path_setup(c.P, c.H, nullptr, i0, cs, c.n, c.W.recs, c.W.status, false,
                                                    c.s));
      PROF(PCT_K_RESIDUAL, pct::launch_residual_fused(Pb, c.W.recs, cs, c.W.xb, c.W.partials, c.W.status, i0 > 0,
                                                      c.s));
    }
    if (c.n == 0) HIPCHECK(pct::launch_fill_f64(c.W.partials, pct::kResidFusedGrid, 0.0, c.s));
    HIPCHECK(pct::launch_residual_final(c.W.partials, pct::kResidFusedGrid, out, c.s));
  }
  return PCT_OK;
}

pct_status setup(Ctx &c, const pct_grid *grid, const pct_geom *geom, const pct_histories *hist, void *ws,
                  size_t ws_bytes, void *stream, int extra = 0) {
  pct_status r;
  if ((r = check_grid(grid)) != PCT_OK) return r;
  if ((r = check_hist(hist)) != PCT_OK) return r;
  if ((r = make_params(grid, geom, c.P)) != PCT_OK) return r;
  c.M = grid_voxels(grid);
  c.Mw = brick_voxels(grid);
  c.n = hist->n;
  c.extra = extra;
  if ((r = check_ws(ws, ws_bytes, c.Mw, c.n, 0, extra)) != PCT_OK) return r;
  c.H = hist_ptrs(hist);
  c.W = pct::carve_workspace(ws, c.Mw, c.n, 0, 0, 0, false, extra);
  c.ws = ws;
  c.ws_bytes = ws_bytes;
  c.s = reinterpret_cast<hipStream_t>(stream);
  return PCT_OK;
}

// ------------------------------------------------------------------ plans
struct PlanDims {
  int64_t n, B, nb, T;
  int32_t ntx, nty, ntz;
};

PlanDims plan_dims(const pct_grid *g, int64_t n, int64_t B) {
  PlanDims d;
  d.n = n;
  d.B = B;
  d.nb = n > 0 ? (n + B - 1) / B : 0;
  d.ntx = (g->nx + pct::kTX - 1) / pct::kTX;
  d.nty = (g->ny + pct::kTY - 1) / pct::kTY;
  d.ntz = (g->nz + pct::kTZ - 1) / pct::kTZ;
  d.T = (int64_t)d.ntx * d.nty * d.ntz;
  return d;
}

int64_t plan_scratch_len(const PlanDims &d) { return d.nb * d.T + d.nb + 8; }

enum {
  L_REFBASE, L_BT_OFF, L_BT_CUR, L_ORDROW, L_RVALS, L_EMASK, L_CFE, L_PACKED, L_LEN, L_REFCNT, L_REFS, L_BPERM, L_N2PERM,
  L_PARTIAL, L_RESPART, L_SCANTMP, L_ENDSLOT, L_META, L_COUNT
};

size_t plan_layout(const pct_plan *p, size_t off[L_COUNT]) {
  const int64_t nbT = p->n_blocks * p->n_tiles;
  const size_t lb = p->len_dtype == 0 ? 4 : 2;
  const size_t sz[] = {(size_t)(p->n + 1) * 8,   (size_t)(nbT + 1) * 8,   (size_t)nbT * 8,
                              (size_t)p->refs * 4,     (size_t)p->block_size * 4,
                              (size_t)p->chunks * 8,   (size_t)(p->chunks + 1) * 8,
                              (size_t)p->entries * 2,  (size_t)p->entries * lb, (size_t)p->n * 4,
                              (size_t)p->refs * 4,     (size_t)p->n * 4,         (size_t)p->n * 8,
                              (size_t)p->max_ends * 4, (size_t)pct::kResidAllGrid * 8,
                              (size_t)((p->chunks + pct::kScanChunk - 1) / pct::kScanChunk + 2) * 8,
                              (size_t)p->refs * 4,
                              (size_t)p->chunks * 16};
  static_assert(sizeof(sz) / sizeof(sz[0]) == L_COUNT, "one size per plan region");
  size_t o = 0;
  for (int k = 0; k < L_COUNT; ++k) {
    off[k] = o;
    o += align_up(sz[k] > 0 ? sz[k] : 8);
  }
  return o;
}

pct::PlanView plan_view(const pct_plan *p, float len_unit) {
  size_t off[L_COUNT];
  plan_layout(p, off);
  char *m = static_cast<char *>(p->mem);
  pct::PlanView V;
  std::memset(&V, 0, sizeof V);
  V.n = p->n;
  V.B = p->block_size;
  V.nb = p->n_blocks;
  V.T = p->n_tiles;
  V.E = p->entries;
  V.C = p->chunks;
  V.R = p->refs;
  V.P = p->max_ends;
  V.maxc = p->max_chunks;
  V.nx = p->nx;
  V.ny = p->ny;
  V.nz = p->nz;
  V.ntx = (p->nx + pct::kTX - 1) / pct::kTX;
  V.nty = (p->ny + pct::kTY - 1) / pct::kTY;
  V.ntz = (p->nz + pct::kTZ - 1) / pct::kTZ;
  V.len_dtype = p->len_dtype;
  V.len_unit = len_unit;
  if (!m) return V;
  V.bt_off = reinterpret_cast<int64_t *>(m + off[L_BT_OFF]);
  V.bt_cur = reinterpret_cast<unsigned long long *>(m + off[L_BT_CUR]);
  V.ord_row = reinterpret_cast<uint32_t *>(m + off[L_ORDROW]);
  V.rvals = reinterpret_cast<float *>(m + off[L_RVALS]);
  V.end_mask = reinterpret_cast<uint64_t *>(m + off[L_EMASK]);
  V.chunk_first_end = reinterpret_cast<int64_t *>(m + off[L_CFE]);
  V.packed = reinterpret_cast<uint16_t *>(m + off[L_PACKED]);
  V.len = m + off[L_LEN];
  V.ref_base = reinterpret_cast<int64_t *>(m + off[L_REFBASE]);
  V.ref_cnt = reinterpret_cast<int32_t *>(m + off[L_REFCNT]);
  V.refs = reinterpret_cast<uint32_t *>(m + off[L_REFS]);
  V.b_perm = reinterpret_cast<float *>(m + off[L_BPERM]);
  V.n2_perm = reinterpret_cast<double *>(m + off[L_N2PERM]);
  V.partial = reinterpret_cast<float *>(m + off[L_PARTIAL]);
  V.res_part = reinterpret_cast<double *>(m + off[L_RESPART]);
  V.end_slot = reinterpret_cast<uint32_t *>(m + off[L_ENDSLOT]);
  V.meta = m + off[L_META];
  return V;
}

int64_t *plan_scan_tmp(const pct_plan *p) {
  size_t off[L_COUNT];
  plan_layout(p, off);
  return reinterpret_cast<int64_t *>(static_cast<char *>(p->mem) + off[L_SCANTMP]);
}

pct_status check_plan_params(const pct_sweep_params *p, int64_t n) {
  if (!p) return fail(PCT_EINVAL, "params are NULL");
  if (p->algo != 1) return fail(PCT_EINVAL, "plans serve DROP (algo 1)");
  if (p->block_size < 1 || p->block_size > pct::kMaxPlanBlock)
    return fail(PCT_EINVAL, "plans need 1 <= block_size <= %lld", (long long)pct::kMaxPlanBlock);
  if (!(p->lambda > 0.f && p->lambda < 2.f)) return fail(PCT_EINVAL, "lambda must be in (0, 2)");
  (void)n;
  return check_tvs_params(p);
}

// sizing pass + (when plan->mem is set) construction
pct_status do_plan_build(Ctx &c, const pct_grid *g, const pct_rows *rows, const pct_sweep_params *params,
                         pct_plan *plan, void *ws, size_t ws_bytes) {
  const PlanDims d = plan_dims(g, c.n, params->block_size);
  const int64_t scr = plan_scratch_len(d);
  pct_status r = check_ws(ws, ws_bytes, c.Mw, c.n, scr);
  if (r != PCT_OK) return r;
  c.W = pct::carve_workspace(ws, c.Mw, c.n, scr);
  const float unit = len_unit(g);
  pct_plan tmp = *plan;
  tmp.n = d.n;
  tmp.block_size = d.B;
  tmp.n_blocks = d.nb;
  tmp.n_tiles = d.T;
  tmp.nx = g->nx;
  tmp.ny = g->ny;
  tmp.nz = g->nz;
  tmp.len_dtype = rows->len_dtype;
  tmp.ready = 0;
  pct::PlanView V = plan_view(&tmp, unit);  // dims only (no memory yet)
  int64_t *bt_cnt = c.W.plan_scratch;
  int64_t *blk_cap = bt_cnt + d.nb * d.T;
  HIPCHECK(pct::launch_fill_u32(reinterpret_cast<uint32_t *>(c.W.plan_scratch), 2 * scr, 0u, c.s));
  HIPCHECK(pct::launch_fill_u32(c.W.status, 4, 0u, c.s));
  // the per-row capacities go straight into the plan's ref_base (first region)
  // when the plan memory is there and large enough to hold it
  int64_t *row_cap = nullptr;
  if (plan->mem && plan->bytes >= (size_t)(c.n + 1) * 8) row_cap = static_cast<int64_t *>(plan->mem);
  PROF(PCT_K_PLAN_BUILD, pct::launch_plan_count(rows->row_ptr, rows->idx, params->order, c.n, d.B, c.M, V, bt_cnt,
                                                row_cap, blk_cap, c.W.status, c.s));
  std::vector<int64_t> host((size_t)scr);
  HIPCHECK(hipMemcpyAsync(host.data(), c.W.plan_scratch, (size_t)scr * 8, hipMemcpyDeviceToHost, c.s));
  uint32_t st = 0;
  if ((r = read_status(c, &st)) != PCT_OK) return r;
  if (st) return status_to_code(st);
  std::vector<int64_t> bt_off((size_t)(d.nb * d.T + 1), 0);
  int64_t E = 0, maxc = 0, P = 1, Rtot = 0;
  for (int64_t b = 0; b < d.nb; ++b) {
    int64_t eb = 0;
    for (int64_t t = 0; t < d.T; ++t) {
      const int64_t k = b * d.T + t;
      const int64_t pad = (host[k] + 63) / 64 * 64;
      bt_off[k] = E;
      E += pad;
      eb += pad;
    }
    maxc = std::max(maxc, eb / 64);
    P = std::max(P, host[d.nb * d.T + b]);
    Rtot += host[d.nb * d.T + b];
  }
  bt_off[d.nb * d.T] = E;
  tmp.entries = E;
  tmp.chunks = E / 64;
  tmp.refs = Rtot;
  tmp.max_chunks = std::max<int64_t>(maxc, 1);
  tmp.max_ends = P;
  size_t off[L_COUNT];
  const size_t need = plan_layout(&tmp, off);
  if (E >= (int64_t(1) << 32)) return fail(PCT_EINVAL, "plan has more than 2^32 entries");
  if (!plan->mem) {
    tmp.bytes = need;
    tmp.mem = nullptr;
    *plan = tmp;
    return PCT_OK;
  }
  if (plan->bytes < need) {
    plan->bytes = need;
    return fail(PCT_ENOMEM, "plan needs %zu bytes", need);
  }
  tmp.order = params->order;
  tmp.rows_idx = rows->idx;
  V = plan_view(&tmp, unit);
  HIPCHECK(hipMemcpyAsync(V.bt_off, bt_off.data(), bt_off.size() * 8, hipMemcpyHostToDevice, c.s));
  HIPCHECK(pct::launch_copy_i64_to_u64(V.bt_cur, V.bt_off, d.nb * d.T, c.s));
  if (row_cap != V.ref_base) return fail(PCT_EDEVICE, "plan layout: ref_base is not the first region");
  HIPCHECK(pct::launch_scan_rows(V.ref_base, 0, c.n, c.W.scan, c.s));
  HIPCHECK(pct::launch_fill_u32(reinterpret_cast<uint32_t *>(V.packed), E / 2, 0u, c.s));
  PROF(PCT_K_PLAN_BUILD, pct::launch_plan_fill(rows->row_ptr, rows->idx, rows->len, rows->len_dtype, params->order,
                                               c.H.wepl, rows->norm2, c.M, V, c.W.status, c.s));
  PROF(PCT_K_PLAN_BUILD, pct::launch_plan_chunks(V, c.s));
  HIPCHECK(pct::launch_scan_rows(V.chunk_first_end, 0, tmp.chunks, plan_scan_tmp(&tmp), c.s));
  PROF(PCT_K_PLAN_BUILD, pct::launch_plan_ref_ordinals(V, c.s));
  int64_t refs_total = 0, ends = 0;
  HIPCHECK(hipMemcpyAsync(&refs_total, V.ref_base + c.n, 8, hipMemcpyDeviceToHost, c.s));
  HIPCHECK(hipMemcpyAsync(&ends, V.chunk_first_end + tmp.chunks, 8, hipMemcpyDeviceToHost, c.s));
  if ((r = read_status(c, &st)) != PCT_OK) return r;
  if (st) return status_to_code(st);
  if (refs_total != tmp.refs) return fail(PCT_EDEVICE, "plan reference count changed between passes");
  tmp.ends = ends;
  tmp.ready = 1;
  *plan = tmp;
  return PCT_OK;
}

pct_status check_plan(const pct_plan *plan, const pct_grid *g) {
  if (!plan || !plan->mem || !plan->ready) return fail(PCT_EINVAL, "plan is not built");
  if (plan->nx != g->nx || plan->ny != g->ny || plan->nz != g->nz) return fail(PCT_EINVAL, "plan grid differs");
  size_t off[L_COUNT];
  if (plan->bytes < plan_layout(plan, off)) return fail(PCT_EINVAL, "plan bytes smaller than its layout");
  return PCT_OK;
}

pct_status do_plan_sweep(Ctx &c, const pct_plan *plan, const pct::PlanView &V, float *x,
                         const pct_sweep_params *p) {
  HIPCHECK(pct::launch_mask(x, p->hull_mask, c.M, c.s));
  const bool tv = tvs_on(p);
  if (tv && !c.W.tvs) return fail(PCT_ENOMEM, "workspace carved without the TV superiorization scratch");
  for (int64_t b = 0; b < plan->n_blocks; ++b) {
    if (tv) PROF(PCT_K_TVS, run_tvs(c, plan->nx, plan->ny, plan->nz, x, p->hull_mask, p->tvs));
    PROF(PCT_K_PLAN_DOT, pct::launch_plan_dot(V, b, x, c.s));
    PROF(PCT_K_PLAN_ROWS, pct::launch_plan_rows(V, b, c.s));
    PROF(PCT_K_PLAN_SCATTER, pct::launch_plan_scatter(V, b, x, p->hull_mask, p->lambda, c.s));
  }
  return PCT_OK;
}

// ||Ax - b|| over every block with one dot pass (its partials at the rows'
// absolute slots) and one pass over the rows
pct_status do_plan_residual(Ctx &c, const pct_plan *plan, const pct::PlanView &V, const float *x, double *out) {
  (void)plan;
  PROF(PCT_K_RESIDUAL, pct::launch_plan_dot_all(V, x, c.s));
  PROF(PCT_K_RESIDUAL, pct::launch_plan_resid_all(V, V.res_part, c.s));
  PROF(PCT_K_RESIDUAL, pct::launch_sum_partials(V.res_part, pct::kResidAllGrid, out, 1, c.s));
  return PCT_OK;
}

}  // namespace

namespace pct {

// fixed part (status, DROP accumulators, partial sums, scan chunks) followed
// by one shared tail: the plan sizing counters during a plan build, the
// staged rows during a trace (never both at once)
static int64_t rec_rows_for(int64_t n_hist, bool recs_all) {
  const int64_t n = std::max<int64_t>(n_hist, 0);
  return recs_all ? n : std::min<int64_t>(n, kStageRows);
}

static size_t extra_bytes(int64_t M, int extra) {
  size_t b = 0;
  if (extra & kWsTvs) b += align_up(tvs_scratch_bytes(M));
  if (extra & kWsCarp) b += 2 * align_up((size_t)M * 4) + align_up((size_t)M * 2) + align_up((size_t)M);
  return b;
}

size_t workspace_bytes(int64_t M, int64_t n_hist, int64_t plan_bt, int64_t stage_slots, int64_t blk_cnt_elems,
                       bool recs_all, int extra) {
  size_t b = align_up(4 * sizeof(uint32_t));
  b += align_up((size_t)M * sizeof(float));
  b += align_up((size_t)M * sizeof(uint32_t));
  b += align_up((size_t)kMaxPartials * sizeof(double));
  b += align_up((size_t)M * sizeof(float));
  b += extra_bytes(M, extra);
  b += align_up((size_t)((n_hist + kScanChunk - 1) / kScanChunk + 2) * sizeof(int64_t));
  b += align_up((size_t)rec_rows_for(n_hist, recs_all) * kPathRecBytes);
  const size_t plan_b = (size_t)(plan_bt > 0 ? plan_bt : 0) * sizeof(int64_t);
  const size_t stage_b = 2 * align_up((size_t)(stage_slots > 0 ? stage_slots : 0) * 4);
  b += align_up(std::max(plan_b, stage_b));
  b += align_up((size_t)(blk_cnt_elems > 0 ? blk_cnt_elems : 0) * sizeof(uint16_t));
  if (blk_cnt_elems > 0 || recs_all) b += align_up((size_t)M * sizeof(unsigned long long));
  return b;
}

Workspace carve_workspace(void *base, int64_t M, int64_t n_hist, int64_t plan_bt, int64_t stage_slots,
                          int64_t blk_cnt_elems, bool recs_all, int extra) {
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
  w.xb = reinterpret_cast<float *>(p);
  p += align_up((size_t)M * sizeof(float));
  w.tvs = nullptr;
  w.carp_xs = w.carp_acc = nullptr;
  w.carp_tc = nullptr;
  w.carp_touched = nullptr;
  if (extra & kWsTvs) {
    w.tvs = p;
    p += align_up(tvs_scratch_bytes(M));
  }
  if (extra & kWsCarp) {
    w.carp_xs = reinterpret_cast<float *>(p);
    p += align_up((size_t)M * 4);
    w.carp_acc = reinterpret_cast<float *>(p);
    p += align_up((size_t)M * 4);
    w.carp_tc = reinterpret_cast<uint16_t *>(p);
    p += align_up((size_t)M * 2);
    w.carp_touched = reinterpret_cast<uint8_t *>(p);
    p += align_up((size_t)M);
  }
  w.scan = reinterpret_cast<int64_t *>(p);
  p += align_up((size_t)((n_hist + kScanChunk - 1) / kScanChunk + 2) * sizeof(int64_t));
  w.recs = p;
  w.rec_rows = rec_rows_for(n_hist, recs_all);
  p += align_up((size_t)w.rec_rows * kPathRecBytes);
  w.plan_scratch = reinterpret_cast<int64_t *>(p);
  w.st_idx = reinterpret_cast<int32_t *>(p);
  w.st_len = reinterpret_cast<float *>(p + align_up((size_t)(stage_slots > 0 ? stage_slots : 0) * 4));
  const size_t plan_b = (size_t)(plan_bt > 0 ? plan_bt : 0) * sizeof(int64_t);
  const size_t stage_b = 2 * align_up((size_t)(stage_slots > 0 ? stage_slots : 0) * 4);
  p += align_up(std::max(plan_b, stage_b));
  w.blk_cnt = blk_cnt_elems > 0 ? reinterpret_cast<uint16_t *>(p) : nullptr;
  p += align_up((size_t)(blk_cnt_elems > 0 ? blk_cnt_elems : 0) * sizeof(uint16_t));
  w.pk = (blk_cnt_elems > 0 || recs_all) ? reinterpret_cast<unsigned long long *>(p) : nullptr;
  return w;
}

}  // namespace pct

extern "C" {

size_t pct_workspace_size(const pct_grid *grid, const pct_geom *geom, const pct_sweep_params *params,
                          int64_t n_hist, int32_t fused) {
  if (!grid || grid->nx <= 0 || grid->ny <= 0 || grid->nz <= 0 || n_hist < 0) return 0;
  int64_t plan_bt = 0;
  if (params && !fused && params->algo == 1 && params->block_size >= 1)
    plan_bt = plan_scratch_len(plan_dims(grid, n_hist, params->block_size));
  int64_t stage = 0;
  pct::PathParams P;
  if (geom && !fused && make_params(grid, geom, P) == PCT_OK)
    stage = std::min<int64_t>(n_hist, pct::kStageRows) * P.emax;
  const int64_t blk = fused ? fused_count_elems(brick_voxels(grid), n_hist, params) : 0;
  return pct::workspace_bytes(brick_voxels(grid), n_hist, plan_bt, stage, blk, fused != 0,
                              tvs_on(params) ? pct::kWsTvs : 0);
}

size_t pct_carp_workspace_size(const pct_grid *grid, const pct_geom *geom, const pct_sweep_params *params,
                               int64_t n_hist, int32_t fused) {
  if (!grid || grid->nx <= 0 || grid->ny <= 0 || grid->nz <= 0 || n_hist < 0) return 0;
  int64_t stage = 0;
  pct::PathParams P;
  if (geom && !fused && make_params(grid, geom, P) == PCT_OK)
    stage = std::min<int64_t>(n_hist, pct::kStageRows) * P.emax;
  return pct::workspace_bytes(brick_voxels(grid), n_hist, 0, stage, 0, fused != 0,
                              pct::kWsCarp | (tvs_on(params) ? pct::kWsTvs : 0));
}

pct_status pct_mlp_trace(const pct_grid *grid, const pct_geom *geom, const pct_histories *hist, pct_rows *rows,
                         void *workspace, size_t ws_bytes, void *stream) {
  g_err.clear();
  Ctx c;
  pct_status r = setup(c, grid, geom, hist, workspace, ws_bytes, stream);
  if (r != PCT_OK) return r;
  if ((r = check_rows(rows, c.n, false)) != PCT_OK) return r;
  if (rows->idx && (!rows->len || !rows->norm2)) return fail(PCT_EINVAL, "rows.len / rows.norm2 are NULL");
  return do_trace(c, grid, rows);
}

pct_status pct_project_sweep(const pct_grid *grid, const pct_geom *geom, const pct_histories *hist,
                             const pct_rows *rows, float *x, const pct_sweep_params *params, double *resid_out,
                             void *workspace, size_t ws_bytes, void *stream) {
  g_err.clear();
  Ctx c;
  pct_status r;
  if ((r = check_params(params, rows != nullptr)) != PCT_OK) return r;
  if ((r = setup(c, grid, geom, hist, workspace, ws_bytes, stream, tvs_on(params) ? pct::kWsTvs : 0)) != PCT_OK)
    return r;
  if (rows && (r = check_rows(rows, c.n, true)) != PCT_OK) return r;
  if (!x) return fail(PCT_EINVAL, "x is NULL");
  HIPCHECK(pct::launch_fill_u32(c.W.status, 4, 0u, c.s));
  if (!rows && params->algo == 1 && carve_fused(c, 0)) {
    HIPCHECK(pct::launch_fill_u32(c.W.status, 4, 0u, c.s));
    if ((r = prepare_records(c)) != PCT_OK) return r;
  }
  if ((r = do_sweep(c, grid, rows, x, params)) != PCT_OK) return r;
  if (resid_out) {
    if ((r = do_residual(c, grid, rows, x, resid_out)) != PCT_OK) return r;
    HIPCHECK(pct::launch_poison_on_status(resid_out, c.W.status, c.s));
  }
  return PCT_OK;
}

// ---- one sweep over cached rows with no workspace argument: its scratch
// (status word, DROP numerators and counts, residual partial sums) is the
// library's static device array below, one copy per GPU
namespace {

constexpr int64_t kNoAllocMaxVoxels = int64_t(1) << 21;
constexpr size_t kNoAllocStatusBytes = 256;
constexpr size_t kNoAllocBytes =
    kNoAllocStatusBytes + 2 * (size_t)kNoAllocMaxVoxels * 4 + (size_t)pct::kMaxPartials * sizeof(double);
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kNoAllocMaxDevices] = {};

// the device address of `scratch` on the current device (looked up once per
// device; host code never uses the array's name as an address)
pct_status noalloc_scratch(void **out) {
  int dev = -1;
  HIPCHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocMaxDevices) return fail(PCT_EDEVICE, "device index %d out of range", dev);
  std::lock_guard<std::mutex> g(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(PCT_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_noalloc_ptr[dev] = p;
  }
  *out = g_noalloc_ptr[dev];
  return PCT_OK;
}

}  // namespace

pct_status pct_project_sweep_noalloc(const pct_grid *grid, const pct_geom *geom, const pct_histories *hist,
                                     const pct_rows *rows, float *x, const pct_sweep_params *params,
                                     double *resid_out, void *stream) {
  g_err.clear();
  Ctx c;
  pct_status r;
  if (!rows) return fail(PCT_EINVAL, "the no-allocation sweep needs cached rows");
  if ((r = check_params(params, true)) != PCT_OK) return r;
  if (tvs_on(params)) return fail(PCT_EINVAL, "the no-allocation sweep runs without TV superiorization");
  if ((r = check_grid(grid)) != PCT_OK) return r;
  if ((r = check_hist(hist)) != PCT_OK) return r;
  if ((r = make_params(grid, geom, c.P)) != PCT_OK) return r;
  c.M = grid_voxels(grid);
  c.Mw = c.M;  // rows only: linear accumulators
  c.n = hist->n;
  if (c.M > kNoAllocMaxVoxels)
    return fail(PCT_EINVAL, "grid of %lld voxels exceeds the no-allocation scratch (at most %lld voxels)",
                (long long)c.M, (long long)kNoAllocMaxVoxels);
  if ((r = check_rows(rows, c.n, true)) != PCT_OK) return r;
  if (!x) return fail(PCT_EINVAL, "x is NULL");
  void *base = nullptr;
  if ((r = noalloc_scratch(&base)) != PCT_OK) return r;
  char *p = static_cast<char *>(base);
  c.H = hist_ptrs(hist);
  c.W = pct::Workspace{};
  c.W.status = reinterpret_cast<uint32_t *>(p);
  c.W.num = reinterpret_cast<float *>(p + kNoAllocStatusBytes);
  c.W.cnt = reinterpret_cast<uint32_t *>(p + kNoAllocStatusBytes + (size_t)kNoAllocMaxVoxels * 4);
  c.W.partials = reinterpret_cast<double *>(p + kNoAllocStatusBytes + 2 * (size_t)kNoAllocMaxVoxels * 4);
  c.s = reinterpret_cast<hipStream_t>(stream);
  // the array keeps the previous call's contents: the status word is cleared
  // here, the numerators and counts by do_sweep, the partials are written
  // before they are read
  HIPCHECK(pct::launch_fill_u32(c.W.status, 4, 0u, c.s));
  if ((r = do_sweep(c, grid, rows, x, params)) != PCT_OK) return r;
  if (resid_out) {
    if ((r = do_residual(c, grid, rows, x, resid_out)) != PCT_OK) return r;
    HIPCHECK(pct::launch_poison_on_status(resid_out, c.W.status, c.s));
  }
  return PCT_OK;
}

pct_status pct_plan_build(const pct_grid *grid, const pct_histories *hist, const pct_rows *rows,
                          const pct_sweep_params *params, pct_plan *plan, void *workspace, size_t ws_bytes,
                          void *stream) {
  g_err.clear();
  Ctx c;
  pct_status r;
  if ((r = check_grid(grid)) != PCT_OK) return r;
  if ((r = check_hist(hist)) != PCT_OK) return r;
  if ((r = check_rows(rows, hist->n, true)) != PCT_OK) return r;
  if ((r = check_plan_params(params, hist->n)) != PCT_OK) return r;
  if (!plan) return fail(PCT_EINVAL, "plan is NULL");
  c.M = grid_voxels(grid);
  c.Mw = brick_voxels(grid);
  c.n = hist->n;
  c.H = hist_ptrs(hist);
  c.s = reinterpret_cast<hipStream_t>(stream);
  return do_plan_build(c, grid, rows, params, plan, workspace, ws_bytes);
}

pct_status pct_plan_sweep(const pct_grid *grid, const pct_plan *plan, float *x, const pct_sweep_params *params,
                          double *resid_out, void *workspace, size_t ws_bytes, void *stream) {
  g_err.clear();
  pct_status r;
  if ((r = check_grid(grid)) != PCT_OK) return r;
  if ((r = check_plan(plan, grid)) != PCT_OK) return r;
  if ((r = check_plan_params(params, plan->n)) != PCT_OK) return r;
  if (params->block_size != plan->block_size || params->order != plan->order)
    return fail(PCT_EINVAL, "params (order, block_size) differ from those the plan was built for");
  if (!x) return fail(PCT_EINVAL, "x is NULL");
  Ctx c;
  c.M = grid_voxels(grid);
  c.Mw = brick_voxels(grid);
  c.n = plan->n;
  c.extra = tvs_on(params) ? pct::kWsTvs : 0;
  if ((r = check_ws(workspace, ws_bytes, c.Mw, c.n, 0, c.extra)) != PCT_OK) return r;
  c.W = pct::carve_workspace(workspace, c.Mw, c.n, 0, 0, 0, false, c.extra);
  c.s = reinterpret_cast<hipStream_t>(stream);
  const pct::PlanView V = plan_view(plan, len_unit(grid));
  HIPCHECK(pct::launch_fill_u32(c.W.status, 4, 0u, c.s));
  if ((r = do_plan_sweep(c, plan, V, x, params)) != PCT_OK) return r;
  if (resid_out) {
    if ((r = do_plan_residual(c, plan, V, x, resid_out)) != PCT_OK) return r;
    HIPCHECK(pct::launch_poison_on_status(resid_out, c.W.status, c.s));
  }
  return PCT_OK;
}

pct_status pct_plan_residual(const pct_grid *grid, const pct_plan *plan, const float *x, double *out,
                             void *workspace, size_t ws_bytes, void *stream) {
  g_err.clear();
  pct_status r;
  if ((r = check_grid(grid)) != PCT_OK) return r;
  if ((r = check_plan(plan, grid)) != PCT_OK) return r;
  if (!x || !out) return fail(PCT_EINVAL, "x / out is NULL");
  Ctx c;
  c.M = grid_voxels(grid);
  c.Mw = brick_voxels(grid);
  c.n = plan->n;
  (void)workspace;
  (void)ws_bytes;
  c.s = reinterpret_cast<hipStream_t>(stream);
  const pct::PlanView V = plan_view(plan, len_unit(grid));
  return do_plan_residual(c, plan, V, x, out);
}

pct_status pct_reconstruct(const pct_grid *grid, const pct_geom *geom, const pct_histories *hist,
                           const pct_sweep_params *params, pct_rows *rows, pct_plan *plan, float *x_inout,
                           double *resid_host, void *workspace, size_t ws_bytes, void *stream) {
  g_err.clear();
  Ctx c;
  pct_status r;
  if ((r = check_params(params, rows != nullptr)) != PCT_OK) return r;
  if ((r = setup(c, grid, geom, hist, workspace, ws_bytes, stream, tvs_on(params) ? pct::kWsTvs : 0)) != PCT_OK)
    return r;
  if (rows && (r = check_rows(rows, c.n, true)) != PCT_OK) return r;
  if (plan && !rows) return fail(PCT_EINVAL, "a plan needs cached rows");
  if (plan && (r = check_plan_params(params, c.n)) != PCT_OK) return r;
  if (plan && !plan->mem) return fail(PCT_EINVAL, "plan memory is NULL (size it with pct_plan_build first)");
  if (!x_inout) return fail(PCT_EINVAL, "x is NULL");
  pct_status trace_st = PCT_OK;
  int count_mode = 0;  // fused sweeps: keep the per-block counts when the workspace holds them
  if (rows) {
    trace_st = do_trace(c, grid, rows);
    if (trace_st != PCT_OK && trace_st != PCT_ENONFINITE) return trace_st;
  } else {
    const int64_t blk = fused_count_elems(c.Mw, c.n, params);
    const bool all = params->algo == 1 && carve_fused(c, blk);
    if (c.W.blk_cnt) count_mode = 1;
    HIPCHECK(pct::launch_fill_u32(c.W.status, 4, 0u, c.s));
    if (all && (r = prepare_records(c)) != PCT_OK) return r;
  }
  pct::PlanView V;
  if (plan) {
    Ctx cp = c;
    if ((r = do_plan_build(cp, grid, rows, params, plan, workspace, ws_bytes)) != PCT_OK) return r;
    V = plan_view(plan, len_unit(grid));
    HIPCHECK(pct::launch_fill_u32(c.W.status, 4, 0u, c.s));
  }
  double *dres = c.W.partials + (pct::kMaxPartials - 1);
  for (int32_t sw = 0; sw < params->n_sweeps; ++sw) {
    if (plan) {
      if ((r = do_plan_sweep(c, plan, V, x_inout, params)) != PCT_OK) return r;
    } else if ((r = do_sweep(c, grid, rows, x_inout, params, count_mode)) != PCT_OK) {
      return r;
    }
    if (count_mode == 1) {
      // the stored counts serve the later sweeps unless one of them overflowed 16 bits
      uint32_t st = 0;
      if ((r = read_status(c, &st)) != PCT_OK) return r;
      count_mode = (st & pct::kStCountSat) ? 0 : 2;
    }
    if (resid_host) {
      // partial sums use the front of the array; the result sits in its last slot
      if (plan)
        r = do_plan_residual(c, plan, V, x_inout, dres);
      else
        r = do_residual(c, grid, rows, x_inout, dres);
      if (r != PCT_OK) return r;
      HIPCHECK(hipMemcpyAsync(&resid_host[sw], dres, sizeof(double), hipMemcpyDeviceToHost, c.s));
    }
  }
  uint32_t st = 0;
  if ((r = read_status(c, &st)) != PCT_OK) return r;
  r = status_to_code(st);
  if (r != PCT_OK) return r;
  return trace_st;
}

pct_status pct_tvs_apply(const pct_grid *grid, float *x, const uint8_t *hull_mask, const pct_tvs *tvs,
                         void *workspace, size_t ws_bytes, void *stream) {
  g_err.clear();
  pct_status r;
  if ((r = check_grid(grid)) != PCT_OK) return r;
  if (!x || !tvs) return fail(PCT_EINVAL, "x / tvs is NULL");
  if ((r = check_tvs(tvs)) != PCT_OK) return r;
  if (tvs->n_steps == 0) return PCT_OK;
  const int64_t M = grid_voxels(grid);
  const size_t need = pct::tvs_scratch_bytes(M);
  if (!workspace || ws_bytes < need)
    return fail(PCT_ENOMEM, "workspace of %zu bytes given, %zu needed", workspace ? ws_bytes : (size_t)0, need);
  Ctx c;
  c.s = reinterpret_cast<hipStream_t>(stream);
  c.W.tvs = workspace;
  PROF(PCT_K_TVS, run_tvs(c, grid->nx, grid->ny, grid->nz, x, hull_mask, tvs));
  return PCT_OK;
}

pct_status pct_carp(const pct_grid *grid, const pct_geom *geom, const pct_histories *hist,
                    const pct_sweep_params *params, int32_t n_strings, const pct_rows *rows, float *x_inout,
                    double *resid_host, void *workspace, size_t ws_bytes, void *stream) {
  g_err.clear();
  Ctx c;
  pct_status r;
  if ((r = check_params(params, rows != nullptr)) != PCT_OK) return r;
  if (params->algo != 1) return fail(PCT_EINVAL, "CARP strings run DROP sweeps (algo 1)");
  if (n_strings < 1 || n_strings > 4096) return fail(PCT_EINVAL, "n_strings must be 1..4096");
  const int extra = pct::kWsCarp | (tvs_on(params) ? pct::kWsTvs : 0);
  if ((r = setup(c, grid, geom, hist, workspace, ws_bytes, stream, extra)) != PCT_OK) return r;
  if (rows && (r = check_rows(rows, c.n, true)) != PCT_OK) return r;
  if (!x_inout) return fail(PCT_EINVAL, "x is NULL");
  HIPCHECK(pct::launch_fill_u32(c.W.status, 4, 0u, c.s));
  if (!rows && carve_fused(c, 0)) {
    HIPCHECK(pct::launch_fill_u32(c.W.status, 4, 0u, c.s));
    if ((r = prepare_records(c)) != PCT_OK) return r;
  }
  // the strings' sweeps: DROP without TVS (CARP applies it once per iteration)
  pct_sweep_params ps = *params;
  ps.tvs = nullptr;
  PROF(PCT_K_CARP, pct::launch_fill_f32(c.W.carp_acc, c.M, 0.f, c.s));
  HIPCHECK(pct::launch_fill_u8(reinterpret_cast<uint8_t *>(c.W.carp_tc), 2 * c.M, 0, c.s));
  HIPCHECK(pct::launch_fill_u8(c.W.carp_touched, c.M, 0, c.s));
  HIPCHECK(pct::launch_mask(x_inout, params->hull_mask, c.M, c.s));
  double *dres = c.W.partials + (pct::kMaxPartials - 1);
  for (int32_t it = 0; it < params->n_sweeps; ++it) {
    if (tvs_on(params)) PROF(PCT_K_TVS, run_tvs(c, grid->nx, grid->ny, grid->nz, x_inout, params->hull_mask,
                                                params->tvs));
    for (int32_t s = 0; s < n_strings; ++s) {
      const int64_t p0 = c.n * s / n_strings, p1 = c.n * (s + 1) / n_strings;
      PROF(PCT_K_CARP, pct::launch_copy_f32(x_inout, c.W.carp_xs, c.M, c.s));
      if ((r = do_sweep(c, grid, rows, c.W.carp_xs, &ps, 0, p0, p1, c.W.carp_touched)) != PCT_OK) return r;
      PROF(PCT_K_CARP, pct::launch_carp_accumulate(c.W.carp_xs, c.W.carp_touched, c.W.carp_acc, c.W.carp_tc, c.M,
                                                   c.s));
    }
    PROF(PCT_K_CARP, pct::launch_carp_average(x_inout, c.W.carp_acc, c.W.carp_tc, c.M, c.s));
    if (resid_host) {
      if ((r = do_residual(c, grid, rows, x_inout, dres)) != PCT_OK) return r;
      HIPCHECK(hipMemcpyAsync(&resid_host[it], dres, sizeof(double), hipMemcpyDeviceToHost, c.s));
    }
  }
  uint32_t st = 0;
  if ((r = read_status(c, &st)) != PCT_OK) return r;
  return status_to_code(st);
}

pct_status pct_carve_hull(const pct_grid *grid, const pct_geom *geom, const pct_histories *hist, float wepl_max,
                          float min_len, uint8_t *hull_out, int64_t *n_used, void *workspace, size_t ws_bytes,
                          void *stream) {
  g_err.clear();
  pct_status r;
  pct::PathParams P;
  if ((r = check_grid(grid)) != PCT_OK) return r;
  if ((r = check_hist(hist)) != PCT_OK) return r;
  if ((r = make_params(grid, geom, P)) != PCT_OK) return r;
  if (!hull_out) return fail(PCT_EINVAL, "hull_out is NULL");
  if (!std::isfinite(wepl_max) || !(min_len >= 0.f) || !std::isfinite(min_len))
    return fail(PCT_EINVAL, "wepl_max must be finite and min_len >= 0");
  if (!workspace || ws_bytes < 256) return fail(PCT_ENOMEM, "workspace of at least 256 bytes needed");
  Ctx c;
  c.s = reinterpret_cast<hipStream_t>(stream);
  unsigned long long *used = static_cast<unsigned long long *>(workspace);
  const int64_t M = grid_voxels(grid);
  HIPCHECK(pct::launch_fill_u8(hull_out, M, 1, c.s));
  HIPCHECK(pct::launch_fill_u32(reinterpret_cast<uint32_t *>(used), 2, 0u, c.s));
  PROF(PCT_K_CARVE, pct::launch_carve(P, hist_ptrs(hist), hist->n, (double)wepl_max, (double)min_len, hull_out,
                                      used, c.s));
  if (n_used) {
    unsigned long long u = 0;
    HIPCHECK(hipMemcpyAsync(&u, used, sizeof u, hipMemcpyDeviceToHost, c.s));
    HIPCHECK(hipStreamSynchronize(c.s));
    *n_used = (int64_t)u;
  }
  return PCT_OK;
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
  if (!rows && carve_fused(c, 0)) {
    HIPCHECK(pct::launch_fill_u32(c.W.status, 4, 0u, c.s));
    if ((r = prepare_records(c)) != PCT_OK) return r;
  }
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
      // the events are reused: wait for the last recorded ones (a failed
      // wait leaves nothing to do for a timing record that is discarded)
      (void)hipEventSynchronize(r.b);
      g_prof_pool.push_back(r.a);
      g_prof_pool.push_back(r.b);
    }
    g_prof.clear();
  }
  g_prof_on = on != 0;
  return PCT_OK;
}

pct_status pct_probe(int32_t kind, void *buf, size_t buf_bytes, int64_t region, int64_t n_ops, int32_t reps,
                     double *ms_out, void *stream) {
  g_err.clear();
  if (kind < PCT_PROBE_COPY || kind > PCT_PROBE_LDS_ATOMIC) return fail(PCT_EINVAL, "unknown probe kind %d", kind);
  if (!ms_out) return fail(PCT_EINVAL, "ms_out is NULL");
  if (reps < 1 || reps > 1000) return fail(PCT_EINVAL, "reps must be 1..1000");
  if (kind != PCT_PROBE_LDS_ATOMIC && (region < 64 || region > 0x7fffffffLL))
    return fail(PCT_EINVAL, "region must be 64..2^31-1 elements");
  if (kind == PCT_PROBE_COPY && region % 4 != 0) return fail(PCT_EINVAL, "copy region must be a multiple of 4");
  if ((kind == PCT_PROBE_GATHER || kind == PCT_PROBE_ATOMIC || kind == PCT_PROBE_ATOMIC_XCD) && region % 160000 != 0)
    return fail(PCT_EINVAL, "gather and atomic regions must be whole 200 x 200 x 4 slabs (multiples of 160000)");
  if (kind != PCT_PROBE_COPY && (n_ops < 64 * pct::kProbeGrid || n_ops > (int64_t)1 << 40))
    return fail(PCT_EINVAL, "n_ops must be %lld..2^40", (long long)(64 * pct::kProbeGrid));
  const size_t need = pct::probe_bytes(kind, region, n_ops, pct::kProbeGrid);
  if (!buf || buf_bytes < need)
    return fail(PCT_ENOMEM, "probe buffer of %zu bytes given, %zu needed", buf ? buf_bytes : (size_t)0, need);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t a = nullptr, b = nullptr;
  HIPCHECK(hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return fail(PCT_EDEVICE, "hipEventCreate failed");
  }
  hipError_t e = hipEventRecord(a, s);
  for (int32_t r = 0; r < reps && e == hipSuccess; ++r) e = pct::launch_probe(kind, buf, region, n_ops, pct::kProbeGrid, s);
  if (e == hipSuccess) e = hipEventRecord(b, s);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return fail(PCT_EDEVICE, "probe: %s", hipGetErrorString(e));
  *ms_out = (double)ms / reps;
  return PCT_OK;
}

size_t pct_probe_bytes(int32_t kind, int64_t region, int64_t n_ops) {
  if (kind < PCT_PROBE_COPY || kind > PCT_PROBE_LDS_ATOMIC || region < 0 || n_ops < 0) return 0;
  return pct::probe_bytes(kind, region, n_ops, pct::kProbeGrid);
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

// ---- warm-start network operations
#define CNN_VOL_CHECK(C, D, H, W)                                                                       \
  do {                                                                                                  \
    if ((C) <= 0 || (D) <= 0 || (H) <= 0 || (W) <= 0) return fail(PCT_EINVAL, "sizes must be positive"); \
    if ((int64_t)(D) * (H) * (W) >= (int64_t(1) << 31)) return fail(PCT_EINVAL, "volume has 2^31 voxels or more"); \
  } while (0)

pct_status pct_cnn_conv3d(const float *x, const float *w, const float *b, float *y, int32_t cin, int32_t cout,
                          int32_t D, int32_t H, int32_t W, void *stream) {
  g_err.clear();
  CNN_VOL_CHECK(cin, D, H, W);
  if (cout <= 0) return fail(PCT_EINVAL, "cout must be positive");
  if (!x || !w || !y) return fail(PCT_EINVAL, "NULL tensor");
  HIPCHECK(pct::cnn::conv3d(x, w, b, y, cin, cout, D, H, W, reinterpret_cast<hipStream_t>(stream)));
  return PCT_OK;
}

pct_status pct_cnn_conv3d_bwd_data(const float *dy, const float *w, float *dx, float *wt, int32_t cin, int32_t cout,
                                   int32_t D, int32_t H, int32_t W, void *stream) {
  g_err.clear();
  CNN_VOL_CHECK(cin, D, H, W);
  if (cout <= 0) return fail(PCT_EINVAL, "cout must be positive");
  if (!dy || !w || !dx || !wt) return fail(PCT_EINVAL, "NULL tensor");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIPCHECK(pct::cnn::flip_weights(w, wt, cin, cout, s));
  HIPCHECK(pct::cnn::conv3d(dy, wt, nullptr, dx, cout, cin, D, H, W, s));
  return PCT_OK;
}

int64_t pct_cnn_conv3d_bf16_scratch(int32_t cin, int32_t cout) {
  return pct::cnn::mfma_shape_ok(cin, cout) ? pct::cnn::mfma_pack_bytes(cin, cout) : 0;
}

pct_status pct_cnn_conv3d_bf16(const float *x, const float *w, const float *b, float *y, void *wpack, int32_t cin,
                               int32_t cout, int32_t D, int32_t H, int32_t W, void *stream) {
  g_err.clear();
  CNN_VOL_CHECK(cin, D, H, W);
  if (!pct::cnn::mfma_shape_ok(cin, cout))
    return fail(PCT_EINVAL, "bf16 convolution needs cin %% 8 == 0 and cout %% 16 == 0 (got %d, %d)", cin, cout);
  if (!x || !w || !y || !wpack) return fail(PCT_EINVAL, "NULL tensor");
  HIPCHECK(pct::cnn::conv3d_mfma(x, w, b, y, wpack, cin, cout, D, H, W, reinterpret_cast<hipStream_t>(stream)));
  return PCT_OK;
}

pct_status pct_cnn_conv3d_bwd_data_bf16(const float *dy, const float *w, float *dx, float *wt, void *wpack,
                                        int32_t cin, int32_t cout, int32_t D, int32_t H, int32_t W, void *stream) {
  g_err.clear();
  CNN_VOL_CHECK(cin, D, H, W);
  if (!pct::cnn::mfma_shape_ok(cout, cin))
    return fail(PCT_EINVAL, "bf16 input gradient needs cout %% 8 == 0 and cin %% 16 == 0 (got %d, %d)", cin, cout);
  if (!dy || !w || !dx || !wt || !wpack) return fail(PCT_EINVAL, "NULL tensor");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  HIPCHECK(pct::cnn::flip_weights(w, wt, cin, cout, s));
  HIPCHECK(pct::cnn::conv3d_mfma(dy, wt, nullptr, dx, wpack, cout, cin, D, H, W, s));
  return PCT_OK;
}

int64_t pct_cnn_wgrad_scratch(int32_t cin, int32_t cout, int32_t D, int32_t H, int32_t W) {
  if (cin <= 0 || cout <= 0 || D <= 0 || H <= 0 || W <= 0) return 0;
  int64_t parts = pct::cnn::wgrad_chunks(D, H, W);
  if (pct::cnn::mfma_wgrad_ok(cin, cout)) parts = std::max(parts, pct::cnn::wgrad_mfma_slabs(cin, cout, D, H, W));
  return parts * cout * ((int64_t)cin * 27 + 1);
}

pct_status pct_cnn_conv3d_bwd_weight(const float *x, const float *dy, float *dw, float *db, float *scratch,
                                     int32_t cin, int32_t cout, int32_t D, int32_t H, int32_t W, void *stream) {
  g_err.clear();
  CNN_VOL_CHECK(cin, D, H, W);
  if (cout <= 0) return fail(PCT_EINVAL, "cout must be positive");
  if (!x || !dy || !dw || !scratch) return fail(PCT_EINVAL, "NULL tensor");
  HIPCHECK(pct::cnn::conv3d_wgrad(x, dy, dw, db, scratch, cin, cout, D, H, W, reinterpret_cast<hipStream_t>(stream)));
  return PCT_OK;
}

pct_status pct_cnn_conv3d_bwd_weight_bf16(const float *x, const float *dy, float *dw, float *db, float *scratch,
                                          int32_t cin, int32_t cout, int32_t D, int32_t H, int32_t W, void *stream) {
  g_err.clear();
  CNN_VOL_CHECK(cin, D, H, W);
  if (!pct::cnn::mfma_wgrad_ok(cin, cout))
    return fail(PCT_EINVAL, "bf16 weight gradient needs cin %% 16 == 0 and cout %% 16 == 0 (got %d, %d)", cin, cout);
  if ((int64_t)D * H * W >= (int64_t(1) << 27))
    return fail(PCT_EINVAL, "bf16 weight gradient needs a volume of fewer than 2^27 voxels");
  if (!x || !dy || !dw || !scratch) return fail(PCT_EINVAL, "NULL tensor");
  HIPCHECK(pct::cnn::conv3d_wgrad_mfma(x, dy, dw, db, scratch, cin, cout, D, H, W,
                                       reinterpret_cast<hipStream_t>(stream)));
  return PCT_OK;
}

pct_status pct_cnn_relu(const float *x, float *y, int64_t n, void *stream) {
  g_err.clear();
  if (n < 0 || (n > 0 && (!x || !y))) return fail(PCT_EINVAL, "bad relu arguments");
  HIPCHECK(pct::cnn::relu(x, y, n, reinterpret_cast<hipStream_t>(stream)));
  return PCT_OK;
}

pct_status pct_cnn_relu_bwd(const float *y, const float *dy, float *dx, int64_t n, void *stream) {
  g_err.clear();
  if (n < 0 || (n > 0 && (!y || !dy || !dx))) return fail(PCT_EINVAL, "bad relu_bwd arguments");
  HIPCHECK(pct::cnn::relu_bwd(y, dy, dx, n, reinterpret_cast<hipStream_t>(stream)));
  return PCT_OK;
}

pct_status pct_cnn_pool(const float *x, float *y, int32_t C, int32_t D, int32_t H, int32_t W, void *stream) {
  g_err.clear();
  CNN_VOL_CHECK(C, D, H, W);
  if ((D | H | W) & 1) return fail(PCT_EINVAL, "pooling needs even D, H, W");
  if (!x || !y) return fail(PCT_EINVAL, "NULL tensor");
  HIPCHECK(pct::cnn::pool(x, y, C, D, H, W, reinterpret_cast<hipStream_t>(stream)));
  return PCT_OK;
}

pct_status pct_cnn_pool_bwd(const float *dy, float *dx, int32_t C, int32_t D, int32_t H, int32_t W, void *stream) {
  g_err.clear();
  CNN_VOL_CHECK(C, D, H, W);
  if ((D | H | W) & 1) return fail(PCT_EINVAL, "pooling needs even D, H, W");
  if (!dy || !dx) return fail(PCT_EINVAL, "NULL tensor");
  HIPCHECK(pct::cnn::pool_bwd(dy, dx, C, D, H, W, reinterpret_cast<hipStream_t>(stream)));
  return PCT_OK;
}

pct_status pct_cnn_upsample(const float *x, float *y, int32_t C, int32_t d, int32_t h, int32_t w, void *stream) {
  g_err.clear();
  CNN_VOL_CHECK(C, 2 * d, 2 * h, 2 * w);
  if (!x || !y) return fail(PCT_EINVAL, "NULL tensor");
  HIPCHECK(pct::cnn::upsample(x, y, C, d, h, w, reinterpret_cast<hipStream_t>(stream)));
  return PCT_OK;
}

pct_status pct_cnn_upsample_bwd(const float *dy, float *dx, int32_t C, int32_t d, int32_t h, int32_t w,
                                void *stream) {
  g_err.clear();
  CNN_VOL_CHECK(C, 2 * d, 2 * h, 2 * w);
  if (!dy || !dx) return fail(PCT_EINVAL, "NULL tensor");
  HIPCHECK(pct::cnn::upsample_bwd(dy, dx, C, d, h, w, reinterpret_cast<hipStream_t>(stream)));
  return PCT_OK;
}

pct_status pct_cnn_add(const float *a, const float *b, float *y, int64_t n, void *stream) {
  g_err.clear();
  if (n < 0 || (n > 0 && (!a || !b || !y))) return fail(PCT_EINVAL, "bad add arguments");
  HIPCHECK(pct::cnn::add(a, b, y, n, reinterpret_cast<hipStream_t>(stream)));
  return PCT_OK;
}

pct_status pct_cnn_axpy(float a, const float *x, float *y, int64_t n, void *stream) {
  g_err.clear();
  if (n < 0 || (n > 0 && (!x || !y))) return fail(PCT_EINVAL, "bad axpy arguments");
  HIPCHECK(pct::cnn::axpy(a, x, y, n, reinterpret_cast<hipStream_t>(stream)));
  return PCT_OK;
}

pct_status pct_cnn_mask(const float *x, const uint8_t *mask, float *y, int64_t n, void *stream) {
  g_err.clear();
  if (n < 0 || (n > 0 && (!x || !mask || !y))) return fail(PCT_EINVAL, "bad mask arguments");
  HIPCHECK(pct::cnn::mask(x, mask, y, n, reinterpret_cast<hipStream_t>(stream)));
  return PCT_OK;
}

int64_t pct_cnn_mse_scratch(int64_t n) { return n > 0 ? pct::cnn::mse_parts(n) : 0; }

pct_status pct_cnn_mse(const float *y, const float *t, float *dy, double *scratch, double *loss, int64_t n,
                       void *stream) {
  g_err.clear();
  if (n <= 0 || !y || !t || !scratch || !loss) return fail(PCT_EINVAL, "bad mse arguments");
  HIPCHECK(pct::cnn::mse(y, t, dy, scratch, loss, n, reinterpret_cast<hipStream_t>(stream)));
  return PCT_OK;
}

pct_status pct_cnn_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float beta1, float beta2,
                        float eps, int32_t step, void *stream) {
  g_err.clear();
  if (n < 0 || (n > 0 && (!w || !g || !m || !v))) return fail(PCT_EINVAL, "bad adam arguments");
  if (step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return fail(PCT_EINVAL, "bad adam hyper-parameters");
  HIPCHECK(pct::cnn::adam(w, g, m, v, n, lr, beta1, beta2, eps, step, reinterpret_cast<hipStream_t>(stream)));
  return PCT_OK;
}

}  // extern "C"
