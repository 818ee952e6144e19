/*
 * pct.h -- C ABI of the MI355X event-by-event proton CT reconstruction library
 * (libpct.so).
 *
 * The problem (paper Sec. 2): N proton histories, each with an entry position
 * and direction measured by the upstream tracker pair, an exit position and
 * direction measured by the downstream pair, and a water-equivalent path
 * length (WEPL).  The object is a rectangular grid of M voxels whose relative
 * stopping power (RSP) x is sought.  Each proton's most-likely path (MLP)
 * through the object gives one row of the sparse matrix A: the path lengths
 * in the voxels it touches.  The WEPL values form b, and Ax = b is solved by
 * block-iterative row projections (DROP, Sec. 2.1), ART being the block size
 * one case.  (The paper writes A as M x N with one column per proton; with b
 * of length N and x of length M, this library stores A as N x M, one row per
 * proton.)
 *
 * Conventions for every entry point:
 *   - Pointers documented as "device" are HIP device memory owned by the
 *     caller; the library never allocates device memory: scratch space comes
 *     from the caller's `workspace` of pct_workspace_size() bytes.
 *   - `stream` is a hipStream_t (NULL = the default stream); all device work
 *     is enqueued on it.  Calls that must read a device value on the host
 *     (row totals, residuals, device status) synchronise that stream.
 *   - Argument errors are detected on the host before any launch; then nothing
 *     is modified and PCT_EINVAL is returned.  Errors found on the device are
 *     reported by the next call that synchronises.
 *   - pct_last_error() gives a thread-local message for the last failure.
 *   - No C++ exception crosses this interface.
 */
#ifndef PCT_H
#define PCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PCT_OK = 0,
    PCT_EINVAL = -1,      /* bad argument (checked on the host, nothing modified) */
    PCT_ENOMEM = -2,      /* workspace smaller than pct_workspace_size() */
    PCT_EDEVICE = -3,     /* a HIP call failed, or a device-side bound was exceeded */
    PCT_EROWCAP = -4,     /* cached rows do not fit in pct_rows.cap_nnz */
    PCT_ENONFINITE = -5   /* some histories hold NaN/Inf; their rows were left empty */
} pct_status;

/* Voxel grid (Sec. 2: a discrete rectangular grid of M voxels, x an
 * M-element linearised array).  Voxel (i, j, k) covers
 * [o + i d, o + (i + 1) d) on each axis (half-open); its linear index is
 * (k * ny + j) * nx + i.  Object frame in mm, isocentre at the origin. */
typedef struct {
    int32_t nx, ny, nz;
    float dx, dy, dz;
    float ox, oy, oz;
} pct_grid;

/* Scanner geometry and the scattering prior of the most-likely path.
 * Beam frame for gantry angle phi: u along (cos phi, sin phi, 0), t along
 * (-sin phi, cos phi, 0), v along z.  The tracker planes sit at u = u_in and
 * u = u_out.  The object hull is the elliptic cylinder (x/hull_a)^2 +
 * (y/hull_b)^2 <= 1, hull_zmin <= z <= hull_zmax; the path is straight
 * outside it and most-likely inside it, sampled every <= step_mm
 * (0 < step_mm <= min(dx, dy, dz)).  The prior's 1/(beta p)^2 is the
 * polynomial sum_n poly[n] s^n (MeV^-2) in depth s (mm) from the hull entry;
 * highland_log = 1 multiplies each covariance by (1 + 0.038 ln(d / X0_mm))^2
 * for its interval length d.  E0_MeV scales both covariances alike and does
 * not change the path; it is kept for completeness.  path_fp32 = 0 computes
 * path positions in FP64 (coordinates good to ~1e-12 mm); 1 computes them in
 * FP32 (reduced-precision variant, ~1e-5 mm at 100 mm from the isocentre);
 * the voxel walk uses the same precision on sub-voxel coordinates. */
typedef struct {
    float u_in, u_out;
    float hull_a, hull_b, hull_zmin, hull_zmax;
    float step_mm;
    int32_t highland_log;
    int32_t n_poly;          /* 1..8 */
    int32_t path_fp32;       /* 0 or 1 */
    int32_t reserved;        /* must be 0 */
    double poly[8];
    double E0_MeV, X0_mm;
} pct_geom;

/* Proton histories (Sec. 2: entry and exit positions and directions from the
 * two tracker pairs, WEPL from the range detector), structure of arrays,
 * float32, device memory, length n each.  Positions t, v at the tracker
 * planes (mm), directions as slopes dt/du, dv/du, WEPL in mm (this is b). */
typedef struct {
    int64_t n;
    const float *phi, *t_in, *v_in, *dt_in, *dv_in;
    const float *t_out, *v_out, *dt_out, *dv_out, *wepl;
} pct_histories;

/* Cached rows of A (CSR).  Row i belongs to history i.  Entries of a row
 * follow the path from entry to exit; each voxel appears at most once.
 * len_dtype 0: float32 lengths (mm); 1: float16 lengths in units of
 * min(dx, dy, dz).  norm2[i] = sum of squared lengths (mm^2), FP64, computed
 * from the float32 lengths before any float16 rounding.  All arrays device,
 * caller-owned: row_ptr [n_rows + 1], idx/len [cap_nnz], norm2 [n_rows].
 * `nnz` is written by pct_mlp_trace (host field). */
typedef struct {
    int64_t n_rows;
    int64_t cap_nnz;
    int64_t nnz;
    int64_t *row_ptr;
    int32_t *idx;
    void *len;
    int32_t len_dtype;
    double *norm2;
} pct_rows;

/* Total-variation superiorization (Sec. 4.2, the Table 2 discussion: both
 * of the paper's pipelines perturb the image towards lower total variation,
 * DROP before every block, CARP once per iteration; it is what gives DROP its
 * lower noise).  The paper gives no formula; the library takes the
 * superiorization step of the pCT literature it builds on, in 3D:
 *   TV(x) = sum over voxels of sqrt(dx^2 + dy^2 + dz^2 + eps^2) with forward
 *   differences (0 at a grid's last plane), g = dTV/dx (0 outside the hull
 *   mask); a step tries x - beta g / ||g||, multiplies beta by `a` after every
 *   trial, keeps the first trial with TV not above TV(x), and gives up after
 *   max_trials trials.  n_steps steps per application.
 * state: device double[8], caller-owned; state[0] = the current beta (set it
 * to the initial step size before the first call; the library shrinks it),
 * state[5] counts the steps kept; the other slots are the library's.  TV
 * sums are FP64 in a fixed order, the image stays float32. */
typedef struct {
    int32_t n_steps;         /* 0 = off */
    int32_t max_trials;      /* 1..16 */
    double a;                /* 0 < a < 1 */
    double eps;              /* > 0 */
    double *state;
} pct_tvs;

/* Block-iterative solver parameters (Sec. 2.1).  Rows are visited in the
 * order `order` (device int64 [n], a permutation of 0..n-1; NULL = identity)
 * in consecutive blocks of block_size rows (the last block may be short).
 * algo 1 (DROP): for each block, with x fixed at its block-start value,
 *   r_i = (b_i - a_i.x) / ||a_i||^2, x_j += lambda * sum_i r_i a_ij / s_j,
 *   s_j = number of rows of the block that touch voxel j.
 * algo 0 (ART): the same with block_size 1, rows strictly one after another
 *   (cached rows only).
 * hull_mask (device uint8 [M], NULL = none): voxels with 0 are held at 0.
 * n_sweeps: passes over all blocks (Sec. 2.1: a fixed iteration count).
 * tvs (host struct, NULL = none): DROP applies its steps to the image that
 *   enters every block (not with ART). */
typedef struct {
    int32_t algo;
    int64_t block_size;
    float lambda;            /* 0 < lambda < 2 */
    int32_t n_sweeps;
    const int64_t *order;
    const uint8_t *hull_mask;
    const pct_tvs *tvs;
} pct_sweep_params;

/* A sweep plan: cached rows regrouped, block by block, into lists per spatial
 * tile of 16 x 16 x 8 voxels (row pieces), which both the projections and the
 * update read, so that a DROP block runs without global atomics.  The update
 * adds each tile's contributions in on-chip memory as 64-bit fixed-point
 * integers (r_i a_ij scaled by 2^(58 - ceil(log2 block_size)) and rounded),
 * so its sums do not depend on the order of the additions; a contribution of
 * magnitude 16 or more is added in float32 instead.  `entries` counts the
 * padded list entries, `refs` the reference slots reserved per row (an upper
 * bound on piece ends), `ends` the piece ends (a piece, or its part in one
 * 64-entry chunk, gives one partial dot product).  It describes the same
 * matrix A as the rows it was built from, for one block order and block size,
 * and holds b and ||a_i||^2 in block order.  `mem` is caller-owned device
 * memory of `bytes` bytes; the other fields are written by pct_plan_build and
 * describe the layout.  A plan is used by one stream at a time. */
typedef struct {
    void *mem;
    size_t bytes;
    int64_t n, block_size, n_blocks, n_tiles;
    int64_t entries, chunks, refs, max_chunks, max_ends, ends;
    int32_t len_dtype, nx, ny, nz;
    const void *order, *rows_idx;
    int32_t ready, reserved;
} pct_plan;

/* Bytes of scratch that the calls below need for a grid, solver and history
 * count.  `fused` = 1 when rows are recomputed in every sweep (no plan).  With
 * geom given and fused = 0 the size includes the row staging area of the
 * trace (up to 2^20 rows of the longest possible row: 2 entries per path
 * sample + 16, 8 bytes per entry); a
 * trace given less stages fewer rows at a time (PCT_ENOMEM below one row).
 * With fused = 1 the size includes one path set-up record per history (128
 * bytes: hull entry and exit, end states, the prior's moments at the exit,
 * b_i), formed once per call and read by every later path pass; a fused call
 * given less sets up each block's histories just before projecting them.
 * With fused = 1 and params of a DROP run of two or more sweeps the size also
 * includes the per-block voxel counts s_j (n_blocks x M x 2 bytes, kept up to
 * 32 GiB): pct_reconstruct then forms them in its first sweep and reads them
 * back in the later ones instead of counting again with atomics (the block
 * composition is the same every sweep, Sec. 2.1); with a smaller workspace it
 * counts in every sweep.  The same workspace may be reused by consecutive
 * calls on one stream. */
size_t pct_workspace_size(const pct_grid *grid, const pct_geom *geom, const pct_sweep_params *params,
                          int64_t n_hist, int32_t fused);

/* Rows of A for all histories (Sec. 2: MLP per proton, then the path length
 * in each voxel it touches).  One path pass per proton: rows are built into
 * the workspace's staging area chunk by chunk, then compacted into CSR.  If
 * rows->idx is NULL only row_ptr and rows->nnz are produced (a sizing call).
 * If the total exceeds rows->cap_nnz, row_ptr and nnz are written, the rows
 * that fit are written, and PCT_EROWCAP is returned.  Histories with NaN/Inf get empty rows and the call
 * returns PCT_ENONFINITE after finishing the rest.  Synchronises `stream`. */
pct_status pct_mlp_trace(const pct_grid *grid, const pct_geom *geom, const pct_histories *hist,
                         pct_rows *rows, void *workspace, size_t ws_bytes, void *stream);

/* One sweep of the block-iterative solver over all histories (Sec. 2.1),
 * updating x (device float32 [M]) in place.  rows != NULL: cached rows from
 * pct_mlp_trace; rows == NULL: every row is recomputed from the histories
 * inside the sweep and never stored.  b is hist->wepl.  resid_out (device
 * double, or NULL): ||Ax - b||_2 over non-empty rows after the sweep, FP64;
 * it is set to NaN if the device found an error during the sweep (an order
 * entry outside [0, n), a cached voxel index outside [0, M), a row bound
 * exceeded).  params->n_sweeps is ignored (one sweep).  Asynchronous. */
pct_status pct_project_sweep(const pct_grid *grid, const pct_geom *geom, const pct_histories *hist,
                             const pct_rows *rows, float *x, const pct_sweep_params *params, double *resid_out,
                             void *workspace, size_t ws_bytes, void *stream);

/* pct_project_sweep over cached rows for callers that cannot allocate or
 * pass device memory of their own: code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation.  Same arguments and
 * results as pct_project_sweep with rows != NULL, but no workspace: the
 * sweep's scratch (status word, DROP numerators and counts, residual partial
 * sums; 16.5 MiB) is a static device array of the library, one per GPU,
 * held until the process ends.  Nothing is allocated by the call.  The grid
 * may hold at most 2^21 voxels (PCT_EINVAL beyond); rows must be given
 * (PCT_EINVAL for NULL) and TV superiorization is not available here
 * (PCT_EINVAL if params->tvs asks for steps).  The array keeps the last
 * call's contents; each call clears what it needs.  Every call on one GPU
 * shares that GPU's array, so calls that overlap on one GPU (several
 * streams or threads at once) race and give undefined results.  Runs on the
 * device current on the calling thread.  Asynchronous. */
pct_status pct_project_sweep_noalloc(const pct_grid *grid, const pct_geom *geom, const pct_histories *hist,
                                     const pct_rows *rows, float *x, const pct_sweep_params *params,
                                     double *resid_out, void *stream);

/* Build the sweep plan of cached rows for params (DROP, block_size <= 2^18;
 * b from hist->wepl).  With plan->mem == NULL this is a sizing call: it sets
 * plan->bytes and returns PCT_OK.  Otherwise plan->bytes must be at least the
 * size a sizing call reports (else PCT_ENOMEM, with the size in plan->bytes).
 * Synchronises `stream`. */
pct_status pct_plan_build(const pct_grid *grid, const pct_histories *hist, const pct_rows *rows,
                          const pct_sweep_params *params, pct_plan *plan, void *workspace, size_t ws_bytes,
                          void *stream);

/* One DROP sweep over all blocks with a plan (same result as
 * pct_project_sweep on the rows the plan was built from, up to the order of
 * floating-point additions).  params must match the plan's order and
 * block_size.  resid_out as in pct_project_sweep.  Asynchronous. */
pct_status pct_plan_sweep(const pct_grid *grid, const pct_plan *plan, float *x, const pct_sweep_params *params,
                          double *resid_out, void *workspace, size_t ws_bytes, void *stream);

/* ||Ax - b||_2 (FP64) with a plan, into *out (device double).  Asynchronous. */
pct_status pct_plan_residual(const pct_grid *grid, const pct_plan *plan, const float *x, double *out,
                             void *workspace, size_t ws_bytes, void *stream);

/* Whole reconstruction: if rows != NULL, trace into them first (as
 * pct_mlp_trace); if plan != NULL too, build the plan (as pct_plan_build) and
 * sweep with it; then params->n_sweeps sweeps from x_inout (the initial
 * guess, Sec. 2.1).  resid_host (host double [n_sweeps], or NULL): residual
 * after each sweep.  Synchronises `stream`. */
pct_status pct_reconstruct(const pct_grid *grid, const pct_geom *geom, const pct_histories *hist,
                           const pct_sweep_params *params, pct_rows *rows, pct_plan *plan, float *x_inout,
                           double *resid_host, void *workspace, size_t ws_bytes, void *stream);

/* The TV superiorization steps of `tvs` applied once to x (device float32
 * [M]), voxels with hull_mask 0 (device uint8 [M] or NULL) left as they are.
 * workspace: pct_workspace_size() of the grid with params holding tvs (or at
 * least 4 M + 16 ceil(M / 256) + 512 bytes).  Asynchronous. */
pct_status pct_tvs_apply(const pct_grid *grid, float *x, const uint8_t *hull_mask, const pct_tvs *tvs,
                         void *workspace, size_t ws_bytes, void *stream);

/* CARP (Sec. 2.2, component-averaged row projections): the positions of
 * params->order are split into n_strings consecutive strings (string s holds
 * positions [n s / S, n (s+1) / S)); every iteration (params->n_sweeps of
 * them) each string starts from the same x and runs one DROP sweep over its
 * own rows, in blocks of params->block_size from the string's start, into an
 * image of its own; then every voxel becomes the mean of the string images
 * over the strings whose rows touch it (others keep their value).  With
 * params->tvs, its steps are applied once to x at the start of every
 * iteration.  rows != NULL: cached rows from pct_mlp_trace; rows == NULL:
 * rows recomputed in every block.  1 <= n_strings <= 4096.
 * resid_host (host double [n_sweeps] or NULL): ||Ax - b|| after each
 * iteration.  Workspace: pct_workspace_size() plus 12 M bytes (string image,
 * sums, string counts, touched flags) -- pct_carp_workspace_size().
 * Synchronises `stream`. */
size_t pct_carp_workspace_size(const pct_grid *grid, const pct_geom *geom, const pct_sweep_params *params,
                               int64_t n_hist, int32_t fused);
pct_status pct_carp(const pct_grid *grid, const pct_geom *geom, const pct_histories *hist,
                    const pct_sweep_params *params, int32_t n_strings, const pct_rows *rows, float *x_inout,
                    double *resid_host, void *workspace, size_t ws_bytes, void *stream);

/* Space-carving hull (a hull from the data, for objects with no known
 * outline): a history whose WEPL is below wepl_max crossed only air, so each
 * voxel its straight entry line (entry position and slope, from u_in to
 * u_out) passes through for more than min_len mm is outside the object.
 * hull_out (device uint8 [M]) is set to 1 everywhere, then to 0 on every
 * carved voxel; it can serve as pct_sweep_params.hull_mask.  n_used (host,
 * or NULL): histories used (synchronises `stream` when given).  Voxels are
 * cut along the line by plane-crossing parameters (plane - p) / (q - p) in
 * FP64, a sub-interval's voxel taken at its midpoint. */
pct_status pct_carve_hull(const pct_grid *grid, const pct_geom *geom, const pct_histories *hist, float wepl_max,
                          float min_len, uint8_t *hull_out, int64_t *n_used, void *workspace, size_t ws_bytes,
                          void *stream);

/* ||Ax - b||_2 over non-empty rows (FP64) into *out (device double).
 * rows == NULL recomputes the rows.  Asynchronous. */
pct_status pct_residual(const pct_grid *grid, const pct_geom *geom, const pct_histories *hist,
                        const pct_rows *rows, const float *x, double *out, void *workspace, size_t ws_bytes,
                        void *stream);

/* ROI analysis (Sec. 3.2, 4.2): for labels 1..n_labels, sums[l-1] = sum of
 * x over voxels with label l (FP64), counts[l-1] = their number.  labels
 * device uint8 [M] (0 = no ROI), sums device double [n_labels], counts
 * device int64 [n_labels]; n_labels <= 255.  Asynchronous. */
pct_status pct_roi_stats(const float *x, const uint8_t *labels, int64_t M, int32_t n_labels, double *sums,
                         int64_t *counts, void *stream);

/* Kernel timing with HIP events, for benchmarking (off by default).
 * pct_profile_enable(1) clears the counters and records an event pair on the
 * launching stream around every kernel the calls above launch;
 * pct_profile_enable(0) stops recording.  pct_profile_read waits for the
 * recorded events and returns, per kernel class, the number of launches and
 * their summed device time in ms (arrays of PCT_K_COUNT, host memory).
 * Recording adds host work per launch; leave it off outside measurements. */
enum {
    PCT_K_TRACE_PATH = 0,    /* MLP + voxel walk of every proton (staged rows) */
    PCT_K_TRACE_COMPACT = 1, /* staged rows -> CSR */
    PCT_K_PROJECT = 2,       /* block projection + scatter (cached or fused) */
    PCT_K_APPLY = 3,         /* block update of x */
    PCT_K_RESIDUAL = 4,      /* ||Ax - b|| */
    PCT_K_ART = 5,           /* sequential ART */
    PCT_K_OTHER = 6,         /* fills, scans, masks */
    PCT_K_PLAN_DOT = 7,      /* plan: partial dot products per piece */
    PCT_K_PLAN_ROWS = 8,     /* plan: r_i per row */
    PCT_K_PLAN_SCATTER = 9,  /* plan: per-tile accumulation + block update */
    PCT_K_PLAN_BUILD = 10,   /* plan construction */
    PCT_K_PATH_SETUP = 11,   /* per-proton path set-up (hull, end states), one thread per proton */
    PCT_K_TVS = 12,          /* total-variation superiorization steps */
    PCT_K_CARP = 13,         /* CARP string copies, sums and averages */
    PCT_K_CARVE = 14,        /* space-carving hull */
    PCT_K_PROJECT_COUNTING = 15, /* rebuilt-row projection that also counts s_j (atomics; first sweep) */
    PCT_K_COUNT = 16
};
pct_status pct_profile_enable(int32_t on);
pct_status pct_profile_read(int64_t *launches, double *ms);

/* Memory-path microbenchmarks: the measured peaks against which the sweeps'
 * achieved rates are reported (the paper's Sec. 4.1 finds the reconstruction
 * bound by its data movement; the last-level cache bandwidth and the atomic
 * rate of the device have no published figure).  Each call runs `reps`
 * launches of one probe on `stream` and returns the mean device time of a
 * launch in *ms_out (HIP events; the call synchronises the stream).
 *   PCT_PROBE_COPY        copies `region` floats (buf[0:region] ->
 *                         buf[region:2 region]); region % 4 == 0.  Bytes
 *                         moved per launch: 8 region.
 *   PCT_PROBE_GATHER      n_ops 4-byte reads of an image of `region` voxels
 *                         (buf[0:region]; one float per thread written
 *                         after it), 64 per wavefront pass along a straight
 *                         line at a hashed angle in a z plane of a 200 x 200
 *                         x (region / 40000) grid numbered in 4 x 4 x 4
 *                         bricks, as the rebuilt-row sweeps read x; region a
 *                         multiple of 160000.
 *   PCT_PROBE_ATOMIC      n_ops FP32 atomic adds of 1.0 along the same runs
 *                         into buf[0:region], as the rebuilt-row sweeps add
 *                         their numerators.
 *   PCT_PROBE_ATOMIC_XCD  the same into one private copy per die
 *                         (buf[8 region]; copy = the die's hardware id), with
 *                         workgroup-scope atomics.
 *   PCT_PROBE_LDS_ATOMIC  n_ops FP32 atomic adds at hashed positions of a
 *                         2048-float image in each workgroup's LDS (region
 *                         unused).
 * buf: device, at least pct_probe_bytes(kind, region, n_ops) bytes, caller
 * owned; the atomic probes add into it (zero it to check the total: each
 * launch adds floor(n_ops / 64) * 64).  n_ops >= 64 * 2048 for every probe
 * but the copy.  Errors: PCT_EINVAL for a bad kind, size or count,
 * PCT_ENOMEM for a short buffer, PCT_EDEVICE for a failed launch. */
typedef enum {
    PCT_PROBE_COPY = 0,
    PCT_PROBE_GATHER = 1,
    PCT_PROBE_ATOMIC = 2,
    PCT_PROBE_ATOMIC_XCD = 3,
    PCT_PROBE_LDS_ATOMIC = 4
} pct_probe_kind;
size_t pct_probe_bytes(int32_t kind, int64_t region, int64_t n_ops);
pct_status pct_probe(int32_t kind, void *buf, size_t buf_bytes, int64_t region, int64_t n_ops, int32_t reps,
                     double *ms_out, void *stream);

/* Message for the last failing call on this thread (empty if none). */
const char *pct_last_error(void);

/* ---- Learned warm start: operations of a small 3D U-Net on the image.
 * A network trained on pairs (image after a few sweeps, image after many
 * sweeps) produced by the solver itself gives the initial guess x0 of the
 * sweeps (the paper leaves x0 to the user, Sec. 2.1); the plain sweeps from
 * the hull start stay the fallback.  Tensors are device float32 [C][D][H][W]
 * (W fastest), caller-owned; outputs must not alias inputs, except that
 * relu, relu_bwd, add and mask may run in place (output == an input).  D*H*W < 2^31.
 * Gradients are written, not accumulated.  Every call is asynchronous on
 * `stream` and returns PCT_EINVAL for NULL pointers or bad sizes. */

/* y[co] = b[co] + sum_ci w[co][ci] (*) x[ci], 3x3x3 kernel, zero padding.
 * w [cout][cin][3][3][3]; b [cout] or NULL. */
pct_status pct_cnn_conv3d(const float *x, const float *w, const float *b, float *y, int32_t cin, int32_t cout,
                          int32_t D, int32_t H, int32_t W, void *stream);
/* input gradient dx [cin] of the convolution from dy [cout]; wt: scratch of
 * cin * cout * 27 floats */
pct_status pct_cnn_conv3d_bwd_data(const float *dy, const float *w, float *dx, float *wt, int32_t cin, int32_t cout,
                                   int32_t D, int32_t H, int32_t W, void *stream);
/* The same two operations on the matrix cores (v_mfma_f32_16x16x32_bf16):
 * inputs and weights rounded to bfloat16 (nearest, ties to even), products
 * accumulated in FP32, the result stored as FP32; for networks whose
 * activations the warm start (Sec. 2.1's x0) may hold at bfloat16 precision.
 * pct_cnn_conv3d_bf16 needs cin % 8 == 0 and cout % 16 == 0, the input
 * gradient cout % 8 == 0 and cin % 16 == 0 (else PCT_EINVAL).  wpack: device
 * scratch of pct_cnn_conv3d_bf16_scratch(cin, cout) bytes (0 for a shape
 * they do not take) for the packed bfloat16 weights; wt as above. */
int64_t pct_cnn_conv3d_bf16_scratch(int32_t cin, int32_t cout);
pct_status pct_cnn_conv3d_bf16(const float *x, const float *w, const float *b, float *y, void *wpack, int32_t cin,
                               int32_t cout, int32_t D, int32_t H, int32_t W, void *stream);
pct_status pct_cnn_conv3d_bwd_data_bf16(const float *dy, const float *w, float *dx, float *wt, void *wpack,
                                        int32_t cin, int32_t cout, int32_t D, int32_t H, int32_t W, void *stream);
/* floats of scratch that pct_cnn_conv3d_bwd_weight and, for the shapes it
 * takes, pct_cnn_conv3d_bwd_weight_bf16 need */
int64_t pct_cnn_wgrad_scratch(int32_t cin, int32_t cout, int32_t D, int32_t H, int32_t W);
/* weight gradient dw [cout][cin][27] and bias gradient db [cout] (or NULL)
 * from the layer input x [cin] and dy [cout]; fixed summation order */
pct_status pct_cnn_conv3d_bwd_weight(const float *x, const float *dy, float *dw, float *db, float *scratch,
                                     int32_t cin, int32_t cout, int32_t D, int32_t H, int32_t W, void *stream);
/* The weight gradient on the matrix cores: x and dy rounded to bfloat16
 * (nearest, ties to even), products accumulated in FP32 in a fixed order;
 * the bias gradient sums dy unrounded.  Needs cin % 16 == 0, cout % 16 == 0
 * and D*H*W < 2^27 (else PCT_EINVAL); scratch as above. */
pct_status pct_cnn_conv3d_bwd_weight_bf16(const float *x, const float *dy, float *dw, float *db, float *scratch,
                                          int32_t cin, int32_t cout, int32_t D, int32_t H, int32_t W,
                                          void *stream);
/* y = max(x, 0); dx = dy where y > 0 (y = the ReLU output) */
pct_status pct_cnn_relu(const float *x, float *y, int64_t n, void *stream);
pct_status pct_cnn_relu_bwd(const float *y, const float *dy, float *dx, int64_t n, void *stream);
/* 2x2x2 average pooling [C][D][H][W] -> [C][D/2][H/2][W/2] (D, H, W even) and
 * its gradient */
pct_status pct_cnn_pool(const float *x, float *y, int32_t C, int32_t D, int32_t H, int32_t W, void *stream);
pct_status pct_cnn_pool_bwd(const float *dy, float *dx, int32_t C, int32_t D, int32_t H, int32_t W, void *stream);
/* nearest 2x upsampling [C][d][h][w] -> [C][2d][2h][2w] and its gradient */
pct_status pct_cnn_upsample(const float *x, float *y, int32_t C, int32_t d, int32_t h, int32_t w, void *stream);
pct_status pct_cnn_upsample_bwd(const float *dy, float *dx, int32_t C, int32_t d, int32_t h, int32_t w,
                                void *stream);
/* y = a + b (elementwise, n values) */
pct_status pct_cnn_add(const float *a, const float *b, float *y, int64_t n, void *stream);
/* y += a * x (n values; x and y must not alias) */
pct_status pct_cnn_axpy(float a, const float *x, float *y, int64_t n, void *stream);
/* y = x inside the mask (mask[i] != 0, uint8 [n]), 0 outside; may run in place */
pct_status pct_cnn_mask(const float *x, const uint8_t *mask, float *y, int64_t n, void *stream);
/* *loss (device double) = mean (y - t)^2 over n values (FP64 sums in fixed
 * order); dy = 2 (y - t) / n when dy != NULL; scratch: pct_cnn_mse_scratch(n)
 * doubles */
int64_t pct_cnn_mse_scratch(int64_t n);
pct_status pct_cnn_mse(const float *y, const float *t, float *dy, double *scratch, double *loss, int64_t n,
                       void *stream);
/* one Adam step (Kingma & Ba 2015, bias-corrected, step >= 1) on n weights */
pct_status pct_cnn_adam(float *w, const float *g, float *m, float *v, int64_t n, float lr, float beta1, float beta2,
                        float eps, int32_t step, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* PCT_H */
