"""FP64 CPU oracle of event-by-event pCT reconstruction.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline may use this package; the product path (the HIP library and its
binding) never imports, loads or calls it, and shares no code with it.

The arithmetic lives in ``oracle.c`` (plain FP64 C):
  * ``mlp_path``     -- most-likely path polyline of one history (Sec. 2; the
                        Bayesian path formalism the paper cites, Schulte 2008);
  * ``polyline_row`` -- Siddon voxel traversal of a polyline, fully merged;
  * ``trace``        -- the rows of A for a set of histories (Sec. 2: one row
                        per proton, path lengths in the voxels it touches);
  * ``drop``         -- block-iterative row projections (DROP, Sec. 2.1), ART
                        as block size 1;
  * ``drop_recompute`` -- the same DROP with no stored A: each block's rows are
                        traced, projected and dropped (A too large to keep,
                        Sec. 2 and Sec. 4.1);
  * ``residual``     -- ||Ax - b||_2;
  * ``tv``, ``tv_grad``, ``tvs_apply`` -- total variation and the TV
                        superiorization step (Sec. 4.2); ``drop_tvs`` -- DROP
                        with it before every block;
  * ``carp``         -- component-averaged row projections (Sec. 2.2);
  * ``carve``        -- the space-carving hull from protons that crossed
                        only air.
``roi_means`` is the ROI analysis of Sec. 3.2 / 4.2 (mean RSP per insert).
``oracle.cnn`` (NumPy, FP64) holds the operations and gradients of the
warm-start network that produces x0 (Sec. 2.1 leaves x0 open).

Parity pins: see tests/test_oracle_*.py.  The full reconstructed image has no
closed form; it is pinned only piecewise (path, traversal, solver), so the
image itself is "parity unpinned" beyond those pins.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
FIELDS = ("phi", "t_in", "v_in", "dt_in", "dv_in", "t_out", "v_out", "dt_out", "dv_out", "wepl")


def build(force: bool = True) -> str:
    if force or not os.path.exists(_SO):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _SO + ".tmp",
                               os.path.join(_HERE, "oracle.c"), "-lm"])
        os.replace(_SO + ".tmp", _SO)
    return _SO


class OrcGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("ox", ctypes.c_double), ("oy", ctypes.c_double), ("oz", ctypes.c_double)]


class OrcGeom(ctypes.Structure):
    _fields_ = [("u_in", ctypes.c_double), ("u_out", ctypes.c_double), ("hull_a", ctypes.c_double),
                ("hull_b", ctypes.c_double), ("hull_zmin", ctypes.c_double), ("hull_zmax", ctypes.c_double),
                ("step", ctypes.c_double), ("highland_log", ctypes.c_int32), ("n_poly", ctypes.c_int32),
                ("poly", ctypes.c_double * 8), ("E0", ctypes.c_double), ("X0", ctypes.c_double)]


class OrcTvs(ctypes.Structure):
    _fields_ = [("n_steps", ctypes.c_int32), ("max_trials", ctypes.c_int32), ("a", ctypes.c_double),
                ("eps", ctypes.c_double)]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        lib.orc_mlp_path.restype = ctypes.c_int
        lib.orc_mlp_path.argtypes = [ctypes.POINTER(OrcGeom), _dp, ctypes.c_int, _dp, _dp, _dp]
        lib.orc_polyline_row.restype = ctypes.c_int64
        lib.orc_polyline_row.argtypes = [ctypes.POINTER(OrcGrid), ctypes.c_int32, _dp, _i32p, _dp, ctypes.c_int64,
                                         _dp]
        lib.orc_trace.restype = ctypes.c_int64
        lib.orc_trace.argtypes = [ctypes.POINTER(OrcGrid), ctypes.POINTER(OrcGeom), ctypes.c_int64,
                                  ctypes.POINTER(ctypes.POINTER(ctypes.c_float)), _i64p, _i32p, _dp, _dp,
                                  ctypes.c_int32]
        lib.orc_residual.restype = ctypes.c_double
        lib.orc_residual.argtypes = [ctypes.c_int64, _i64p, _i32p, _dp, _dp, _dp]
        lib.orc_drop.restype = ctypes.c_int
        lib.orc_drop.argtypes = [ctypes.c_int64, _i64p, _i32p, _dp, _dp, _dp, _i64p, ctypes.c_int64,
                                 ctypes.c_double, ctypes.POINTER(ctypes.c_uint8), ctypes.c_int64, ctypes.c_int32,
                                 _dp, _dp, ctypes.c_int32]
        lib.orc_drop_recompute.restype = ctypes.c_int
        lib.orc_drop_recompute.argtypes = [ctypes.POINTER(OrcGrid), ctypes.POINTER(OrcGeom), ctypes.c_int64,
                                           ctypes.POINTER(ctypes.POINTER(ctypes.c_float)), _i64p, ctypes.c_int64,
                                           ctypes.c_double, ctypes.POINTER(ctypes.c_uint8), ctypes.c_int64,
                                           ctypes.c_int32, _dp, _dp, ctypes.c_int32]
        lib.orc_tv.restype = ctypes.c_double
        lib.orc_tv.argtypes = [ctypes.POINTER(OrcGrid), _dp, ctypes.c_double]
        lib.orc_tv_grad.restype = None
        lib.orc_tv_grad.argtypes = [ctypes.POINTER(OrcGrid), _dp, ctypes.c_double, _dp]
        lib.orc_tvs_apply.restype = ctypes.c_int
        lib.orc_tvs_apply.argtypes = [ctypes.POINTER(OrcGrid), ctypes.POINTER(OrcTvs), ctypes.POINTER(ctypes.c_uint8),
                                      _dp, _dp]
        lib.orc_drop_tvs.restype = ctypes.c_int
        lib.orc_drop_tvs.argtypes = [ctypes.POINTER(OrcGrid), ctypes.c_int64, _i64p, _i32p, _dp, _dp, _dp, _i64p,
                                     ctypes.c_int64, ctypes.c_double, ctypes.POINTER(ctypes.c_uint8), ctypes.c_int32,
                                     ctypes.POINTER(OrcTvs), _dp, _dp, _dp, ctypes.c_int32]
        lib.orc_carp.restype = ctypes.c_int
        lib.orc_carp.argtypes = [ctypes.POINTER(OrcGrid), ctypes.c_int64, _i64p, _i32p, _dp, _dp, _dp, _i64p,
                                 ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.POINTER(ctypes.c_uint8),
                                 ctypes.c_int32, ctypes.POINTER(OrcTvs), _dp, _dp, _dp, ctypes.c_int32]
        lib.orc_carve.restype = ctypes.c_int64
        lib.orc_carve.argtypes = [ctypes.POINTER(OrcGrid), ctypes.POINTER(OrcGeom), ctypes.c_int64,
                                  ctypes.POINTER(ctypes.POINTER(ctypes.c_float)), ctypes.c_double, ctypes.c_double,
                                  ctypes.POINTER(ctypes.c_uint8), ctypes.c_int32]
        _lib = lib
    return _lib


def _threads(t):
    """Threads for the OpenMP loops: the caller's count, else every core this
    process may run on, limited by OMP_NUM_THREADS when that is set (a host
    that shares its cores among several jobs sets it to this job's share)."""
    if t:
        return t
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def make_grid(nx, ny, nz, dx, dy, dz, ox, oy, oz) -> OrcGrid:
    return OrcGrid(nx, ny, nz, dx, dy, dz, ox, oy, oz)


def make_geom(u_in, u_out, hull_a, hull_b, hull_zmin, hull_zmax, step, poly, highland_log=True,
              E0=13.6, X0=360.8) -> OrcGeom:
    g = OrcGeom()
    g.u_in, g.u_out = u_in, u_out
    g.hull_a, g.hull_b, g.hull_zmin, g.hull_zmax = hull_a, hull_b, hull_zmin, hull_zmax
    g.step = step
    g.highland_log = 1 if highland_log else 0
    poly = list(poly)
    if len(poly) > 8:
        raise ValueError("at most 8 prior coefficients")
    g.n_poly = len(poly)
    for q, c in enumerate(poly):
        g.poly[q] = float(c)
    g.E0, g.X0 = E0, X0
    return g


def mlp_path(geom: OrcGeom, hist_row) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(u, t, v) samples of the most-likely path of one history (10 values)."""
    lib = _load()
    h = np.ascontiguousarray(np.asarray(hist_row, dtype=np.float64))
    cap = 4096
    while True:
        u = np.empty(cap)
        t = np.empty(cap)
        v = np.empty(cap)
        n = lib.orc_mlp_path(ctypes.byref(geom), h.ctypes.data_as(_dp), cap, u.ctypes.data_as(_dp),
                             t.ctypes.data_as(_dp), v.ctypes.data_as(_dp))
        if n >= 0:
            return u[:n], t[:n], v[:n]
        cap = -n


def polyline_row(grid: OrcGrid, xyz) -> tuple[np.ndarray, np.ndarray, float]:
    """(idx ascending, lengths, ||a||^2) of a polyline given in the object frame."""
    lib = _load()
    P = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1, 3))
    cnt = lib.orc_polyline_row(ctypes.byref(grid), P.shape[0], P.ctypes.data_as(_dp), None, None, 0, None)
    idx = np.empty(max(cnt, 1), dtype=np.int32)
    ln = np.empty(max(cnt, 1))
    n2 = ctypes.c_double()
    lib.orc_polyline_row(ctypes.byref(grid), P.shape[0], P.ctypes.data_as(_dp), idx.ctypes.data_as(_i32p),
                         ln.ctypes.data_as(_dp), cnt, ctypes.byref(n2))
    return idx[:cnt], ln[:cnt], n2.value


class Rows:
    """CSR rows of A in FP64: row_ptr [n+1], idx [nnz] ascending per row, len [nnz], norm2 [n]."""

    def __init__(self, row_ptr, idx, length, norm2):
        self.row_ptr, self.idx, self.len, self.norm2 = row_ptr, idx, length, norm2

    @property
    def n(self):
        return len(self.row_ptr) - 1

    def row(self, i):
        a, b = self.row_ptr[i], self.row_ptr[i + 1]
        return self.idx[a:b], self.len[a:b]


def _hist_ptrs(hist: dict):
    arrs = [np.ascontiguousarray(hist[k], dtype=np.float32) for k in FIELDS]
    fp = ctypes.POINTER(ctypes.c_float)
    arr_t = fp * len(FIELDS)
    return arrs, arr_t(*[a.ctypes.data_as(fp) for a in arrs])


def trace(grid: OrcGrid, geom: OrcGeom, hist: dict, threads: int | None = None) -> Rows:
    lib = _load()
    arrs, ptrs = _hist_ptrs(hist)
    n = len(arrs[0])
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    nnz = lib.orc_trace(ctypes.byref(grid), ctypes.byref(geom), n, ptrs, row_ptr.ctypes.data_as(_i64p), None, None,
                        None, _threads(threads))
    idx = np.empty(max(nnz, 1), dtype=np.int32)
    ln = np.empty(max(nnz, 1))
    n2 = np.empty(n)
    lib.orc_trace(ctypes.byref(grid), ctypes.byref(geom), n, ptrs, row_ptr.ctypes.data_as(_i64p),
                  idx.ctypes.data_as(_i32p), ln.ctypes.data_as(_dp), n2.ctypes.data_as(_dp), _threads(threads))
    return Rows(row_ptr, idx[:nnz], ln[:nnz], n2)


def residual(rows: Rows, b, x) -> float:
    lib = _load()
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib.orc_residual(rows.n, rows.row_ptr.ctypes.data_as(_i64p), rows.idx.ctypes.data_as(_i32p),
                            rows.len.ctypes.data_as(_dp), b.ctypes.data_as(_dp), x.ctypes.data_as(_dp))


def drop(rows: Rows, b, x0, order, block: int, lam: float, sweeps: int, mask=None,
         threads: int | None = None) -> tuple[np.ndarray, np.ndarray]:
    """Block-iterative projections (block = 1 is ART).  Returns (x, residual per sweep)."""
    lib = _load()
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    order = np.ascontiguousarray(order, dtype=np.int64)
    if len(order) != rows.n:
        raise ValueError("order must be a permutation of all rows")
    res = np.empty(max(sweeps, 1))
    mptr = None
    if mask is not None:
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        mptr = mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    rc = lib.orc_drop(rows.n, rows.row_ptr.ctypes.data_as(_i64p), rows.idx.ctypes.data_as(_i32p),
                      rows.len.ctypes.data_as(_dp), rows.norm2.ctypes.data_as(_dp), b.ctypes.data_as(_dp),
                      order.ctypes.data_as(_i64p), block, lam, mptr, len(x), sweeps, x.ctypes.data_as(_dp),
                      res.ctypes.data_as(_dp), _threads(threads))
    if rc != 0:
        raise ValueError("bad block size")
    return x, res[:sweeps]


def drop_recompute(grid: OrcGrid, geom: OrcGeom, hist: dict, x0, order, block: int, lam: float, sweeps: int,
                   mask=None, threads: int | None = None) -> tuple[np.ndarray, np.ndarray]:
    """DROP with no stored rows: each block's rows are traced just before the
    block is projected and then dropped (the case of A too large to keep,
    Sec. 2 and Sec. 4.1); the residual after each sweep traces every row
    again.  Same rows and summation order as ``drop(trace(...), ...)``.
    Returns (x, residual per sweep)."""
    lib = _load()
    arrs, ptrs = _hist_ptrs(hist)
    n = len(arrs[0])
    x = np.array(x0, dtype=np.float64, copy=True)
    order = np.ascontiguousarray(order, dtype=np.int64)
    if len(order) != n:
        raise ValueError("order must be a permutation of all histories")
    res = np.empty(max(sweeps, 1))
    mptr = None
    if mask is not None:
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        mptr = mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    rc = lib.orc_drop_recompute(ctypes.byref(grid), ctypes.byref(geom), n, ptrs, order.ctypes.data_as(_i64p), block,
                                lam, mptr, len(x), sweeps, x.ctypes.data_as(_dp), res.ctypes.data_as(_dp),
                                _threads(threads))
    if rc != 0:
        raise ValueError("bad block size")
    return x, res[:sweeps]


def _u8p(mask):
    if mask is None:
        return None, None
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    return m, m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def tv(grid: OrcGrid, x, eps: float) -> float:
    """Total variation (forward differences, smoothed by eps) of an image."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    return _load().orc_tv(ctypes.byref(grid), x.ctypes.data_as(_dp), eps)


def tv_grad(grid: OrcGrid, x, eps: float) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    g = np.empty_like(x)
    _load().orc_tv_grad(ctypes.byref(grid), x.ctypes.data_as(_dp), eps, g.ctypes.data_as(_dp))
    return g


def make_tvs(n_steps: int = 1, max_trials: int = 3, a: float = 0.995, eps: float = 1e-3) -> OrcTvs:
    return OrcTvs(int(n_steps), int(max_trials), float(a), float(eps))


def tvs_apply(grid: OrcGrid, x, tvs: OrcTvs, beta: float, mask=None) -> tuple[np.ndarray, float, int]:
    """TVS steps (Sec. 4.2) on a copy of x; returns (x, beta after, accepted steps)."""
    x = np.array(x, dtype=np.float64, copy=True)
    b = ctypes.c_double(beta)
    m, mp = _u8p(mask)
    acc = _load().orc_tvs_apply(ctypes.byref(grid), ctypes.byref(tvs), mp, x.ctypes.data_as(_dp), ctypes.byref(b))
    return x, b.value, acc


def drop_tvs(grid: OrcGrid, rows: Rows, b, x0, order, block: int, lam: float, sweeps: int, tvs: OrcTvs,
             beta: float, mask=None, threads: int | None = None) -> tuple[np.ndarray, np.ndarray, float]:
    """DROP with TVS steps on the image entering every block.  Returns (x,
    residual per sweep, beta after)."""
    lib = _load()
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    order = np.ascontiguousarray(order, dtype=np.int64)
    res = np.empty(max(sweeps, 1))
    bt = ctypes.c_double(beta)
    m, mp = _u8p(mask)
    rc = lib.orc_drop_tvs(ctypes.byref(grid), rows.n, rows.row_ptr.ctypes.data_as(_i64p),
                          rows.idx.ctypes.data_as(_i32p), rows.len.ctypes.data_as(_dp),
                          rows.norm2.ctypes.data_as(_dp), b.ctypes.data_as(_dp), order.ctypes.data_as(_i64p), block,
                          lam, mp, sweeps, ctypes.byref(tvs), ctypes.byref(bt), x.ctypes.data_as(_dp),
                          res.ctypes.data_as(_dp), _threads(threads))
    if rc != 0:
        raise ValueError("bad arguments")
    return x, res[:sweeps], bt.value


def carp(grid: OrcGrid, rows: Rows, b, x0, order, n_strings: int, block: int, lam: float, iters: int,
         mask=None, tvs: OrcTvs | None = None, beta: float = 0.0,
         threads: int | None = None) -> tuple[np.ndarray, np.ndarray, float]:
    """CARP (Sec. 2.2): strings of consecutive order positions, each a DROP
    sweep from the common x, then component averaging over the strings that
    touch each voxel.  Returns (x, residual per iteration, beta after)."""
    lib = _load()
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    order = np.ascontiguousarray(order, dtype=np.int64)
    res = np.empty(max(iters, 1))
    bt = ctypes.c_double(beta)
    m, mp = _u8p(mask)
    rc = lib.orc_carp(ctypes.byref(grid), rows.n, rows.row_ptr.ctypes.data_as(_i64p), rows.idx.ctypes.data_as(_i32p),
                      rows.len.ctypes.data_as(_dp), rows.norm2.ctypes.data_as(_dp), b.ctypes.data_as(_dp),
                      order.ctypes.data_as(_i64p), n_strings, block, lam, mp, iters,
                      ctypes.byref(tvs) if tvs is not None else None, ctypes.byref(bt), x.ctypes.data_as(_dp),
                      res.ctypes.data_as(_dp), _threads(threads))
    if rc != 0:
        raise ValueError("bad arguments")
    return x, res[:iters], bt.value


def carve(grid: OrcGrid, geom: OrcGeom, hist: dict, wepl_max: float, min_len: float = 1e-6,
          threads: int | None = None) -> tuple[np.ndarray, int]:
    """Space-carving hull: (carved mask uint8 [M], histories used).  Voxels
    that the straight line of a history with WEPL below wepl_max crosses for
    more than min_len mm are carved (outside the object)."""
    lib = _load()
    arrs, ptrs = _hist_ptrs(hist)
    M = grid.nx * grid.ny * grid.nz
    out = np.zeros(M, dtype=np.uint8)
    used = lib.orc_carve(ctypes.byref(grid), ctypes.byref(geom), len(arrs[0]), ptrs, wepl_max, min_len,
                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), _threads(threads))
    return out, int(used)


def roi_means(x, labels, n_labels: int) -> np.ndarray:
    """Mean of x over each label 1..n_labels (ROI analysis)."""
    x = np.asarray(x, dtype=np.float64)
    sums = np.bincount(labels, weights=x, minlength=n_labels + 1)[1:n_labels + 1]
    cnts = np.bincount(labels, minlength=n_labels + 1)[1:n_labels + 1]
    return sums / np.maximum(cnts, 1)


def rsp_error(x, labels, true_rsp) -> float:
    """max_k |ROI mean_k - true_k| / true_k."""
    m = roi_means(x, labels, len(true_rsp))
    return float(np.max(np.abs(m - true_rsp) / true_rsp))
