"""Python binding of libpct.so with torch tensors as device memory.

Each function marshals arguments into the C structs of include/pct.h and calls
the entry point of the same name; every step of the reconstruction runs in
the library's HIP kernels.  Torch supplies device allocations and the current
stream only.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import check, pct_geom, pct_grid, pct_histories, pct_plan, pct_rows, pct_sweep_params, pct_tvs

FIELDS = ("phi", "t_in", "v_in", "dt_in", "dv_in", "t_out", "v_out", "dt_out", "dv_out", "wepl")


def make_grid(nx, ny, nz, dx=1.0, dy=1.0, dz=1.0, ox=0.0, oy=0.0, oz=0.0) -> pct_grid:
    return pct_grid(int(nx), int(ny), int(nz), float(dx), float(dy), float(dz), float(ox), float(oy), float(oz))


def make_geom(u_in, u_out, hull_a, hull_b, hull_zmin, hull_zmax, step_mm, poly, highland_log=True, E0_MeV=13.6,
              X0_mm=360.8, path_fp32=False) -> pct_geom:
    g = pct_geom()
    g.u_in, g.u_out = float(u_in), float(u_out)
    g.hull_a, g.hull_b, g.hull_zmin, g.hull_zmax = float(hull_a), float(hull_b), float(hull_zmin), float(hull_zmax)
    g.step_mm = float(step_mm)
    g.highland_log = 1 if highland_log else 0
    g.path_fp32 = 1 if path_fp32 else 0
    poly = [float(c) for c in poly]
    g.n_poly = len(poly)
    for q, c in enumerate(poly[:8]):
        g.poly[q] = c
    g.E0_MeV, g.X0_mm = float(E0_MeV), float(X0_mm)
    return g


def _stream_ptr(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


class Histories:
    """Device SoA of proton histories (float32 tensors of equal length)."""

    def __init__(self, tensors: dict):
        n = None
        self.t = {}
        for k in FIELDS:
            v = tensors[k]
            if not (v.is_cuda and v.dtype == torch.float32 and v.is_contiguous() and v.dim() == 1):
                raise ValueError(f"history field {k} must be a contiguous 1-D float32 device tensor")
            if n is None:
                n = v.numel()
            elif v.numel() != n:
                raise ValueError("history fields differ in length")
            self.t[k] = v
        self.n = int(n or 0)

    @classmethod
    def from_numpy(cls, h: dict, device="cuda"):
        return cls({k: torch.from_numpy(h[k]).to(device=device, dtype=torch.float32).contiguous() for k in FIELDS})

    def struct(self) -> pct_histories:
        s = pct_histories()
        s.n = self.n
        for k in FIELDS:
            setattr(s, k, self.t[k].data_ptr())
        return s

    def permuted(self, order: torch.Tensor) -> "Histories":
        return Histories({k: v.index_select(0, order).contiguous() for k, v in self.t.items()})


@dataclass
class Rows:
    """Cached rows of A (CSR, device)."""
    row_ptr: torch.Tensor
    idx: torch.Tensor | None
    len: torch.Tensor | None
    norm2: torch.Tensor | None
    len_dtype: int
    nnz: int = 0

    @property
    def n_rows(self) -> int:
        return self.row_ptr.numel() - 1

    def struct(self) -> pct_rows:
        r = pct_rows()
        r.n_rows = self.n_rows
        r.cap_nnz = 0 if self.idx is None else self.idx.numel()
        r.nnz = self.nnz
        r.row_ptr = self.row_ptr.data_ptr()
        r.idx = _ptr(self.idx)
        r.len = _ptr(self.len)
        r.len_dtype = self.len_dtype
        r.norm2 = _ptr(self.norm2)
        return r


class Tvs:
    """pct_tvs (total-variation superiorization, Sec. 4.2) with its device
    state (state[0] = the current step size, shrunk by the library)."""

    def __init__(self, beta0: float = 2.0, n_steps: int = 1, max_trials: int = 3, a: float = 0.995,
                 eps: float = 1e-3, device=None):
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.state = torch.zeros(8, dtype=torch.float64, device=dev)
        self.state[0] = float(beta0)
        self.struct = pct_tvs(int(n_steps), int(max_trials), float(a), float(eps), self.state.data_ptr())

    @property
    def beta(self) -> float:
        return float(self.state[0].item())

    @property
    def accepted(self) -> int:
        return int(self.state[5].item())


class SweepParams:
    """pct_sweep_params plus references to the device tensors it points to
    (so they stay allocated while the struct is in use)."""

    def __init__(self, algo="drop", block_size=200_000, lam=0.5, n_sweeps=1, order=None, hull_mask=None,
                 tvs: Tvs | None = None):
        for name, t, dt in (("order", order, torch.int64), ("hull_mask", hull_mask, torch.uint8)):
            if t is not None and not (t.is_cuda and t.dtype == dt and t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous {dt} device tensor")
        self.order = order
        self.hull_mask = hull_mask
        s = pct_sweep_params()
        s.algo = {"art": 0, "drop": 1}[algo] if isinstance(algo, str) else int(algo)
        s.block_size = int(block_size)
        s.lambda_ = float(lam)
        s.n_sweeps = int(n_sweeps)
        s.order = _ptr(order)
        s.hull_mask = _ptr(hull_mask)
        self.tvs = tvs
        if tvs is not None:
            s.tvs = ctypes.pointer(tvs.struct)
        self.struct = s

    @property
    def n_sweeps(self) -> int:
        return int(self.struct.n_sweeps)


def sweep_params(algo="drop", block_size=200_000, lam=0.5, n_sweeps=1, order=None, hull_mask=None,
                 tvs: Tvs | None = None) -> SweepParams:
    return SweepParams(algo, block_size, lam, n_sweeps, order, hull_mask, tvs)


_ws_cache: dict = {}


def workspace(grid: pct_grid, n_hist: int, device=None, params: "SweepParams | None" = None,
              geom: pct_geom | None = None, fused: bool = False) -> torch.Tensor:
    """Device scratch of pct_workspace_size bytes, cached per device and grown
    on demand (geom given: includes the trace's row staging area; fused with
    params of several DROP sweeps: includes the kept per-block counts)."""
    lib = _lib.load()
    nbytes = lib.pct_workspace_size(ctypes.byref(grid), ctypes.byref(geom) if geom is not None else None,
                                    ctypes.byref(params.struct) if params else None, int(n_hist), 1 if fused else 0)
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    ws = _ws_cache.get(dev)
    if ws is None or ws.numel() < nbytes:
        _ws_cache.pop(dev, None)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        _ws_cache[dev] = ws
    return ws


def mlp_trace(grid: pct_grid, geom: pct_geom, hist: Histories, len_dtype: int = 0, rows: Rows | None = None,
              stream=None, allow_nonfinite: bool = False) -> Rows:
    """pct_mlp_trace: sizing call, allocation, fill call."""
    lib = _lib.load()
    dev = hist.t["phi"].device
    ws = workspace(grid, hist.n, dev, geom=geom)
    allow = (_lib.PCT_OK, _lib.PCT_ENONFINITE) if allow_nonfinite else (_lib.PCT_OK,)
    if rows is None:
        rows = Rows(torch.empty(hist.n + 1, dtype=torch.int64, device=dev), None, None, None, len_dtype)
        rs = rows.struct()
        hs = hist.struct()
        check(lib.pct_mlp_trace(ctypes.byref(grid), ctypes.byref(geom), ctypes.byref(hs), ctypes.byref(rs),
                                ws.data_ptr(), ws.numel(), _stream_ptr(stream)), allow)
        nnz = int(rs.nnz)
        rows.idx = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
        rows.len = torch.empty(max(nnz, 1), dtype=torch.float32 if len_dtype == 0 else torch.float16, device=dev)
        rows.norm2 = torch.empty(max(hist.n, 1), dtype=torch.float64, device=dev)
    rs = rows.struct()
    hs = hist.struct()
    check(lib.pct_mlp_trace(ctypes.byref(grid), ctypes.byref(geom), ctypes.byref(hs), ctypes.byref(rs),
                            ws.data_ptr(), ws.numel(), _stream_ptr(stream)), allow)
    rows.nnz = int(rs.nnz)
    return rows


def _check_lengths(grid, hist: Histories, x: torch.Tensor, params: SweepParams):
    M = grid.nx * grid.ny * grid.nz
    if not (x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and x.numel() == M):
        raise ValueError(f"x must be a contiguous float32 device tensor of {M} voxels")
    if params.order is not None and params.order.numel() != hist.n:
        raise ValueError("order must hold one entry per history")
    if params.hull_mask is not None and params.hull_mask.numel() != M:
        raise ValueError("hull_mask must hold one entry per voxel")


def project_sweep(grid, geom, hist: Histories, rows: Rows | None, x: torch.Tensor, params: SweepParams,
                  resid_out: torch.Tensor | None = None, stream=None):
    lib = _lib.load()
    _check_lengths(grid, hist, x, params)
    ws = workspace(grid, hist.n, x.device, fused=rows is None)
    hs = hist.struct()
    rs = rows.struct() if rows is not None else None
    check(lib.pct_project_sweep(ctypes.byref(grid), ctypes.byref(geom), ctypes.byref(hs),
                                ctypes.byref(rs) if rs is not None else None, x.data_ptr(), ctypes.byref(params.struct),
                                _ptr(resid_out), ws.data_ptr(), ws.numel(), _stream_ptr(stream)))


class Plan:
    """A sweep plan (pct_plan) with its device memory."""

    def __init__(self):
        self.struct = pct_plan()
        self.mem = None

    @property
    def ready(self) -> bool:
        return bool(self.struct.ready)


def plan_build(grid, hist: Histories, rows: Rows, params: SweepParams, plan: Plan | None = None,
               stream=None) -> Plan:
    """pct_plan_build: sizing call, allocation (if needed), build."""
    lib = _lib.load()
    dev = hist.t["phi"].device
    ws = workspace(grid, hist.n, dev, params)
    hs = hist.struct()
    rs = rows.struct()
    plan = plan or Plan()
    if plan.mem is None:
        plan.struct.mem = None
        check(lib.pct_plan_build(ctypes.byref(grid), ctypes.byref(hs), ctypes.byref(rs), ctypes.byref(params.struct),
                                 ctypes.byref(plan.struct), ws.data_ptr(), ws.numel(), _stream_ptr(stream)))
        plan.mem = torch.empty(int(plan.struct.bytes), dtype=torch.uint8, device=dev)
        plan.struct.mem = plan.mem.data_ptr()
        plan.struct.bytes = plan.mem.numel()
    check(lib.pct_plan_build(ctypes.byref(grid), ctypes.byref(hs), ctypes.byref(rs), ctypes.byref(params.struct),
                             ctypes.byref(plan.struct), ws.data_ptr(), ws.numel(), _stream_ptr(stream)))
    plan.struct.mem = plan.mem.data_ptr()
    plan.struct.bytes = plan.mem.numel()
    plan.params = params
    return plan


def plan_sweep(grid, plan: Plan, x: torch.Tensor, params: SweepParams, resid_out: torch.Tensor | None = None,
               stream=None):
    lib = _lib.load()
    ws = workspace(grid, int(plan.struct.n), x.device)
    check(lib.pct_plan_sweep(ctypes.byref(grid), ctypes.byref(plan.struct), x.data_ptr(), ctypes.byref(params.struct),
                             _ptr(resid_out), ws.data_ptr(), ws.numel(), _stream_ptr(stream)))


def plan_residual(grid, plan: Plan, x: torch.Tensor, stream=None) -> float:
    lib = _lib.load()
    ws = workspace(grid, int(plan.struct.n), x.device)
    out = torch.empty(1, dtype=torch.float64, device=x.device)
    check(lib.pct_plan_residual(ctypes.byref(grid), ctypes.byref(plan.struct), x.data_ptr(), out.data_ptr(),
                                ws.data_ptr(), ws.numel(), _stream_ptr(stream)))
    return float(out.item())


def reconstruct(grid, geom, hist: Histories, params: SweepParams, x: torch.Tensor, rows: Rows | None = None,
                plan: Plan | None = None, want_residuals: bool = True, stream=None, allow_nonfinite: bool = False):
    """pct_reconstruct: x is updated in place; returns the residual per sweep (host list).
    With a plan, its memory must already be allocated (plan_build sizes it)."""
    lib = _lib.load()
    _check_lengths(grid, hist, x, params)
    ws = workspace(grid, hist.n, x.device, params, geom=geom if rows is not None else None, fused=rows is None)
    hs = hist.struct()
    rs = rows.struct() if rows is not None else None
    res = (ctypes.c_double * max(params.n_sweeps, 1))()
    allow = (_lib.PCT_OK, _lib.PCT_ENONFINITE) if allow_nonfinite else (_lib.PCT_OK,)
    check(lib.pct_reconstruct(ctypes.byref(grid), ctypes.byref(geom), ctypes.byref(hs), ctypes.byref(params.struct),
                              ctypes.byref(rs) if rs is not None else None,
                              ctypes.byref(plan.struct) if plan is not None else None, x.data_ptr(),
                              res if want_residuals else None, ws.data_ptr(), ws.numel(), _stream_ptr(stream)),
          allow)
    if rows is not None:
        rows.nnz = int(rs.nnz)
    if plan is not None:
        plan.struct.mem = plan.mem.data_ptr()
        plan.struct.bytes = plan.mem.numel()
    return [res[k] for k in range(params.n_sweeps)] if want_residuals else []


def residual(grid, geom, hist: Histories, rows: Rows | None, x: torch.Tensor, stream=None) -> float:
    lib = _lib.load()
    ws = workspace(grid, hist.n, x.device, fused=rows is None)
    out = torch.empty(1, dtype=torch.float64, device=x.device)
    hs = hist.struct()
    rs = rows.struct() if rows is not None else None
    check(lib.pct_residual(ctypes.byref(grid), ctypes.byref(geom), ctypes.byref(hs),
                           ctypes.byref(rs) if rs is not None else None, x.data_ptr(), out.data_ptr(),
                           ws.data_ptr(), ws.numel(), _stream_ptr(stream)))
    return float(out.item())


def tvs_apply(grid, x: torch.Tensor, tvs: Tvs, hull_mask: torch.Tensor | None = None, stream=None):
    """pct_tvs_apply: the TV superiorization steps on x, in place."""
    lib = _lib.load()
    ws = workspace(grid, 0, x.device, SweepParams(tvs=tvs))
    check(lib.pct_tvs_apply(ctypes.byref(grid), x.data_ptr(), _ptr(hull_mask), ctypes.byref(tvs.struct),
                            ws.data_ptr(), ws.numel(), _stream_ptr(stream)))


def carp(grid, geom, hist: Histories, params: SweepParams, n_strings: int, x: torch.Tensor, rows: Rows | None = None,
         want_residuals: bool = True, stream=None):
    """pct_carp (Sec. 2.2): params.n_sweeps iterations of n_strings strings;
    x updated in place; returns the residual per iteration."""
    lib = _lib.load()
    _check_lengths(grid, hist, x, params)
    fused = rows is None
    nbytes = lib.pct_carp_workspace_size(ctypes.byref(grid), ctypes.byref(geom) if not fused else None,
                                         ctypes.byref(params.struct), hist.n, 1 if fused else 0)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    hs = hist.struct()
    rs = rows.struct() if rows is not None else None
    res = (ctypes.c_double * max(params.n_sweeps, 1))()
    check(lib.pct_carp(ctypes.byref(grid), ctypes.byref(geom), ctypes.byref(hs), ctypes.byref(params.struct),
                       int(n_strings), ctypes.byref(rs) if rs is not None else None, x.data_ptr(),
                       res if want_residuals else None, ws.data_ptr(), ws.numel(), _stream_ptr(stream)))
    return [res[k] for k in range(params.n_sweeps)] if want_residuals else []


def carve_hull(grid, geom, hist: Histories, wepl_max: float = 1.5, min_len: float = 1e-6, stream=None):
    """pct_carve_hull: (hull mask uint8 [M] on the device, histories used)."""
    lib = _lib.load()
    dev = hist.t["phi"].device
    M = grid.nx * grid.ny * grid.nz
    out = torch.empty(M, dtype=torch.uint8, device=dev)
    ws = workspace(grid, 0, dev)
    used = ctypes.c_int64(0)
    hs = hist.struct()
    check(lib.pct_carve_hull(ctypes.byref(grid), ctypes.byref(geom), ctypes.byref(hs), float(wepl_max),
                             float(min_len), out.data_ptr(), ctypes.byref(used), ws.data_ptr(), ws.numel(),
                             _stream_ptr(stream)))
    return out, int(used.value)


def roi_stats(x: torch.Tensor, labels: torch.Tensor, n_labels: int, stream=None):
    lib = _lib.load()
    sums = torch.empty(n_labels, dtype=torch.float64, device=x.device)
    counts = torch.empty(n_labels, dtype=torch.int64, device=x.device)
    check(lib.pct_roi_stats(x.data_ptr(), labels.data_ptr(), x.numel(), int(n_labels), sums.data_ptr(),
                            counts.data_ptr(), _stream_ptr(stream)))
    return sums, counts


def profile_enable(on: bool = True) -> None:
    check(_lib.load().pct_profile_enable(1 if on else 0))


def profile_read() -> dict:
    """{kernel class: (launches, total ms)} recorded since profile_enable(True)."""
    n = len(_lib.KERNEL_CLASSES)
    launches = (ctypes.c_int64 * n)()
    ms = (ctypes.c_double * n)()
    check(_lib.load().pct_profile_read(launches, ms))
    return {k: (int(launches[i]), float(ms[i])) for i, k in enumerate(_lib.KERNEL_CLASSES)}


def probe(kind: str, region: int, n_ops: int = 0, reps: int = 5, buf: torch.Tensor | None = None,
          stream=None) -> tuple[float, torch.Tensor]:
    """Mean device time (ms) of one launch of memory-path probe `kind` (one of
    _lib.PROBE_KINDS; see pct_probe in include/pct.h) and the buffer it ran
    on (zeroed first, so an atomic probe's buffer sums to reps x the adds of
    a launch)."""
    lib = _lib.load()
    k = _lib.PROBE_KINDS[kind]
    need = int(lib.pct_probe_bytes(k, region, n_ops))
    if buf is None:
        buf = torch.zeros((need + 3) // 4, dtype=torch.float32, device="cuda")
    else:
        buf.zero_()
    ms = ctypes.c_double(0.0)
    _lib.check(lib.pct_probe(k, _ptr(buf), buf.numel() * buf.element_size(), region, n_ops, reps,
                             ctypes.byref(ms), _stream_ptr(stream)))
    return ms.value, buf
