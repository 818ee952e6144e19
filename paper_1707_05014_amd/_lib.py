"""ctypes mirror of include/pct.h and the loader of libpct.so.

Argument marshalling only: every step of the reconstruction runs in the HIP
kernels of libpct.so.  If the library is missing this module raises; there
is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpct.so")

PCT_OK = 0
PCT_EINVAL = -1
PCT_ENOMEM = -2
PCT_EDEVICE = -3
PCT_EROWCAP = -4
PCT_ENONFINITE = -5
PROBE_KINDS = {"copy": 0, "gather": 1, "atomic": 2, "atomic_xcd": 3, "lds_atomic": 4}
STATUS_NAMES = {0: "PCT_OK", -1: "PCT_EINVAL", -2: "PCT_ENOMEM", -3: "PCT_EDEVICE", -4: "PCT_EROWCAP",
                -5: "PCT_ENONFINITE"}


class pct_grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_float), ("dy", ctypes.c_float), ("dz", ctypes.c_float),
                ("ox", ctypes.c_float), ("oy", ctypes.c_float), ("oz", ctypes.c_float)]


class pct_geom(ctypes.Structure):
    _fields_ = [("u_in", ctypes.c_float), ("u_out", ctypes.c_float),
                ("hull_a", ctypes.c_float), ("hull_b", ctypes.c_float),
                ("hull_zmin", ctypes.c_float), ("hull_zmax", ctypes.c_float),
                ("step_mm", ctypes.c_float), ("highland_log", ctypes.c_int32),
                ("n_poly", ctypes.c_int32), ("path_fp32", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("poly", ctypes.c_double * 8),
                ("E0_MeV", ctypes.c_double), ("X0_mm", ctypes.c_double)]


_fp = ctypes.c_void_p


class pct_histories(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("phi", _fp), ("t_in", _fp), ("v_in", _fp), ("dt_in", _fp),
                ("dv_in", _fp), ("t_out", _fp), ("v_out", _fp), ("dt_out", _fp), ("dv_out", _fp),
                ("wepl", _fp)]


class pct_rows(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("cap_nnz", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", _fp), ("idx", _fp), ("len", _fp), ("len_dtype", ctypes.c_int32),
                ("norm2", _fp)]


class pct_plan(ctypes.Structure):
    _fields_ = [("mem", _fp), ("bytes", ctypes.c_size_t), ("n", ctypes.c_int64), ("block_size", ctypes.c_int64),
                ("n_blocks", ctypes.c_int64), ("n_tiles", ctypes.c_int64), ("entries", ctypes.c_int64),
                ("chunks", ctypes.c_int64), ("refs", ctypes.c_int64), ("max_chunks", ctypes.c_int64),
                ("max_ends", ctypes.c_int64), ("ends", ctypes.c_int64),
                ("len_dtype", ctypes.c_int32),
                ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("order", _fp), ("rows_idx", _fp),
                ("ready", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class pct_tvs(ctypes.Structure):
    _fields_ = [("n_steps", ctypes.c_int32), ("max_trials", ctypes.c_int32), ("a", ctypes.c_double),
                ("eps", ctypes.c_double), ("state", _fp)]


class pct_sweep_params(ctypes.Structure):
    _fields_ = [("algo", ctypes.c_int32), ("block_size", ctypes.c_int64), ("lambda_", ctypes.c_float),
                ("n_sweeps", ctypes.c_int32), ("order", _fp), ("hull_mask", _fp),
                ("tvs", ctypes.POINTER(pct_tvs))]


EXPORTS = ("pct_workspace_size", "pct_mlp_trace", "pct_project_sweep", "pct_project_sweep_noalloc", "pct_plan_build", "pct_plan_sweep",
           "pct_plan_residual", "pct_reconstruct", "pct_residual", "pct_roi_stats", "pct_profile_enable",
           "pct_tvs_apply", "pct_carp", "pct_carp_workspace_size", "pct_carve_hull",
           "pct_profile_read", "pct_last_error", "pct_probe", "pct_probe_bytes",
           "pct_cnn_conv3d", "pct_cnn_conv3d_bwd_data", "pct_cnn_wgrad_scratch", "pct_cnn_conv3d_bwd_weight", "pct_cnn_conv3d_bwd_weight_bf16",
           "pct_cnn_conv3d_bf16_scratch", "pct_cnn_conv3d_bf16", "pct_cnn_conv3d_bwd_data_bf16",
           "pct_cnn_relu", "pct_cnn_relu_bwd", "pct_cnn_pool", "pct_cnn_pool_bwd", "pct_cnn_upsample",
           "pct_cnn_upsample_bwd", "pct_cnn_add", "pct_cnn_axpy", "pct_cnn_mask", "pct_cnn_mse_scratch", "pct_cnn_mse", "pct_cnn_adam")
KERNEL_CLASSES = ("trace_path", "trace_compact", "project", "apply", "residual", "art", "other", "plan_dot",
                  "plan_rows", "plan_scatter", "plan_build", "path_setup", "tvs", "carp", "carve", "project_counting")

_lib = None


class PctError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def load(path: str | None = None):
    """Load libpct.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} is missing: build it with paper_1707_05014_amd.build.build() "
                          f"(or __graft_entry__.build())")
    lib = ctypes.CDLL(p)
    P = ctypes.POINTER
    lib.pct_workspace_size.restype = ctypes.c_size_t
    lib.pct_workspace_size.argtypes = [P(pct_grid), P(pct_geom), P(pct_sweep_params), ctypes.c_int64,
                                       ctypes.c_int32]
    lib.pct_mlp_trace.restype = ctypes.c_int
    lib.pct_mlp_trace.argtypes = [P(pct_grid), P(pct_geom), P(pct_histories), P(pct_rows), _fp, ctypes.c_size_t,
                                  _fp]
    lib.pct_project_sweep.restype = ctypes.c_int
    lib.pct_project_sweep.argtypes = [P(pct_grid), P(pct_geom), P(pct_histories), P(pct_rows), _fp,
                                      P(pct_sweep_params), _fp, _fp, ctypes.c_size_t, _fp]
    lib.pct_project_sweep_noalloc.restype = ctypes.c_int
    lib.pct_project_sweep_noalloc.argtypes = [P(pct_grid), P(pct_geom), P(pct_histories), P(pct_rows), _fp,
                                              P(pct_sweep_params), _fp, _fp]
    lib.pct_plan_build.restype = ctypes.c_int
    lib.pct_plan_build.argtypes = [P(pct_grid), P(pct_histories), P(pct_rows), P(pct_sweep_params), P(pct_plan),
                                   _fp, ctypes.c_size_t, _fp]
    lib.pct_plan_sweep.restype = ctypes.c_int
    lib.pct_plan_sweep.argtypes = [P(pct_grid), P(pct_plan), _fp, P(pct_sweep_params), _fp, _fp, ctypes.c_size_t,
                                   _fp]
    lib.pct_plan_residual.restype = ctypes.c_int
    lib.pct_plan_residual.argtypes = [P(pct_grid), P(pct_plan), _fp, _fp, _fp, ctypes.c_size_t, _fp]
    lib.pct_reconstruct.restype = ctypes.c_int
    lib.pct_reconstruct.argtypes = [P(pct_grid), P(pct_geom), P(pct_histories), P(pct_sweep_params), P(pct_rows),
                                    P(pct_plan), _fp, P(ctypes.c_double), _fp, ctypes.c_size_t, _fp]
    lib.pct_residual.restype = ctypes.c_int
    lib.pct_residual.argtypes = [P(pct_grid), P(pct_geom), P(pct_histories), P(pct_rows), _fp, _fp, _fp,
                                 ctypes.c_size_t, _fp]
    lib.pct_tvs_apply.restype = ctypes.c_int
    lib.pct_tvs_apply.argtypes = [P(pct_grid), _fp, _fp, P(pct_tvs), _fp, ctypes.c_size_t, _fp]
    lib.pct_carp_workspace_size.restype = ctypes.c_size_t
    lib.pct_carp_workspace_size.argtypes = [P(pct_grid), P(pct_geom), P(pct_sweep_params), ctypes.c_int64,
                                            ctypes.c_int32]
    lib.pct_carp.restype = ctypes.c_int
    lib.pct_carp.argtypes = [P(pct_grid), P(pct_geom), P(pct_histories), P(pct_sweep_params), ctypes.c_int32,
                             P(pct_rows), _fp, P(ctypes.c_double), _fp, ctypes.c_size_t, _fp]
    lib.pct_carve_hull.restype = ctypes.c_int
    lib.pct_carve_hull.argtypes = [P(pct_grid), P(pct_geom), P(pct_histories), ctypes.c_float, ctypes.c_float, _fp,
                                   P(ctypes.c_int64), _fp, ctypes.c_size_t, _fp]
    lib.pct_roi_stats.restype = ctypes.c_int
    lib.pct_roi_stats.argtypes = [_fp, _fp, ctypes.c_int64, ctypes.c_int32, _fp, _fp, _fp]
    lib.pct_profile_enable.restype = ctypes.c_int
    lib.pct_profile_enable.argtypes = [ctypes.c_int32]
    lib.pct_profile_read.restype = ctypes.c_int
    lib.pct_profile_read.argtypes = [P(ctypes.c_int64), P(ctypes.c_double)]
    lib.pct_probe_bytes.restype = ctypes.c_size_t
    lib.pct_probe_bytes.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64]
    lib.pct_probe.restype = ctypes.c_int
    lib.pct_probe.argtypes = [ctypes.c_int32, _fp, ctypes.c_size_t, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                              P(ctypes.c_double), _fp]
    lib.pct_last_error.restype = ctypes.c_char_p
    lib.pct_last_error.argtypes = []
    i32, i64, f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    cnn = {
        "pct_cnn_conv3d": [_fp, _fp, _fp, _fp, i32, i32, i32, i32, i32, _fp],
        "pct_cnn_conv3d_bwd_data": [_fp, _fp, _fp, _fp, i32, i32, i32, i32, i32, _fp],
        "pct_cnn_conv3d_bwd_weight": [_fp, _fp, _fp, _fp, _fp, i32, i32, i32, i32, i32, _fp],
        "pct_cnn_conv3d_bwd_weight_bf16": [_fp, _fp, _fp, _fp, _fp, i32, i32, i32, i32, i32, _fp],
        "pct_cnn_conv3d_bf16": [_fp, _fp, _fp, _fp, _fp, i32, i32, i32, i32, i32, _fp],
        "pct_cnn_conv3d_bwd_data_bf16": [_fp, _fp, _fp, _fp, _fp, i32, i32, i32, i32, i32, _fp],
        "pct_cnn_relu": [_fp, _fp, i64, _fp],
        "pct_cnn_relu_bwd": [_fp, _fp, _fp, i64, _fp],
        "pct_cnn_pool": [_fp, _fp, i32, i32, i32, i32, _fp],
        "pct_cnn_pool_bwd": [_fp, _fp, i32, i32, i32, i32, _fp],
        "pct_cnn_upsample": [_fp, _fp, i32, i32, i32, i32, _fp],
        "pct_cnn_upsample_bwd": [_fp, _fp, i32, i32, i32, i32, _fp],
        "pct_cnn_add": [_fp, _fp, _fp, i64, _fp],
        "pct_cnn_mask": [_fp, _fp, _fp, i64, _fp],
        "pct_cnn_axpy": [f32, _fp, _fp, i64, _fp],
        "pct_cnn_mse": [_fp, _fp, _fp, _fp, _fp, i64, _fp],
        "pct_cnn_adam": [_fp, _fp, _fp, _fp, i64, f32, f32, f32, f32, i32, _fp],
    }
    for name, argt in cnn.items():
        fn = getattr(lib, name)
        fn.restype = ctypes.c_int
        fn.argtypes = argt
    lib.pct_cnn_conv3d_bf16_scratch.restype = i64
    lib.pct_cnn_conv3d_bf16_scratch.argtypes = [i32, i32]
    lib.pct_cnn_wgrad_scratch.restype = i64
    lib.pct_cnn_wgrad_scratch.argtypes = [i32, i32, i32, i32, i32]
    lib.pct_cnn_mse_scratch.restype = i64
    lib.pct_cnn_mse_scratch.argtypes = [i64]
    if path is None:
        _lib = lib
    return lib


def check(code: int, allow=(PCT_OK,)) -> int:
    if code not in allow:
        msg = load().pct_last_error().decode(errors="replace")
        raise PctError(code, msg)
    return code
