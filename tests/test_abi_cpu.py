"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol include/pct.h declares, and rejects bad arguments on the host
before touching the device."""
import ctypes
import os
import re

import pytest

from paper_1707_05014_amd import _lib, api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pct.h")).read()
    return sorted(set(re.findall(r"\b(pct_[a-z_0-9]+)\s*\(", src)))


def test_header_matches_exports():
    names = _declared()
    assert set(names) == set(_lib.EXPORTS)
    lib = _lib.load()
    for n in names:
        assert hasattr(lib, n), n


def test_struct_sizes_match_header():
    # sizes the C compiler gives the structs (x86-64 SysV): checked against ctypes
    assert ctypes.sizeof(_lib.pct_grid) == 36
    assert ctypes.sizeof(_lib.pct_geom) == 48 + 64 + 16
    assert ctypes.sizeof(_lib.pct_histories) == 8 + 10 * 8
    assert ctypes.sizeof(_lib.pct_rows) == 3 * 8 + 3 * 8 + 8 + 8
    assert ctypes.sizeof(_lib.pct_sweep_params) == 4 + 4 + 8 + 4 + 4 + 8 + 8 + 8
    assert ctypes.sizeof(_lib.pct_tvs) == 4 + 4 + 8 + 8 + 8
    assert ctypes.sizeof(_lib.pct_plan) == 8 + 8 + 10 * 8 + 4 * 4 + 2 * 8 + 2 * 4


def _grid():
    return api.make_grid(8, 8, 4, 1, 1, 1, -4, -4, -2)


def _geom(**kw):
    d = dict(u_in=-10, u_out=10, hull_a=3, hull_b=3, hull_zmin=-1, hull_zmax=1, step_mm=1.0, poly=[7.5e-6])
    d.update(kw)
    return api.make_geom(**d)


def test_workspace_size():
    lib = _lib.load()
    g = _grid()
    a = lib.pct_workspace_size(ctypes.byref(g), None, None, 100, 0)
    b = lib.pct_workspace_size(ctypes.byref(g), None, None, 10 ** 6, 0)
    assert 0 < a <= b
    bad = api.make_grid(0, 8, 4)
    assert lib.pct_workspace_size(ctypes.byref(bad), None, None, 100, 0) == 0


@pytest.mark.parametrize("kw,msg", [
    (dict(step_mm=2.0), "step_mm"),
    (dict(step_mm=0.0), "step_mm"),
    (dict(hull_a=0.0), "hull"),
    (dict(u_in=10, u_out=-10), "u_out"),
    (dict(poly=[]), "n_poly"),
])
def test_invalid_geometry_rejected(kw, msg):
    lib = _lib.load()
    g = _grid()
    geo = _geom(**kw)
    hs = _lib.pct_histories()
    hs.n = 0
    rs = _lib.pct_rows()
    rs.n_rows = 0
    rs.row_ptr = 1  # never dereferenced: the call fails validation first
    ws = ctypes.create_string_buffer(1)
    code = lib.pct_mlp_trace(ctypes.byref(g), ctypes.byref(geo), ctypes.byref(hs), ctypes.byref(rs), ws, 1, None)
    assert code == _lib.PCT_EINVAL
    assert msg in lib.pct_last_error().decode()


def test_small_workspace_rejected():
    lib = _lib.load()
    g = _grid()
    geo = _geom()
    hs = _lib.pct_histories()
    hs.n = 0
    rs = _lib.pct_rows()
    rs.n_rows = 0
    rs.row_ptr = 1
    ws = ctypes.create_string_buffer(16)
    code = lib.pct_mlp_trace(ctypes.byref(g), ctypes.byref(geo), ctypes.byref(hs), ctypes.byref(rs), ws, 16, None)
    assert code == _lib.PCT_ENOMEM


def test_bad_params_rejected():
    lib = _lib.load()
    g = _grid()
    geo = _geom()
    hs = _lib.pct_histories()
    hs.n = 0
    need = lib.pct_workspace_size(ctypes.byref(g), None, None, 0, 0)
    ws = ctypes.create_string_buffer(need)
    x = ctypes.create_string_buffer(4 * 256)
    for p in (api.sweep_params("drop", 0, 0.5), api.sweep_params("drop", 10, 2.5),
              api.sweep_params("drop", 10, 0.0)):
        code = lib.pct_project_sweep(ctypes.byref(g), ctypes.byref(geo), ctypes.byref(hs), None, x,
                                     ctypes.byref(p.struct), None, ws, need, None)
        assert code == _lib.PCT_EINVAL
    # ART needs cached rows
    p = api.sweep_params("art", 1, 0.5)
    code = lib.pct_project_sweep(ctypes.byref(g), ctypes.byref(geo), ctypes.byref(hs), None, x, ctypes.byref(p.struct),
                                 None, ws, need, None)
    assert code == _lib.PCT_EINVAL
    assert "ART" in lib.pct_last_error().decode()


def test_roi_args_rejected():
    lib = _lib.load()
    assert lib.pct_roi_stats(None, None, 10, 3, None, None, None) == _lib.PCT_EINVAL
    assert lib.pct_roi_stats(None, None, 0, 0, None, None, None) == _lib.PCT_EINVAL


def test_cnn_args_rejected_on_host():
    """The warm-start network's entry points check sizes and pointers on the
    host (nothing is launched for a bad call)."""
    lib = _lib.load()
    p = ctypes.c_void_p(1)  # never dereferenced: every call below fails validation first
    E = _lib.PCT_EINVAL
    assert lib.pct_cnn_conv3d(None, p, None, p, 1, 1, 4, 4, 4, None) == E
    assert lib.pct_cnn_conv3d(p, p, None, p, 0, 1, 4, 4, 4, None) == E
    assert lib.pct_cnn_conv3d(p, p, None, p, 1, 0, 4, 4, 4, None) == E
    assert lib.pct_cnn_conv3d(p, p, None, p, 1, 1, 0, 4, 4, None) == E
    assert lib.pct_cnn_conv3d_bwd_data(p, p, p, None, 1, 1, 4, 4, 4, None) == E
    assert lib.pct_cnn_conv3d_bwd_weight(p, p, p, None, None, 1, 1, 4, 4, 4, None) == E
    assert lib.pct_cnn_conv3d_bwd_weight_bf16(p, p, p, None, p, 8, 16, 4, 4, 4, None) == E   # cin % 16 != 0
    assert lib.pct_cnn_conv3d_bwd_weight_bf16(p, p, p, None, p, 16, 24, 4, 4, 4, None) == E  # cout % 16 != 0
    assert lib.pct_cnn_conv3d_bwd_weight_bf16(p, p, p, None, None, 16, 16, 4, 4, 4, None) == E
    assert lib.pct_cnn_conv3d_bwd_weight_bf16(p, p, p, None, p, 16, 16, 512, 512, 512, None) == E  # 2^27 voxels
    assert lib.pct_cnn_pool(p, p, 1, 3, 4, 4, None) == E  # odd depth
    assert lib.pct_cnn_pool_bwd(p, p, 1, 4, 5, 4, None) == E
    assert lib.pct_cnn_upsample(None, p, 1, 2, 2, 2, None) == E
    assert lib.pct_cnn_relu(p, p, -1, None) == E
    assert lib.pct_cnn_add(p, None, p, 10, None) == E
    assert lib.pct_cnn_axpy(1.0, None, p, 10, None) == E
    assert lib.pct_cnn_mask(p, None, p, 10, None) == E
    assert lib.pct_cnn_mse(p, p, None, None, p, 10, None) == E
    assert lib.pct_cnn_adam(p, p, p, p, 10, 1e-3, 0.9, 0.999, 1e-8, 0, None) == E  # step < 1
    assert lib.pct_cnn_adam(p, p, p, p, 10, -1.0, 0.9, 0.999, 1e-8, 1, None) == E
    assert lib.pct_cnn_adam(p, p, p, p, 10, 1e-3, 1.0, 0.999, 1e-8, 1, None) == E
    # zero-sized elementwise calls are valid no-ops
    assert lib.pct_cnn_relu(None, None, 0, None) == _lib.PCT_OK
    assert lib.pct_cnn_add(None, None, None, 0, None) == _lib.PCT_OK
    # scratch sizes
    assert lib.pct_cnn_wgrad_scratch(2, 3, 5, 18, 70) == 2 * 2 * 1 * 3 * (2 * 27 + 1)  # 2 x 2 x 1 tiles
    assert lib.pct_cnn_wgrad_scratch(0, 3, 5, 18, 70) == 0
    # shapes the matrix-core form takes: room for its slabs of 32 x 4 x 2 voxel
    # tiles too (here 3 x 5 x 3 = 45 tiles, one slab each, 2 x 1 channel tiles)
    assert lib.pct_cnn_wgrad_scratch(16, 32, 5, 18, 70) == 45 * 32 * (16 * 27 + 1)
    assert lib.pct_cnn_mse_scratch(257) == 2


def test_workspace_grows_for_fused_records():
    """A fused workspace holds one 128-byte path record per history (and,
    for a DROP run of several sweeps, the per-block voxel counts)."""
    lib = _lib.load()
    g = _grid()
    n = 3 << 20
    cached = lib.pct_workspace_size(ctypes.byref(g), None, None, n, 0)
    fused = lib.pct_workspace_size(ctypes.byref(g), None, None, n, 1)
    assert fused - cached >= (n - (1 << 20)) * 128
    p = api.sweep_params("drop", 1 << 20, 0.5, 4)
    kept = lib.pct_workspace_size(ctypes.byref(g), None, ctypes.byref(p.struct), n, 1)
    assert kept - fused >= 3 * g.nx * g.ny * g.nz * 2


def test_tvs_carp_carve_args_rejected_on_host():
    lib = _lib.load()
    g = _grid()
    geo = _geom()
    x = ctypes.c_float(0.0)
    t = _lib.pct_tvs(1, 0, 0.9, 1e-3, None)       # max_trials 0
    assert lib.pct_tvs_apply(ctypes.byref(g), ctypes.addressof(x), None, ctypes.byref(t), None, 0, None) == \
        _lib.PCT_EINVAL
    t = _lib.pct_tvs(1, 3, 1.5, 1e-3, None)       # a outside (0, 1)
    assert lib.pct_tvs_apply(ctypes.byref(g), ctypes.addressof(x), None, ctypes.byref(t), None, 0, None) == \
        _lib.PCT_EINVAL
    t = _lib.pct_tvs(0, 0, 0.0, 0.0, None)        # off: nothing to do
    assert lib.pct_tvs_apply(ctypes.byref(g), ctypes.addressof(x), None, ctypes.byref(t), None, 0, None) == _lib.PCT_OK
    h = _lib.pct_histories()
    h.n = 0
    p = api.sweep_params("drop", 10, 0.5, 1)
    for ns in (0, 5000):
        assert lib.pct_carp(ctypes.byref(g), ctypes.byref(geo), ctypes.byref(h), ctypes.byref(p.struct), ns, None,
                            ctypes.addressof(x), None, None, 0, None) == _lib.PCT_EINVAL
    assert lib.pct_carve_hull(ctypes.byref(g), ctypes.byref(geo), ctypes.byref(h), 1.5, 1e-6, None, None, None, 0,
                              None) == _lib.PCT_EINVAL
    assert lib.pct_carve_hull(ctypes.byref(g), ctypes.byref(geo), ctypes.byref(h), float("inf"), 1e-6,
                              ctypes.addressof(x), None, None, 0, None) == _lib.PCT_EINVAL
    # ART with TVS is refused
    tv = _lib.pct_tvs(1, 3, 0.9, 1e-3, ctypes.addressof(ctypes.c_double(1.0)))
    pa = api.sweep_params("art", 1, 0.5, 1)
    pa.struct.tvs = ctypes.pointer(tv)
    assert lib.pct_project_sweep(ctypes.byref(g), ctypes.byref(geo), ctypes.byref(h), None, ctypes.addressof(x),
                                 ctypes.byref(pa.struct), None, None, 0, None) == _lib.PCT_EINVAL


def test_probe_args_rejected_on_host():
    """The memory-path probes check kind, sizes, counts and the buffer on the
    host before any launch."""
    lib = _lib.load()
    ms = ctypes.c_double(0.0)
    buf = ctypes.c_void_p(1)  # never dereferenced: every call below fails validation first
    E = _lib.PCT_EINVAL
    K = _lib.PROBE_KINDS
    assert lib.pct_probe(9, buf, 1 << 30, 1024, 1 << 20, 1, ctypes.byref(ms), None) == E
    assert lib.pct_probe(K["copy"], buf, 1 << 30, 1022, 0, 1, ctypes.byref(ms), None) == E   # not a multiple of 4
    assert lib.pct_probe(K["atomic"], buf, 1 << 30, 32, 1 << 20, 1, ctypes.byref(ms), None) == E  # region < 64
    assert lib.pct_probe(K["atomic"], buf, 1 << 30, 100_000, 1 << 20, 1, ctypes.byref(ms), None) == E  # not slabs
    assert lib.pct_probe(K["atomic"], buf, 1 << 30, 160_000, 100, 1, ctypes.byref(ms), None) == E  # too few ops
    assert lib.pct_probe(K["gather"], buf, 1 << 30, 160_000, 1 << 20, 0, ctypes.byref(ms), None) == E  # reps
    assert lib.pct_probe(K["gather"], buf, 1 << 30, 160_000, 1 << 20, 1, None, None) == E
    need = lib.pct_probe_bytes(K["atomic_xcd"], 1_600_000, 1 << 26)
    assert need == 8 * 4 * 1_600_000
    assert lib.pct_probe(K["atomic_xcd"], buf, need - 1, 1_600_000, 1 << 26, 1, ctypes.byref(ms), None) == \
        _lib.PCT_ENOMEM
    assert lib.pct_probe_bytes(K["copy"], 1024, 0) == 8 * 1024
    assert lib.pct_probe_bytes(7, 1024, 0) == 0
