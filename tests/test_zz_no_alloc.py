"""pct_project_sweep_noalloc (the sweep over cached rows with the library's
static scratch instead of a workspace) against pct_project_sweep on the same
inputs, through the C ABI: two calls in a row, the second on a smaller input
(fewer histories, a smaller grid), each compared with the workspace form's
image and residual.  The DROP numerators are FP32 atomic sums in both forms,
so their order, and the last bits of the image, may differ between runs: the
images must agree to 1e-6 relative L2 and the residuals to 1e-6 relative."""
import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402
from helpers import pct_args  # noqa: E402
from paper_1707_05014_amd import _lib, api  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _case(cfg, n, block, algo):
    h = synth.generate(cfg, n=n)
    order = synth.block_order(n, cfg.perm_seed)
    mask = synth.hull_mask(cfg)
    grid, geom = pct_args(cfg)
    H = api.Histories.from_numpy(h)
    rows = api.mlp_trace(grid, geom, H)
    params = api.sweep_params(algo, block, 0.5, 1, order=torch.from_numpy(order).cuda(),
                              hull_mask=torch.from_numpy(mask).cuda())
    x0 = torch.from_numpy(mask.astype(np.float32)).cuda()
    return grid, geom, H, rows, params, x0


def _noalloc(grid, geom, H, rows, x, params, res):
    lib = _lib.load()
    hs, rs = H.struct(), rows.struct()
    return lib.pct_project_sweep_noalloc(ctypes.byref(grid), ctypes.byref(geom), ctypes.byref(hs), ctypes.byref(rs),
                                         x.data_ptr(), ctypes.byref(params.struct),
                                         res.data_ptr() if res is not None else None, None)


def _rel(a, b):
    return float(torch.linalg.vector_norm((a - b).double()) / torch.linalg.vector_norm(b.double()))


def test_noalloc_sweep_matches_workspace_sweep():
    big = synth.config(1, n=40_000)
    small = synth.config(1, n=40_000)
    small.grid = synth.Grid(40, 40, 12, 1.0, 1.0, 1.0, -20.0, -20.0, -6.0)
    cases = [("DROP, 40000 histories, 64x64x16 voxels", big, 40_000, 1000, "drop"),
             ("DROP, 9000 histories, 40x40x12 voxels", small, 9_000, 700, "drop"),
             ("ART, 3000 histories, 40x40x12 voxels", small, 3_000, 1, "art")]
    for name, cfg, n, block, algo in cases:
        _say(f"no-alloc sweep: {name}")
        grid, geom, H, rows, params, x0 = _case(cfg, n, block, algo)
        xa, xb = x0.clone(), x0.clone()
        ra = torch.zeros(1, dtype=torch.float64, device="cuda")
        rb = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        for sweep in range(2):
            api.project_sweep(grid, geom, H, rows, xa, params, resid_out=ra)
            _lib.check(_noalloc(grid, geom, H, rows, xb, params, rb))
            torch.cuda.synchronize()
            e = _rel(xb, xa)
            er = abs(float(rb) - float(ra)) / float(ra)
            moved = _rel(xa, x0)
            _say(f"  sweep {sweep + 1}: image rel-L2 {e:.2e} (moved {moved:.3f}), residual {float(rb):.6g} "
                 f"vs {float(ra):.6g} ({er:.1e})")
            assert moved > 1e-3
            assert e <= 1e-6
            assert er <= 1e-6


def test_noalloc_rejects_what_it_cannot_run():
    cfg = synth.config(1, n=2_000)
    grid, geom, H, rows, params, x0 = _case(cfg, 2_000, 500, "drop")
    lib = _lib.load()
    hs = H.struct()
    # no rows
    st = lib.pct_project_sweep_noalloc(ctypes.byref(grid), ctypes.byref(geom), ctypes.byref(hs), None,
                                       x0.data_ptr(), ctypes.byref(params.struct), None, None)
    assert st == _lib.PCT_EINVAL and b"cached rows" in lib.pct_last_error()
    # a grid beyond the static scratch (2^21 voxels)
    huge = api.make_grid(256, 256, 40, 1, 1, 1, -128, -128, -20)
    st = _noalloc(huge, geom, H, rows, x0, params, None)
    assert st == _lib.PCT_EINVAL and b"no-allocation scratch" in lib.pct_last_error()
    # TV superiorization asks for a workspace
    tv = api.Tvs(n_steps=1)
    p2 = api.sweep_params("drop", 500, 0.5, 1, order=params.order, hull_mask=params.hull_mask, tvs=tv)
    st = _noalloc(grid, geom, H, rows, x0, p2, None)
    assert st == _lib.PCT_EINVAL and b"superiorization" in lib.pct_last_error()
