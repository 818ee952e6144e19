"""Images on the 200 x 200 x 40 grid of the benchmark workloads against the
FP64 oracle, element by element (relative L2 <= 1e-3 after a fixed number
of sweeps, Sec. 2.1's DROP):

* the 1e7-history workload's phantom with its first 2e6 histories, blocks of
  2e5, 6 sweeps from the hull start: the tiled plan with FP32 rows, the plan
  with FP16 rows (its error against the oracle is printed and bounded by the
  same bar), and the plan-less CSR sweep; residuals after every sweep within
  1e-4 relative;
* the 2e8-history workload's phantom (seed 3) with its first 2e6 histories,
  rows rebuilt in every block (never stored) and the block counts kept from
  the first sweep, 2 sweeps, against the oracle's DROP that also traces each
  block's rows afresh and drops them.
"""
import sys
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402
from helpers import oracle_geom, oracle_grid, pct_args  # noqa: E402
from paper_1707_05014_amd import api  # noqa: E402

N = 2_000_000
IMG_TOL = 1e-3


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def head2():
    cfg = synth.config(2, n=N)
    _say(f"oracle: phantom seed 2, {N} histories, {cfg.sweeps} sweeps of blocks of {cfg.block}")
    t0 = time.time()
    h = synth.generate(cfg)
    order = synth.block_order(N, cfg.perm_seed)
    mask = synth.hull_mask(cfg)
    R = oracle.trace(oracle_grid(cfg), oracle_geom(cfg), h)
    x, res = oracle.drop(R, h["wepl"], mask.astype(np.float64), order, cfg.block, cfg.lam, cfg.sweeps, mask=mask)
    del R
    _say(f"  oracle done in {time.time() - t0:.1f} s; residuals {np.round(res, 3).tolist()}")
    return cfg, h, order, mask, x, res


def _gpu(cfg, h, order, mask, sweeps, len_dtype=0, plan=True, fused=False):
    grid, geom = pct_args(cfg)
    H = api.Histories.from_numpy(h)
    x = torch.from_numpy(mask.astype(np.float32)).cuda()
    params = api.sweep_params("drop", cfg.block, cfg.lam, sweeps, order=torch.from_numpy(order).cuda(),
                              hull_mask=torch.from_numpy(mask).cuda())
    rows = None if fused else api.mlp_trace(grid, geom, H, len_dtype=len_dtype)
    pl = api.plan_build(grid, H, rows, params) if (plan and not fused) else None
    res = api.reconstruct(grid, geom, H, params, x, rows=rows, plan=pl)
    torch.cuda.synchronize()
    return x.cpu().numpy().astype(np.float64), np.array(res)


@pytest.mark.parametrize("form", ["plan-f32", "plan-f16", "csr-f32"])
def test_head_1e7_phantom_images_match_oracle(head2, form):
    cfg, h, order, mask, xo, ro = head2
    kind, dt = form.split("-")
    _say(f"GPU: {form}, {N} histories, {cfg.sweeps} sweeps")
    xg, rg = _gpu(cfg, h, order, mask, cfg.sweeps, len_dtype=1 if dt == "f16" else 0, plan=kind == "plan")
    rel = _rel(xg, xo)
    rres = np.max(np.abs(rg - ro) / ro)
    moved = _rel(xo, mask.astype(np.float64))
    _say(f"  image rel-L2 vs oracle {rel:.2e} (the sweeps moved the image by {moved:.3f}); residuals max rel "
         f"diff {rres:.2e}")
    assert moved > 1e-2
    assert rel <= IMG_TOL
    assert rres <= (1e-3 if dt == "f16" else 1e-4)


def test_head_2e8_phantom_fused_kept_counts_match_oracle():
    cfg = synth.config(3, n=N)
    sweeps = 2
    _say(f"oracle (rows traced per block, never stored): phantom seed 3, {N} histories, {sweeps} sweeps")
    t0 = time.time()
    h = synth.generate(cfg)
    order = synth.block_order(N, cfg.perm_seed)
    mask = synth.hull_mask(cfg)
    xo, ro = oracle.drop_recompute(oracle_grid(cfg), oracle_geom(cfg), h, mask.astype(np.float64), order, cfg.block,
                                   cfg.lam, sweeps, mask=mask)
    _say(f"  oracle done in {time.time() - t0:.1f} s; residuals {np.round(ro, 3).tolist()}")
    xg, rg = _gpu(cfg, h, order, mask, sweeps, fused=True)
    rel = _rel(xg, xo)
    rres = np.max(np.abs(rg - ro) / ro)
    _say(f"  fused (kept block counts) image rel-L2 vs oracle {rel:.2e}; residuals max rel diff {rres:.2e}")
    assert rel <= IMG_TOL
    assert rres <= 1e-4
