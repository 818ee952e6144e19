"""TV superiorization (Sec. 4.2), CARP (Sec. 2.2) and the space-carving
hull on the GPU against the FP64 oracle, through the C ABI.

* TVS steps on a noisy image: image within 1e-6 relative L2, the same steps
  kept and the same final step size (the decisions are FP64 sums of the
  same quantities on both sides);
* DROP with TVS before every block (cached rows, tiled plan, rows rebuilt
  in every block) against the oracle's DROP-TVS: image within 1e-3 relative
  L2 after a fixed number of sweeps, same step size at the end;
* CARP (4 strings; cached and rebuilt rows; with and without TVS) against
  the oracle's CARP: image within 1e-3 relative L2, residuals within 1e-3;
* the carved hull: byte-exact against the oracle (both cut the lines at the
  same FP64 crossing parameters), on the tiny and the head grids.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402
from helpers import oracle_geom, oracle_grid, pct_args  # noqa: E402
from paper_1707_05014_amd import api  # noqa: E402

IMG_TOL = 1e-3
TVS = dict(n_steps=2, max_trials=3, a=0.97, eps=1e-3)
BETA0 = 1.5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def c1():
    cfg = synth.config(1, n=40_000)
    h = synth.generate(cfg)
    R = oracle.trace(oracle_grid(cfg), oracle_geom(cfg), h)
    return cfg, h, R


def test_tvs_steps_match_oracle(c1):
    cfg, h, R = c1
    g = cfg.grid
    rng = np.random.default_rng(21)
    truth = synth.truth_image(cfg).astype(np.float64)
    mask = synth.hull_mask(cfg)
    x0 = ((truth + rng.normal(0, 0.05, g.M)) * mask).astype(np.float32).astype(np.float64)
    t = oracle.make_tvs(n_steps=6, max_trials=4, a=0.9, eps=1e-3)
    xo, bo, acc = oracle.tvs_apply(oracle_grid(cfg), x0, t, 3.0, mask=mask)
    grid, _ = pct_args(cfg)
    tv = api.Tvs(beta0=3.0, n_steps=6, max_trials=4, a=0.9, eps=1e-3)
    x = torch.from_numpy(x0.astype(np.float32)).cuda()
    api.tvs_apply(grid, x, tv, torch.from_numpy(mask).cuda())
    torch.cuda.synchronize()
    xg = x.cpu().numpy().astype(np.float64)
    _say(f"TVS: accepted oracle {acc} gpu {tv.accepted}; beta oracle {bo:.9e} gpu {tv.beta:.9e}; rel-L2 "
         f"{_rel(xg, xo):.2e}; TV {oracle.tv(oracle_grid(cfg), x0, 1e-3):.2f} -> {oracle.tv(oracle_grid(cfg), xo, 1e-3):.2f}")
    assert acc == tv.accepted and acc > 0
    assert tv.beta == pytest.approx(bo, rel=1e-12)
    assert _rel(xg, xo) <= 1e-6


@pytest.mark.parametrize("form", ["csr", "plan", "fused"])
def test_drop_with_tvs_matches_oracle(c1, form):
    cfg, h, R = c1
    order = synth.block_order(cfg.n, cfg.perm_seed)
    mask = synth.hull_mask(cfg)
    block, sweeps = 5000, 3
    t = oracle.make_tvs(**TVS)
    xo, ro, bo = oracle.drop_tvs(oracle_grid(cfg), R, h["wepl"], mask.astype(np.float64), order, block, cfg.lam,
                                 sweeps, t, BETA0, mask=mask)
    grid, geom = pct_args(cfg)
    H = api.Histories.from_numpy(h)
    tv = api.Tvs(beta0=BETA0, **TVS)
    params = api.sweep_params("drop", block, cfg.lam, sweeps, order=torch.from_numpy(order).cuda(),
                              hull_mask=torch.from_numpy(mask).cuda(), tvs=tv)
    x = torch.from_numpy(mask.astype(np.float32)).cuda()
    rows = None if form == "fused" else api.mlp_trace(grid, geom, H)
    plan = api.plan_build(grid, H, rows, params) if form == "plan" else None
    rg = api.reconstruct(grid, geom, H, params, x, rows=rows, plan=plan)
    torch.cuda.synchronize()
    xg = x.cpu().numpy().astype(np.float64)
    xd, _ = oracle.drop(R, h["wepl"], mask.astype(np.float64), order, block, cfg.lam, sweeps, mask=mask)
    _say(f"DROP+TVS {form}: rel-L2 {_rel(xg, xo):.2e} (TVS moved the oracle image by {_rel(xo, xd):.2e}); beta "
         f"oracle {bo:.6e} gpu {tv.beta:.6e}; residual oracle {ro[-1]:.4f} gpu {rg[-1]:.4f}")
    assert _rel(xo, xd) > 1e-3
    assert _rel(xg, xo) <= IMG_TOL
    assert tv.beta == pytest.approx(bo, rel=1e-12)
    assert np.allclose(rg, ro, rtol=1e-3)


@pytest.mark.parametrize("form,with_tvs", [("csr", False), ("fused", False), ("csr", True)])
def test_carp_matches_oracle(c1, form, with_tvs):
    cfg, h, R = c1
    order = synth.block_order(cfg.n, cfg.perm_seed)
    mask = synth.hull_mask(cfg)
    strings, block, iters = 4, 2500, 3
    t = oracle.make_tvs(**TVS) if with_tvs else None
    xo, ro, bo = oracle.carp(oracle_grid(cfg), R, h["wepl"], mask.astype(np.float64), order, strings, block, cfg.lam,
                             iters, mask=mask, tvs=t, beta=BETA0)
    grid, geom = pct_args(cfg)
    H = api.Histories.from_numpy(h)
    tv = api.Tvs(beta0=BETA0, **TVS) if with_tvs else None
    params = api.sweep_params("drop", block, cfg.lam, iters, order=torch.from_numpy(order).cuda(),
                              hull_mask=torch.from_numpy(mask).cuda(), tvs=tv)
    x = torch.from_numpy(mask.astype(np.float32)).cuda()
    rows = None if form == "fused" else api.mlp_trace(grid, geom, H)
    rg = api.carp(grid, geom, H, params, strings, x, rows=rows)
    torch.cuda.synchronize()
    xg = x.cpu().numpy().astype(np.float64)
    _say(f"CARP {form} tvs={with_tvs}: rel-L2 {_rel(xg, xo):.2e}; residuals oracle {np.round(ro, 4).tolist()} gpu "
         f"{np.round(rg, 4).tolist()}")
    assert _rel(xg, xo) <= IMG_TOL
    assert np.allclose(rg, ro, rtol=1e-3)
    if with_tvs:
        assert tv.beta == pytest.approx(bo, rel=1e-12)


@pytest.mark.parametrize("key,n_miss,n_hit", [(1, 200_000, 50_000), (2, 400_000, 100_000)])
def test_carved_hull_is_byte_exact(key, n_miss, n_hit):
    cfg = synth.config(key)
    m = synth.generate_misses(cfg, n_miss)
    hh = synth.generate(cfg, n=n_hit)
    h = {k: np.concatenate([m[k], hh[k]]) for k in m}
    co, uo = oracle.carve(oracle_grid(cfg), oracle_geom(cfg), h, wepl_max=1.5)
    grid, geom = pct_args(cfg)
    hull, ug = api.carve_hull(grid, geom, api.Histories.from_numpy(h), wepl_max=1.5)
    torch.cuda.synchronize()
    hg = hull.cpu().numpy()
    diff = int(np.sum(hg != (1 - co)))
    ana = synth.hull_mask(cfg).astype(bool)
    keep = hg.astype(bool)
    _say(f"carve config {key}: used oracle {uo} gpu {ug}; carved {int(co.sum())}; mismatched voxels {diff}; kept "
         f"{int(keep.sum())} vs analytic hull {int(ana.sum())} (analytic voxels carved: {int(np.sum(ana & ~keep))})")
    assert uo == ug
    assert diff == 0
