"""The 1e7-history workload at full size, in the launch configuration that
bench.py times (one trace of all histories, one plan for blocks of 2e5, the
plan sweep), checked on what the oracle can compute one by one and on
properties that hold at any size:

* rows of 200000 seeded-random histories against the FP64 oracle's rows of
  the same histories: index sets identical on >= 99.99 % of them, and of
  those, every length within 1e-4 mm on >= 99.99 %; every voxel on one side
  only lies where the oracle's path passes within 1e-4 mm of its faces, and
  every length more than 1e-4 mm off lies where the path runs within 1e-4 mm
  of one of the voxel's faces (a crossing of a face at a grazing angle moves
  length between two voxels by the position difference over the sine of the
  angle); FP64 squared norms within 1e-4 relative;
* every one of the 1e7 rows holds each voxel once (a device sort of the
  (row, voxel) pairs);
* one plan sweep (tiled, atomic-free) against one sweep of the plan-less CSR
  path (global atomics) over the same rows and blocks: relative L2 <= 1e-5
  (the two differ only in the order of the FP32 sums);
* one fused sweep (rows rebuilt in every block) against the same CSR sweep:
  relative L2 <= 1e-5;
* the residual after the sweep equals the plan-less residual (1e-5 relative).
The CSR and fused paths are themselves checked against the oracle's DROP
on the smaller workload (test_gpu_parity.py).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
import synth  # noqa: E402
from helpers import (check_mismatch_geometry, compare_rows, merge_rows, mismatch_voxels, oracle_geom,  # noqa: E402
                     oracle_grid, pct_args)
from paper_1707_05014_amd import api  # noqa: E402

N_SAMPLE = 200_000


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def full():
    cfg = synth.config(2)
    _say(f"full-size workload: {cfg.n} histories, {cfg.grid.nx}x{cfg.grid.ny}x{cfg.grid.nz}")
    h = synth.generate(cfg)
    grid, geom = pct_args(cfg)
    H = api.Histories.from_numpy(h)
    rows = api.mlp_trace(grid, geom, H)
    torch.cuda.synchronize()
    _say(f"  rows: {rows.nnz} entries")
    return cfg, h, grid, geom, H, rows


def test_full_size_rows_sampled(full):
    cfg, h, grid, geom, H, rows = full
    sel = np.sort(np.random.default_rng(77).choice(cfg.n, N_SAMPLE, replace=False))
    hs = {k: np.ascontiguousarray(v[sel]) for k, v in h.items()}
    R = oracle.trace(oracle_grid(cfg), oracle_geom(cfg), hs)
    rp = rows.row_ptr.cpu().numpy()
    idx = rows.idx[: rows.nnz].cpu().numpy()
    ln = rows.len[: rows.nnz].cpu().numpy().astype(np.float64)
    n2 = rows.norm2.cpu().numpy()
    starts, ends = rp[sel], rp[sel + 1]
    sp = np.zeros(N_SAMPLE + 1, np.int64)
    sp[1:] = np.cumsum(ends - starts)
    take = np.concatenate([np.arange(a, b) for a, b in zip(starts, ends)]) if N_SAMPLE else np.zeros(0, np.int64)
    mp, mi, ml, dups = merge_rows(sp, idx[take], ln[take])
    assert dups == 0
    c = compare_rows(R.row_ptr, R.idx, R.len, mp, mi, ml)
    _say(f"  sampled rows identical {c['frac_identical']:.6f} ({len(c['bad_rows'])} differ); of those, with every "
         f"length within 1e-4 mm {c['frac_len_ok']:.6f}; max dlen {c['max_dlen']:.2e}, max one-sided "
         f"{c['max_only_len']:.2e}")
    assert c["frac_identical"] >= 0.9999
    assert c["frac_len_ok"] >= 0.9999
    cases = mismatch_voxels(R.row_ptr, R.idx, R.len, mp, mi, ml, 1e-4)
    bad, worst = check_mismatch_geometry(cfg, oracle_geom(cfg), h, sel, cases)
    _say(f"  {len(cases)} mismatched voxels; deepest one-sided penetration {worst:.2e} mm; outside the face "
         f"class: {bad[:5]}")
    assert len(cases) <= 400 and not bad
    ok = R.norm2 > 0
    assert np.array_equal(ok, n2[sel] > 0)
    assert np.max(np.abs(n2[sel][ok] - R.norm2[ok]) / R.norm2[ok]) <= 1e-4


def test_full_size_rows_hold_each_voxel_once(full):
    """Duplicates would count a row twice in s_j and split ||a_i||^2 (Sec.
    2.1): checked over every row of the workload by sorting the (row, voxel)
    keys on the device."""
    cfg, h, grid, geom, H, rows = full
    rp = rows.row_ptr
    counts = (rp[1:] - rp[:-1])
    rid = torch.repeat_interleave(torch.arange(cfg.n, device=rp.device, dtype=torch.int64), counts)
    key = rid * (1 << 31) + rows.idx[: rows.nnz].to(torch.int64)
    del rid
    ks, _ = torch.sort(key)
    del key
    dups = int((ks[1:] == ks[:-1]).sum().item())
    _say(f"  {rows.nnz} entries over {cfg.n} rows; duplicate (row, voxel) pairs: {dups}")
    assert dups == 0


def test_full_size_sweeps_agree(full):
    cfg, h, grid, geom, H, rows = full
    order = torch.from_numpy(synth.block_order(cfg.n, cfg.perm_seed)).cuda()
    mask = torch.from_numpy(synth.hull_mask(cfg)).cuda()
    x0 = mask.to(torch.float32)
    params = api.sweep_params("drop", cfg.block, cfg.lam, 1, order=order, hull_mask=mask)
    plan = api.plan_build(grid, H, rows, params)
    xp = x0.clone()
    api.plan_sweep(grid, plan, xp, params)
    res_p = api.plan_residual(grid, plan, xp)
    xc = x0.clone()
    api.project_sweep(grid, geom, H, rows, xc, params)
    res_c = api.residual(grid, geom, H, rows, xc)
    xf = x0.clone()
    api.project_sweep(grid, geom, H, None, xf, params)
    torch.cuda.synchronize()
    rel_p = float(torch.linalg.vector_norm(xp - xc) / torch.linalg.vector_norm(xc))
    rel_f = float(torch.linalg.vector_norm(xf - xc) / torch.linalg.vector_norm(xc))
    moved = float(torch.linalg.vector_norm(xc - x0) / torch.linalg.vector_norm(x0))
    _say(f"  one sweep: plan vs CSR {rel_p:.2e}, fused vs CSR {rel_f:.2e} (the sweep moved x by {moved:.3f}); "
         f"residual plan {res_p:.6f} CSR {res_c:.6f}")
    assert moved > 1e-2
    assert rel_p <= 1e-5
    assert rel_f <= 1e-5
    assert abs(res_p - res_c) <= 1e-5 * res_c
