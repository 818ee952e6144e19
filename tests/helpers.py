"""Shared test helpers: turn a synthetic workload into oracle arguments."""
from __future__ import annotations

import numpy as np

import oracle
import synth


def oracle_grid(cfg: synth.Config) -> oracle.OrcGrid:
    g = cfg.grid
    return oracle.make_grid(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.ox, g.oy, g.oz)


def oracle_geom(cfg: synth.Config, poly=None, highland_log: bool = True, step: float | None = None):
    b = cfg.phantom.body
    poly = synth.prior_poly(cfg.beam.E_kin) if poly is None else poly
    return oracle.make_geom(cfg.beam.u_in, cfg.beam.u_out, b.ax[0], b.ax[1], b.z0, b.z1,
                            min(cfg.grid.dx, cfg.grid.dy, cfg.grid.dz) if step is None else step,
                            poly, highland_log=highland_log)


def hist_row(h: dict, i: int) -> np.ndarray:
    return np.array([h[k][i] for k in oracle.FIELDS], dtype=np.float64)


# ----------------------------------------------------------------- GPU side
def pct_args(cfg: synth.Config, poly=None, highland_log: bool = True, step: float | None = None):
    """(pct_grid, pct_geom) of a workload for the HIP library."""
    from paper_1707_05014_amd import api
    g = cfg.grid
    b = cfg.phantom.body
    poly = synth.prior_poly(cfg.beam.E_kin) if poly is None else poly
    grid = api.make_grid(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.ox, g.oy, g.oz)
    geom = api.make_geom(cfg.beam.u_in, cfg.beam.u_out, b.ax[0], b.ax[1], b.z0, b.z1,
                         min(g.dx, g.dy, g.dz) if step is None else step, poly, highland_log=highland_log)
    return grid, geom


def merge_rows(row_ptr, idx, ln):
    """Per-row sort by voxel and sum of equal voxels (host, numpy).
    Returns (row_ptr, idx, len, dup_count)."""
    row_ptr = np.asarray(row_ptr, np.int64)
    n = len(row_ptr) - 1
    rid = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    key = rid * (1 << 31) + np.asarray(idx, np.int64)
    o = np.argsort(key, kind="stable")
    key = key[o]
    ln = np.asarray(ln, np.float64)[o]
    uk, first = np.unique(key, return_index=True)
    sums = np.add.reduceat(ln, first) if len(ln) else ln
    dups = len(key) - len(uk)
    r = uk >> 31
    new_ptr = np.zeros(n + 1, np.int64)
    np.add.at(new_ptr, r + 1, 1)
    return np.cumsum(new_ptr), (uk & ((1 << 31) - 1)).astype(np.int32), sums, dups


def compare_rows(o_ptr, o_idx, o_len, g_ptr, g_idx, g_len, len_tol=1e-4):
    """Compare two sets of fully merged, voxel-sorted rows.
    Returns dict: frac_identical (index sets), mismatch rows, max |dlen| on
    common voxels of identical rows, max length of a voxel present on one side
    only, and frac_len_ok: the share of the rows with identical index sets
    whose every length is within len_tol."""
    n = len(o_ptr) - 1
    ro = np.repeat(np.arange(n, dtype=np.int64), np.diff(o_ptr))
    rg = np.repeat(np.arange(n, dtype=np.int64), np.diff(g_ptr))
    ko = ro * (1 << 31) + o_idx.astype(np.int64)
    kg = rg * (1 << 31) + g_idx.astype(np.int64)
    in_g = np.isin(ko, kg, assume_unique=True)
    in_o = np.isin(kg, ko, assume_unique=True)
    bad_rows = np.union1d(ro[~in_g], rg[~in_o])
    good = np.ones(n, bool)
    good[bad_rows] = False
    # lengths on common voxels (both arrays sorted by key, so the common parts align)
    lo = o_len[in_g]
    lg = g_len[in_o]
    common_rows = ro[in_g]
    d = np.abs(lo - lg)
    max_d_good = float(d[good[common_rows]].max()) if np.any(good[common_rows]) else 0.0
    only = np.concatenate([o_len[~in_g], g_len[~in_o]])
    ok = good.copy()
    ok[np.unique(common_rows[d > len_tol])] = False
    n_good = int(good.sum())
    return dict(frac_identical=float(good.mean()) if n else 1.0, bad_rows=bad_rows,
                frac_len_ok=float(ok.sum()) / n_good if n_good else 1.0,
                max_dlen=max_d_good, max_dlen_all=float(d.max()) if len(d) else 0.0,
                max_only_len=float(only.max()) if len(only) else 0.0)
