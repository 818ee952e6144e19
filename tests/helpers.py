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
