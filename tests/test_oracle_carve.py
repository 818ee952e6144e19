"""Pins of the oracle's space-carving hull: a hand-worked axis-aligned line,
lines through air never carving a voxel that lies wholly inside the body,
the WEPL threshold, and the union over histories."""
import numpy as np

import oracle
import synth
from helpers import oracle_geom, oracle_grid


def _one(phi, t, v, st=0.0, sv=0.0, w=0.0):
    f = dict(phi=phi, t_in=t, v_in=v, dt_in=st, dv_in=sv, t_out=t, v_out=v, dt_out=st, dv_out=sv, wepl=w)
    return {k: np.array([f[k]], np.float32) for k in oracle.FIELDS}


def test_axis_line_carves_one_voxel_row():
    cfg = synth.config(1)
    g = cfg.grid
    G, geo = oracle_grid(cfg), oracle_geom(cfg)
    # phi = 0: u along x, t along y, v along z; y = 3.5, z = 0.25 -> voxel row j = 35, k = 8
    c, used = oracle.carve(G, geo, _one(0.0, 3.5, 0.25), wepl_max=1.0)
    assert used == 1
    idx = np.nonzero(c)[0]
    ii, jj, kk = idx % g.nx, (idx // g.nx) % g.ny, idx // (g.nx * g.ny)
    assert np.array_equal(np.sort(ii), np.arange(g.nx))
    assert np.all(jj == 35) and np.all(kk == 8)
    # phi = pi/2: u along y, t along -x: x = -3.5 -> i = 28
    c2, _ = oracle.carve(G, geo, _one(np.pi / 2, 3.5, 0.25), wepl_max=1.0)
    idx = np.nonzero(c2)[0]
    assert np.all(idx % g.nx == 28) and len(idx) == g.ny


def test_threshold_and_nonfinite():
    cfg = synth.config(1)
    G, geo = oracle_grid(cfg), oracle_geom(cfg)
    c, used = oracle.carve(G, geo, _one(0.0, 3.5, 0.25, w=2.0), wepl_max=1.5)
    assert used == 0 and not c.any()
    h = _one(0.0, 3.5, 0.25)
    h["t_in"][0] = np.nan
    c, used = oracle.carve(G, geo, h, wepl_max=1.5)
    assert used == 0 and not c.any()


def test_air_lines_never_carve_the_body_and_union_holds():
    cfg = synth.config(1)
    g = cfg.grid
    body = cfg.phantom.body
    G, geo = oracle_grid(cfg), oracle_geom(cfg)
    m = synth.generate_misses(cfg, 20000)
    c, used = oracle.carve(G, geo, m, wepl_max=1.5)
    assert used > 15000 and c.sum() > 0
    # voxels whose 8 corners all lie inside the body
    X, Y, Z = g.centers()
    inside_all = np.ones(g.M, bool)
    for dx in (-0.5, 0.5):
        for dy in (-0.5, 0.5):
            for dz in (-0.5, 0.5):
                px, py, pz = X + dx * g.dx, Y + dy * g.dy, Z + dz * g.dz
                inside_all &= ((px / body.ax[0]) ** 2 + (py / body.ax[1]) ** 2 <= 1.0) & (pz >= body.z0) & (
                    pz <= body.z1)
    assert inside_all.sum() > 1000
    assert not np.any(c.astype(bool) & inside_all)
    # union over two halves of the histories
    a, _ = oracle.carve(G, geo, {k: v[:7000] for k, v in m.items()}, wepl_max=1.5)
    b, _ = oracle.carve(G, geo, {k: v[7000:] for k, v in m.items()}, wepl_max=1.5)
    assert np.array_equal(c, a | b)
