"""Pins of the oracle's voxel traversal (Sec. 2: the entries of A are the path
lengths in the voxels a proton touches).  Fixed by brute force, a hand-worked
example, axis-aligned chords and the total path length."""
import math
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _brute(grid, P, Q, n=400_000):
    """Midpoint sampling of the segment: length per voxel to within |PQ|/n per crossing."""
    P = np.asarray(P, float)
    Q = np.asarray(Q, float)
    a = (np.arange(n) + 0.5) / n
    X = P[None, :] + a[:, None] * (Q - P)[None, :]
    d = np.array([grid.dx, grid.dy, grid.dz])
    o = np.array([grid.ox, grid.oy, grid.oz])
    iv = np.floor((X - o) / d).astype(np.int64)
    nn = np.array([grid.nx, grid.ny, grid.nz])
    ok = np.all((iv >= 0) & (iv < nn), axis=1)
    j = (iv[ok, 2] * grid.ny + iv[ok, 1]) * grid.nx + iv[ok, 0]
    seg = np.linalg.norm(Q - P)
    cnt = np.bincount(j, minlength=grid.nx * grid.ny * grid.nz)
    nz = np.nonzero(cnt)[0]
    return nz, cnt[nz] * seg / n


def test_golden_hand_example():
    grid = oracle.make_grid(4, 4, 4, 1.0, 1.0, 1.0, 0.0, 0.0, 0.0)
    ref = np.loadtxt(os.path.join(GOLD, "siddon_2d_example.txt"))
    idx, ln, n2 = oracle.polyline_row(grid, [[0.5, 0.5, 0.5], [2.5, 1.5, 0.5]])
    assert idx.tolist() == ref[:, 0].astype(int).tolist()
    assert np.allclose(ln, ref[:, 1], rtol=0, atol=1e-15)
    assert n2 == pytest.approx(np.sum(ref[:, 1] ** 2), rel=1e-15)


def test_brute_force_random_segments():
    grid = oracle.make_grid(4, 4, 4, 1.0, 1.0, 1.0, 0.0, 0.0, 0.0)
    rng = np.random.default_rng(1)
    n = 400_000
    for _ in range(25):
        P = rng.uniform(-0.5, 4.5, 3)
        Q = rng.uniform(-0.5, 4.5, 3)
        idx, ln, _ = oracle.polyline_row(grid, [P, Q])
        bj, bl = _brute(grid, P, Q, n)
        seg = np.linalg.norm(Q - P)
        tol = 4 * seg / n
        # every voxel the brute force sees with more than a few samples is in the row
        strong = bl > 3 * tol
        assert set(bj[strong].tolist()) <= set(idx.tolist())
        full = dict(zip(idx.tolist(), ln.tolist()))
        for j, l in zip(bj, bl):
            assert abs(full.get(int(j), 0.0) - l) <= tol
        for j, l in full.items():
            if j not in set(bj.tolist()):
                assert l <= tol


def test_anisotropic_grid_brute_force():
    grid = oracle.make_grid(5, 3, 4, 0.7, 1.3, 0.9, -1.0, 0.5, -2.0)
    rng = np.random.default_rng(2)
    n = 400_000
    for _ in range(10):
        lo = np.array([-1.5, 0.0, -2.5])
        hi = np.array([3.0, 5.0, 2.0])
        P = rng.uniform(lo, hi)
        Q = rng.uniform(lo, hi)
        idx, ln, _ = oracle.polyline_row(grid, [P, Q])
        bj, bl = _brute(grid, P, Q, n)
        full = dict(zip(idx.tolist(), ln.tolist()))
        tol = 4 * np.linalg.norm(Q - P) / n
        for j, l in zip(bj, bl):
            assert abs(full.get(int(j), 0.0) - l) <= tol


def test_axis_chords():
    nx, ny, nz = 7, 5, 3
    grid = oracle.make_grid(nx, ny, nz, 1.0, 1.0, 1.0, 0.0, 0.0, 0.0)
    # along x through voxel interiors: exactly nx entries of length dx
    idx, ln, n2 = oracle.polyline_row(grid, [[-2.0, 2.3, 1.6], [9.0, 2.3, 1.6]])
    assert len(idx) == nx
    assert np.allclose(ln, 1.0, atol=1e-12)
    assert idx.tolist() == [(1 * ny + 2) * nx + i for i in range(nx)]
    assert n2 == pytest.approx(nx)
    # along z
    idx, ln, _ = oracle.polyline_row(grid, [[3.5, 4.5, -1.0], [3.5, 4.5, 5.0]])
    assert idx.tolist() == [(k * ny + 4) * nx + 3 for k in range(nz)]
    assert np.allclose(ln, 1.0, atol=1e-12)


def test_total_length_and_bounds():
    grid = oracle.make_grid(16, 16, 8, 1.0, 1.0, 1.0, -8.0, -8.0, -4.0)
    rng = np.random.default_rng(3)
    diag = math.sqrt(3.0)
    for _ in range(30):
        # polyline strictly inside the grid
        pts = np.cumsum(rng.normal(0, 0.6, (40, 3)), axis=0)
        pts = np.clip(pts, [-7.9, -7.9, -3.9], [7.9, 7.9, 3.9])
        idx, ln, n2 = oracle.polyline_row(grid, pts)
        total = np.sum(np.linalg.norm(np.diff(pts, axis=0), axis=1))
        assert ln.sum() == pytest.approx(total, rel=1e-12)
        assert np.all(np.diff(idx) > 0)
        assert n2 == pytest.approx(np.sum(ln ** 2), rel=1e-14)
        # a single straight segment cannot hold more than a voxel diagonal in one voxel
        idx1, ln1, _ = oracle.polyline_row(grid, pts[[0, -1]])
        assert np.all(ln1 <= diag + 1e-12)


def test_outside_grid_skipped():
    grid = oracle.make_grid(4, 4, 4, 1.0, 1.0, 1.0, 0.0, 0.0, 0.0)
    idx, ln, _ = oracle.polyline_row(grid, [[-3.0, 1.5, 1.5], [7.0, 1.5, 1.5]])
    assert len(idx) == 4 and np.allclose(ln, 1.0)
    idx, ln, _ = oracle.polyline_row(grid, [[-3.0, 9.5, 1.5], [7.0, 9.5, 1.5]])
    assert len(idx) == 0


def test_row_length_bound():
    """The path kernels size each wavefront's row buffer for 2 entries per path
    sample plus 16.  What fixes that: a row has at most one more entry than
    the voxel faces its path crosses, and along each axis a path crosses at
    most (its total variation along the axis) / (voxel size) faces plus one
    per monotone stretch; an MLP path has at most three monotone stretches per
    coordinate, and the total variations add up to at most sqrt(3) times the
    arc length s.  So entries <= sqrt(3) s / dmin + 10, checked on the
    oracle's rows of seeded phantoms (s = the row's total length), and the
    longest row against the buffer size the kernels reserve."""
    import sys

    sys.path.insert(0, os.path.dirname(__file__))
    import synth
    from helpers import oracle_geom, oracle_grid

    for which in (1, 2):
        cfg = synth.config(which, n=20000)
        h = synth.generate(cfg)
        R = oracle.trace(oracle_grid(cfg), oracle_geom(cfg), h)
        cnt = np.diff(R.row_ptr)
        ok = cnt > 0
        s = np.add.reduceat(R.len, R.row_ptr[:-1][ok])
        g = cfg.grid
        dmin = min(g.dx, g.dy, g.dz)
        assert np.all(cnt[ok] <= math.sqrt(3.0) * s / dmin + 10)
        b = cfg.phantom.body
        kmax = math.ceil(2 * max(b.ax[0], b.ax[1]) / dmin) + 2
        emax = 2 * (kmax + 1) + 16
        print(f"config {which}: longest row {cnt.max()} entries, buffer {emax}; "
              f"max entries / (sqrt(3) s / dmin + 10) = {np.max(cnt[ok] / (math.sqrt(3.0) * s / dmin + 10)):.3f}")
        assert cnt.max() <= emax
