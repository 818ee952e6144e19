"""Pins of the oracle's solvers (Sec. 2: iterative solution of the sparse,
over-determined Ax = b; Sec. 2.1: DROP's block-sequential scheme with a
fixed number of iterations).  Fixed by closed-form solutions of small
systems and a hand-worked block update."""
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows_from_dense(A):
    A = np.asarray(A, float)
    rp = [0]
    idx, ln = [], []
    for r in A:
        nz = np.nonzero(r)[0]
        idx += nz.tolist()
        ln += r[nz].tolist()
        rp.append(len(idx))
    return oracle.Rows(np.array(rp, np.int64), np.array(idx, np.int32), np.array(ln, float),
                       np.sum(A * A, axis=1))


def _sparse_pos(rng, n, m, density):
    A = rng.uniform(0.1, 1.5, (n, m)) * (rng.uniform(size=(n, m)) < density)
    for i in range(n):
        if not A[i].any():
            A[i, rng.integers(m)] = 1.0
    return A


def test_golden_block_update():
    ref = np.loadtxt(os.path.join(GOLD, "drop_block_example.txt"))
    R = _rows_from_dense([[1, 2, 0], [0, 1, 1]])
    x, _ = oracle.drop(R, [5.0, 2.0], np.zeros(3), np.arange(2), block=2, lam=1.0, sweeps=1)
    assert np.allclose(x, ref[:, 1], atol=1e-15)


def test_art_minimum_norm():
    """ART from x = 0 on a consistent under-determined system converges to
    the minimum-norm solution pinv(A) b."""
    rng = np.random.default_rng(0)
    A = _sparse_pos(rng, 8, 20, 0.5)
    xt = rng.uniform(0, 2, 20)
    b = A @ xt
    R = _rows_from_dense(A)
    x, _ = oracle.drop(R, b, np.zeros(20), rng.permutation(8), block=1, lam=1.0, sweeps=3000)
    assert np.allclose(x, np.linalg.pinv(A) @ b, atol=1e-11)


def test_drop_consistent_recovers_truth():
    rng = np.random.default_rng(1)
    A = _sparse_pos(rng, 60, 12, 0.5)
    xt = rng.uniform(0.2, 1.8, 12)
    b = A @ xt
    R = _rows_from_dense(A)
    x, res = oracle.drop(R, b, np.zeros(12), np.arange(60), block=60, lam=1.5, sweeps=4000)
    assert np.allclose(x, xt, atol=1e-11)
    assert res[-1] < 1e-9


def test_drop_noisy_weighted_least_squares():
    """One block on inconsistent data: the fixed point solves
    A^T D (b - A x) = 0 with D = diag(1/||a_i||^2)."""
    rng = np.random.default_rng(2)
    A = _sparse_pos(rng, 50, 10, 0.6)
    b = A @ rng.uniform(0.2, 1.8, 10) + rng.normal(0, 0.1, 50)
    R = _rows_from_dense(A)
    x, _ = oracle.drop(R, b, np.zeros(10), np.arange(50), block=50, lam=1.0, sweeps=6000)
    D = np.diag(1.0 / np.sum(A * A, axis=1))
    xw = np.linalg.solve(A.T @ D @ A, A.T @ D @ b)
    assert np.allclose(x, xw, atol=1e-10)


def test_block_count_matters():
    """The per-block voxel counts s_j: a two-row block on disjoint supports
    equals two one-row blocks; on a shared voxel the update is averaged."""
    R = _rows_from_dense([[1, 0], [0, 2]])
    xa, _ = oracle.drop(R, [1.0, 4.0], np.zeros(2), np.arange(2), block=2, lam=1.0, sweeps=1)
    xb, _ = oracle.drop(R, [1.0, 4.0], np.zeros(2), np.arange(2), block=1, lam=1.0, sweeps=1)
    assert np.allclose(xa, [1.0, 2.0]) and np.allclose(xb, [1.0, 2.0])
    R = _rows_from_dense([[1.0], [1.0]])
    x, _ = oracle.drop(R, [2.0, 4.0], np.zeros(1), np.arange(2), block=2, lam=1.0, sweeps=1)
    assert np.allclose(x, [3.0])        # (2 + 4) / 2


def test_mask_and_empty_rows():
    R = _rows_from_dense([[1, 1, 0], [0, 0, 0], [0, 1, 1]])
    mask = np.array([1, 1, 0], np.uint8)
    x, res = oracle.drop(R, [2.0, 7.0, 2.0], np.array([0.0, 0.0, 5.0]), np.arange(3), block=1, lam=1.0,
                         sweeps=1, mask=mask)
    assert x[2] == 0.0
    # row 0: r = 2/2 -> x = [1, 1, 0]; row 1 empty; row 2: r = (2 - 1)/2 -> x1 += 0.5
    assert np.allclose(x, [1.0, 1.5, 0.0])
    # residual over non-empty rows only
    assert res[0] == pytest.approx(np.hypot(2.5 - 2.0, 1.5 - 2.0))


def test_residual_closed_form():
    rng = np.random.default_rng(4)
    A = _sparse_pos(rng, 30, 9, 0.4)
    b = rng.normal(size=30)
    x = rng.normal(size=9)
    assert oracle.residual(_rows_from_dense(A), b, x) == pytest.approx(np.linalg.norm(A @ x - b), rel=1e-14)


def test_roi_means():
    x = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    lab = np.array([0, 1, 1, 2, 0], np.uint8)
    assert np.allclose(oracle.roi_means(x, lab, 2), [2.5, 4.0])
    assert oracle.rsp_error(x, lab, np.array([2.5, 5.0])) == pytest.approx(0.2)


@pytest.mark.parametrize("key,n,block", [(1, 20_000, 1_000), (2, 6_000, 2_500)])
def test_drop_recompute_equals_stored_rows(key, n, block):
    """DROP without stored A (each block's rows traced, projected, dropped;
    Sec. 2 / 4.1) gives exactly the image and residuals of DROP on the
    stored, pinned rows: same rows, same summation order."""
    import synth
    from helpers import oracle_geom, oracle_grid
    cfg = synth.config(key, n=n)
    h = synth.generate(cfg)
    G, g = oracle_grid(cfg), oracle_geom(cfg)
    order = synth.block_order(n, cfg.perm_seed)
    mask = synth.hull_mask(cfg)
    x0 = mask.astype(np.float64)
    R = oracle.trace(G, g, h)
    xs, rs = oracle.drop(R, h["wepl"], x0, order, block, 0.5, 2, mask=mask)
    xr, rr = oracle.drop_recompute(G, g, h, x0, order, block, 0.5, 2, mask=mask)
    assert np.array_equal(xs, xr)
    assert np.array_equal(rs, rr)
    # and the sweeps did move the image (the comparison is not vacuous)
    assert np.linalg.norm(xs - x0) > 1e-2 * np.linalg.norm(x0)
