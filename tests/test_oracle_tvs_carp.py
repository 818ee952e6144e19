"""Pins of the oracle's total-variation superiorization (Sec. 4.2) and of
CARP (Sec. 2.2), by closed forms, finite differences and reductions to the
pinned DROP."""
import numpy as np
import pytest

import oracle


def _grid(nx, ny, nz):
    return oracle.make_grid(nx, ny, nz, 1.0, 1.0, 1.0, 0.0, 0.0, 0.0)


def _rows_from_dense(A):
    A = np.asarray(A, float)
    rp = [0]
    idx, ln = [], []
    for r in A:
        nz = np.nonzero(r)[0]
        idx += nz.tolist()
        ln += r[nz].tolist()
        rp.append(len(idx))
    return oracle.Rows(np.array(rp, np.int64), np.array(idx, np.int32), np.array(ln, float), np.sum(A * A, axis=1))


def test_tv_constant_and_step_closed_forms():
    g = _grid(6, 5, 4)
    M, eps = 120, 0.01
    assert oracle.tv(g, np.full(M, 1.7), eps) == pytest.approx(M * eps, rel=1e-14)
    # a jump h between the halves x < 3 and x >= 3: only the 5 * 4 voxels at i = 2 see it
    x = np.zeros((4, 5, 6))
    x[:, :, 3:] = 0.8
    expect = (M - 20) * eps + 20 * np.sqrt(0.8 ** 2 + eps ** 2)
    assert oracle.tv(g, x.ravel(), eps) == pytest.approx(expect, rel=1e-14)
    # the same jump along z: 6 * 5 voxels at k = 1
    z = np.zeros((4, 5, 6))
    z[2:] = 0.8
    assert oracle.tv(g, z.ravel(), eps) == pytest.approx((M - 30) * eps + 30 * np.sqrt(0.64 + eps ** 2), rel=1e-14)


def test_tv_gradient_by_central_differences():
    g = _grid(5, 4, 3)
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 2, 60)
    eps = 0.05
    an = oracle.tv_grad(g, x, eps)
    h = 1e-6
    fd = np.empty(60)
    for u in range(60):
        e = np.zeros(60)
        e[u] = h
        fd[u] = (oracle.tv(g, x + e, eps) - oracle.tv(g, x - e, eps)) / (2 * h)
    assert np.max(np.abs(an - fd)) <= 1e-7 * np.max(np.abs(an))


def test_tvs_step_lowers_tv_and_follows_the_beta_sequence():
    g = _grid(12, 10, 4)
    rng = np.random.default_rng(5)
    base = np.zeros((4, 10, 12))
    base[:, 3:8, 4:9] = 1.0
    x = (base + rng.normal(0, 0.05, base.shape)).ravel()
    mask = np.ones(480, np.uint8)
    mask[:12] = 0
    x[mask == 0] = 0.0
    t = oracle.make_tvs(n_steps=5, max_trials=4, a=0.9, eps=1e-3)
    beta0 = 0.5
    y, beta, acc = oracle.tvs_apply(g, x, t, beta0, mask=mask)
    tv0, tv1 = oracle.tv(g, x, 1e-3), oracle.tv(g, y, 1e-3)
    assert tv1 < tv0
    assert np.array_equal(y[mask == 0], x[mask == 0])
    # beta shrank by a per trial: trials = accepted steps (first try each) here
    assert acc == 5
    assert beta == pytest.approx(beta0 * 0.9 ** 5, rel=1e-14)
    # each accepted step moved x by exactly the step size in L2
    steps = [beta0 * 0.9 ** k for k in range(5)]
    assert np.linalg.norm(y - x) <= sum(steps) + 1e-12
    # a constant image has no TV gradient: nothing changes, beta untouched
    c, bc, ac = oracle.tvs_apply(g, np.full(480, 0.3), t, beta0)
    assert ac == 0 and bc == beta0 and np.all(c == 0.3)


def test_tvs_rejects_a_step_that_raises_tv():
    """With a step far too large the trial overshoots (TV rises) and is
    refused; the smaller next step is taken."""
    g = _grid(8, 1, 1)
    x = np.array([0, 0, 0, 0, 1, 1, 1, 1.0])
    t = oracle.make_tvs(n_steps=1, max_trials=2, a=1e-3, eps=1e-6)
    y, beta, acc = oracle.tvs_apply(g, x, t, 100.0)
    assert acc == 1
    assert np.linalg.norm(y - x) == pytest.approx(0.1, rel=1e-12)   # the second trial: 100 * 1e-3
    assert beta == pytest.approx(100.0 * 1e-6, rel=1e-12)


def test_drop_tvs_without_steps_is_drop():
    rng = np.random.default_rng(7)
    A = rng.uniform(0.1, 1.5, (40, 24)) * (rng.uniform(size=(40, 24)) < 0.4)
    A[np.arange(40), rng.integers(0, 24, 40)] = 1.0
    R = _rows_from_dense(A)
    b = A @ rng.uniform(0.5, 1.5, 24)
    order = rng.permutation(40)
    g = _grid(24, 1, 1)
    xd, rd = oracle.drop(R, b, np.zeros(24), order, 8, 0.7, 3)
    xt, rt, _ = oracle.drop_tvs(g, R, b, np.zeros(24), order, 8, 0.7, 3, oracle.make_tvs(n_steps=0), 1.0)
    assert np.array_equal(xd, xt) and np.array_equal(rd, rt)


def test_drop_tvs_still_solves_a_consistent_system():
    """Superiorization: summable perturbations leave the solver's limit a
    solution (residual -> 0 on a consistent system)."""
    rng = np.random.default_rng(8)
    A = rng.uniform(0.1, 1.5, (80, 20)) * (rng.uniform(size=(80, 20)) < 0.5)
    A[np.arange(80), rng.integers(0, 20, 80)] = 1.0
    xt = np.repeat([0.5, 1.5], 10) + rng.normal(0, 0.05, 20)
    b = A @ xt
    g = _grid(20, 1, 1)
    x, res, beta = oracle.drop_tvs(g, _rows_from_dense(A), b, np.zeros(20), rng.permutation(80), 20, 1.0, 400,
                                   oracle.make_tvs(n_steps=1, max_trials=3, a=0.9, eps=1e-3), 0.5)
    assert res[-1] <= 1e-8 * np.linalg.norm(b)
    assert np.allclose(x, xt, atol=1e-7)


def test_carp_one_string_is_drop():
    rng = np.random.default_rng(9)
    A = rng.uniform(0.1, 1.5, (50, 30)) * (rng.uniform(size=(50, 30)) < 0.4)
    A[np.arange(50), rng.integers(0, 30, 50)] = 1.0
    R = _rows_from_dense(A)
    b = A @ rng.uniform(0.5, 1.5, 30)
    order = rng.permutation(50)
    xd, rd = oracle.drop(R, b, np.zeros(30), order, 7, 0.6, 4)
    xc, rc, _ = oracle.carp(_grid(30, 1, 1), R, b, np.zeros(30), order, 1, 7, 0.6, 4)
    assert np.array_equal(xd, xc) and np.array_equal(rd, rc)


def test_carp_disjoint_strings_reduce_to_drop_per_string():
    """Two strings whose rows touch disjoint voxels: each voxel is averaged
    over one string only, so one CARP iteration equals one DROP sweep of each
    string on its own."""
    rng = np.random.default_rng(10)
    A = np.zeros((30, 16))
    A[:15, :8] = rng.uniform(0.1, 1.5, (15, 8)) * (rng.uniform(size=(15, 8)) < 0.6)
    A[15:, 8:] = rng.uniform(0.1, 1.5, (15, 8)) * (rng.uniform(size=(15, 8)) < 0.6)
    A[np.arange(15), rng.integers(0, 8, 15)] = 1.0
    A[15 + np.arange(15), 8 + rng.integers(0, 8, 15)] = 1.0
    R = _rows_from_dense(A)
    b = A @ rng.uniform(0.5, 1.5, 16)
    order = np.concatenate([rng.permutation(15), 15 + rng.permutation(15)])
    x0 = rng.uniform(0.5, 1.5, 16)
    xc, _, _ = oracle.carp(_grid(16, 1, 1), R, b, x0, order, 2, 4, 0.8, 1)
    xa, _ = oracle.drop(_rows_from_dense(A[:15]), b[:15], x0, order[:15], 4, 0.8, 1)
    xb, _ = oracle.drop(_rows_from_dense(A[15:]), b[15:], x0, order[15:] - 15, 4, 0.8, 1)
    expect = np.concatenate([xa[:8], xb[8:]])
    assert np.allclose(xc, expect, rtol=0, atol=1e-15)


def test_carp_fixed_point_and_convergence():
    rng = np.random.default_rng(11)
    A = rng.uniform(0.1, 1.5, (90, 18)) * (rng.uniform(size=(90, 18)) < 0.5)
    A[np.arange(90), rng.integers(0, 18, 90)] = 1.0
    xt = rng.uniform(0.3, 1.7, 18)
    b = A @ xt
    R = _rows_from_dense(A)
    g = _grid(18, 1, 1)
    order = rng.permutation(90)
    xf, _, _ = oracle.carp(g, R, b, xt, order, 3, 5, 0.9, 3)
    assert np.allclose(xf, xt, rtol=0, atol=1e-14)
    xc, res, _ = oracle.carp(g, R, b, np.zeros(18), order, 3, 5, 0.9, 3000)
    assert np.allclose(xc, xt, atol=1e-9)
    assert res[-1] <= 1e-9 * np.linalg.norm(b)
