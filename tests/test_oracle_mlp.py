"""Pins of the oracle's most-likely path (Sec. 2: the path estimated from the
entry and exit positions and angles; Bayesian form of Schulte et al. 2008).

Each pin is fixed by mathematics outside the oracle's own code: end states,
the straight-line limit, the cubic-Hermite limit of a constant prior, the
Kalman-gain form with independently integrated covariances, invariances and
symmetries.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.interpolate import CubicHermiteSpline

import oracle
import synth
from helpers import hist_row, oracle_geom

CFG1 = synth.config(1)
CFG2 = synth.config(2)


def _hist(cfg, n=64, seed=None):
    return synth.generate(cfg, n=n, seed=seed)


def _line_state(h, which, u, geom):
    if which == "in":
        return (h[1] + h[3] * (u - geom.u_in), h[2] + h[4] * (u - geom.u_in))
    return (h[5] + h[7] * (u - geom.u_out), h[6] + h[8] * (u - geom.u_out))


def _inside_hull(cfg, phi, u, t, v):
    b = cfg.phantom.body
    x = u * math.cos(phi) - t * math.sin(phi)
    y = u * math.sin(phi) + t * math.cos(phi)
    return (x / b.ax[0]) ** 2 + (y / b.ax[1]) ** 2 <= 1.0 and b.z0 <= v <= b.z1


@pytest.mark.parametrize("cfg", [CFG1, CFG2], ids=["cyl", "ellipse"])
def test_end_states_on_hull(cfg):
    geom = oracle_geom(cfg)
    H = _hist(cfg, 64)
    n_ok = 0
    for i in range(64):
        h = hist_row(H, i)
        u, t, v = oracle.mlp_path(geom, h)
        if len(u) == 0:
            continue
        n_ok += 1
        t0, v0 = _line_state(h, "in", u[0], geom)
        t2, v2 = _line_state(h, "out", u[-1], geom)
        assert t[0] == pytest.approx(t0, abs=1e-12) and v[0] == pytest.approx(v0, abs=1e-12)
        assert t[-1] == pytest.approx(t2, abs=1e-12) and v[-1] == pytest.approx(v2, abs=1e-12)
        # entry point is on the hull boundary: just before outside, just after inside
        eps = 1e-7
        ta, va = _line_state(h, "in", u[0] - eps, geom)
        tb, vb = _line_state(h, "in", u[0] + eps, geom)
        assert not _inside_hull(cfg, h[0], u[0] - eps, ta, va)
        assert _inside_hull(cfg, h[0], u[0] + eps, tb, vb)
        ta, va = _line_state(h, "out", u[-1] - eps, geom)
        tb, vb = _line_state(h, "out", u[-1] + eps, geom)
        assert _inside_hull(cfg, h[0], u[-1] - eps, ta, va)
        assert not _inside_hull(cfg, h[0], u[-1] + eps, tb, vb)
        # uniform samples, spacing at most the step
        du = np.diff(u)
        assert np.allclose(du, du[0], rtol=0, atol=1e-9)
        assert du[0] <= geom.step + 1e-9
        assert len(u) - 1 == max(1, math.ceil((u[-1] - u[0]) / geom.step - 1e-9))
    assert n_ok > 50


@pytest.mark.parametrize("cfg", [CFG1, CFG2], ids=["cyl", "ellipse"])
def test_straight_line_limit(cfg):
    """Exit state = straight extrapolation of the entry state: the MLP is that
    line for any prior, and the row's lengths add up to the hull chord."""
    geom = oracle_geom(cfg)
    rng = np.random.default_rng(5)
    grid = __import__("helpers").oracle_grid(cfg)
    body_only = synth.Phantom(synth.Shape(1, (0, 0, 0), cfg.phantom.body.ax, 0.0, cfg.phantom.body.z0,
                                          cfg.phantom.body.z1, 1.0), [])
    for _ in range(40):
        phi = rng.uniform(0, 2 * np.pi)
        t_in = rng.uniform(-0.8, 0.8) * cfg.phantom.body.ax[1]
        v_in = rng.uniform(-0.8, 0.8) * cfg.phantom.body.z1
        st, sv = rng.normal(0, 0.02, 2)
        L = geom.u_out - geom.u_in
        h = np.array([phi, t_in, v_in, st, sv, t_in + st * L, v_in + sv * L, st, sv, 0.0])
        u, t, v = oracle.mlp_path(geom, h)
        if len(u) == 0:
            continue
        tl = t_in + st * (u - geom.u_in)
        vl = v_in + sv * (u - geom.u_in)
        assert np.max(np.abs(t - tl)) < 1e-9
        assert np.max(np.abs(v - vl)) < 1e-9
        # sum of row lengths = chord of the line through the hull (independent
        # chord from the generator's analytic shape code)
        P = [u[0] * math.cos(phi) - t[0] * math.sin(phi), u[0] * math.sin(phi) + t[0] * math.cos(phi), v[0]]
        uu = np.array([geom.u_in, geom.u_out])
        tt = t_in + st * (uu - geom.u_in)
        vv = v_in + sv * (uu - geom.u_in)
        A = [uu[0] * math.cos(phi) - tt[0] * math.sin(phi), uu[0] * math.sin(phi) + tt[0] * math.cos(phi), vv[0]]
        B = [uu[1] * math.cos(phi) - tt[1] * math.sin(phi), uu[1] * math.sin(phi) + tt[1] * math.cos(phi), vv[1]]
        chord = synth.segment_wepl(body_only, A, B)
        xyz = np.stack([u * math.cos(phi) - t * math.sin(phi), u * math.sin(phi) + t * math.cos(phi), v], 1)
        idx, ln, _ = oracle.polyline_row(grid, xyz)
        assert ln.sum() == pytest.approx(chord, rel=1e-10, abs=1e-9)
        assert P[2] == pytest.approx(v[0])


def test_cubic_hermite_limit():
    """Constant 1/(beta p)^2 and no logarithmic factor: the most-likely path
    is the cubic Hermite interpolant of the two end states (offsets and
    slopes) in each plane."""
    cfg = CFG2
    geom = oracle_geom(cfg, poly=[7.5e-6], highland_log=False)
    H = _hist(cfg, 32)
    for i in range(32):
        h = hist_row(H, i)
        u, t, v = oracle.mlp_path(geom, h)
        if len(u) < 3:
            continue
        sp_t = CubicHermiteSpline([u[0], u[-1]], [t[0], t[-1]], [h[3], h[7]])
        sp_v = CubicHermiteSpline([u[0], u[-1]], [v[0], v[-1]], [h[4], h[8]])
        assert np.max(np.abs(t - sp_t(u))) < 1e-9
        assert np.max(np.abs(v - sp_v(u))) < 1e-9


def _kalman_reference(poly, E0, X0, hl, u0, u2, y0, y2, u):
    """Posterior mode written in Kalman-gain form, covariances integrated by
    adaptive quadrature from their definitions."""
    f = np.polynomial.polynomial.Polynomial(poly)
    L = u2 - u0
    d1 = u - u0

    def g(d):
        return (1.0 + 0.038 * math.log(d / X0)) ** 2 if hl else 1.0

    def S(a, b, e, gg):
        m = [quad(lambda s: f(s) * (e - s) ** k, a, b, epsabs=0, epsrel=1e-13, limit=200)[0] for k in range(3)]
        c = E0 * E0 / X0 * gg
        return c * np.array([[m[2], m[1]], [m[1], m[0]]])

    S1 = S(0.0, d1, d1, g(d1))
    S2 = S(d1, L, L, g(L - d1))
    R0 = np.array([[1.0, d1], [0.0, 1.0]])
    R1 = np.array([[1.0, L - d1], [0.0, 1.0]])
    Kg = S1 @ R1.T @ np.linalg.inv(R1 @ S1 @ R1.T + S2)
    return R0 @ y0 + Kg @ (y2 - R1 @ R0 @ y0)


@pytest.mark.parametrize("hl", [True, False])
def test_kalman_form_with_depth_prior(hl):
    cfg = CFG2
    poly = synth.prior_poly()
    geom = oracle_geom(cfg, poly=poly, highland_log=hl)
    H = _hist(cfg, 12, seed=77)
    checked = 0
    for i in range(12):
        h = hist_row(H, i)
        u, t, v = oracle.mlp_path(geom, h)
        if len(u) < 5:
            continue
        y0t = np.array([t[0], h[3]])
        y2t = np.array([t[-1], h[7]])
        y0v = np.array([v[0], h[4]])
        y2v = np.array([v[-1], h[8]])
        for k in (1, len(u) // 3, len(u) // 2, len(u) - 2):
            rt = _kalman_reference(poly, 13.6, 360.8, hl, u[0], u[-1], y0t, y2t, u[k])
            rv = _kalman_reference(poly, 13.6, 360.8, hl, u[0], u[-1], y0v, y2v, u[k])
            assert t[k] == pytest.approx(rt[0], abs=1e-9)
            assert v[k] == pytest.approx(rv[0], abs=1e-9)
            checked += 1
    assert checked >= 20


def test_invariances():
    """Scaling the Highland constant or the prior's amplitude leaves the path
    unchanged (both covariances scale together)."""
    cfg = CFG2
    poly = synth.prior_poly()
    H = _hist(cfg, 16, seed=9)
    g_a = oracle_geom(cfg, poly=poly)
    g_b = oracle_geom(cfg, poly=3.0 * poly)
    g_c = oracle.make_geom(g_a.u_in, g_a.u_out, g_a.hull_a, g_a.hull_b, g_a.hull_zmin, g_a.hull_zmax, g_a.step,
                           poly, highland_log=True, E0=27.2, X0=360.8)
    for i in range(16):
        h = hist_row(H, i)
        ua, ta, va = oracle.mlp_path(g_a, h)
        for gg in (g_b, g_c):
            ub, tb, vb = oracle.mlp_path(gg, h)
            assert np.allclose(ta, tb, atol=1e-10) and np.allclose(va, vb, atol=1e-10)


def test_mirror_equivariance():
    """Circular hull, slab symmetric about z = 0: mirroring t -> -t and
    v -> -v mirrors the path."""
    cfg = CFG1
    geom = oracle_geom(cfg)
    H = _hist(cfg, 16, seed=11)
    for i in range(16):
        h = hist_row(H, i)
        m = h.copy()
        m[[1, 3, 5, 7]] *= -1.0
        m[[2, 4, 6, 8]] *= -1.0
        u, t, v = oracle.mlp_path(geom, h)
        um, tm, vm = oracle.mlp_path(geom, m)
        assert np.allclose(u, um, atol=1e-12)
        assert np.allclose(t, -tm, atol=1e-10) and np.allclose(v, -vm, atol=1e-10)


def test_reversal_symmetry_constant_prior():
    """With a constant prior and no logarithmic factor, tracing the proton
    backwards (gantry angle + pi, exit and entry swapped) gives the same
    curve in the object frame."""
    cfg = CFG1
    geom = oracle_geom(cfg, poly=[7.5e-6], highland_log=False)
    assert geom.u_in == -geom.u_out
    H = _hist(cfg, 16, seed=13)
    for i in range(16):
        h = hist_row(H, i)
        r = np.array([h[0] + np.pi, -h[5], h[6], h[7], -h[8], -h[1], h[2], h[3], -h[4], h[9]])
        u, t, v = oracle.mlp_path(geom, h)
        ur, tr, vr = oracle.mlp_path(geom, r)
        if len(u) == 0:
            assert len(ur) == 0
            continue
        P = np.stack([u * np.cos(h[0]) - t * np.sin(h[0]), u * np.sin(h[0]) + t * np.cos(h[0]), v], 1)
        Q = np.stack([ur * np.cos(r[0]) - tr * np.sin(r[0]), ur * np.sin(r[0]) + tr * np.cos(r[0]), vr], 1)
        assert len(P) == len(Q)
        assert np.max(np.abs(P - Q[::-1])) < 1e-9


def test_empty_and_nonfinite():
    cfg = CFG1
    geom = oracle_geom(cfg)
    # misses the hull entirely (far off in t)
    h = np.array([0.0, 500.0, 0.0, 0.0, 0.0, 500.0, 0.0, 0.0, 0.0, 1.0])
    assert len(oracle.mlp_path(geom, h)[0]) == 0
    h = np.array([0.0, np.nan, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0])
    assert len(oracle.mlp_path(geom, h)[0]) == 0
