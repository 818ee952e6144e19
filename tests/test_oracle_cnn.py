"""Pins of the FP64 warm-start network oracle (oracle.cnn) against things
other than itself: scipy's n-dimensional correlation, special kernels with a
known result, adjoint identities, central finite differences and a property
of Adam's bias correction."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import cnn as oc


def _rng(seed=0):
    return np.random.default_rng(seed)


@pytest.mark.parametrize("shape", [(1, 1, 5, 6, 7), (3, 2, 4, 5, 3), (2, 3, 1, 1, 1)])
def test_conv_matches_scipy_correlate(shape):
    cin, cout, D, H, W = shape
    r = _rng(1)
    x = r.normal(size=(cin, D, H, W))
    w = r.normal(size=(cout, cin, 3, 3, 3))
    b = r.normal(size=cout)
    y = oc.conv3d(x, w, b)
    ref = np.zeros((cout, D, H, W))
    for co in range(cout):
        ref[co] = b[co]
        for ci in range(cin):
            ref[co] += ndimage.correlate(x[ci], w[co, ci], mode="constant", cval=0.0)
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12)


def test_delta_kernel_is_identity():
    r = _rng(2)
    x = r.normal(size=(3, 4, 5, 6))
    w = np.zeros((3, 3, 3, 3, 3))
    for c in range(3):
        w[c, c, 1, 1, 1] = 1.0
    np.testing.assert_array_equal(oc.conv3d(x, w), x)
    # a shifted delta moves the volume by one voxel, with a zero face
    ws = np.zeros((1, 1, 3, 3, 3))
    ws[0, 0, 1, 1, 2] = 1.0  # tap (0, 0, +1): y[.., x] = x[.., x + 1]
    y = oc.conv3d(x[:1], ws)
    np.testing.assert_array_equal(y[0, :, :, :-1], x[0, :, :, 1:])
    np.testing.assert_array_equal(y[0, :, :, -1], 0.0)


def test_centre_tap_is_channel_matmul():
    r = _rng(3)
    x = r.normal(size=(4, 3, 3, 5))
    w = np.zeros((6, 4, 3, 3, 3))
    m = r.normal(size=(6, 4))
    w[:, :, 1, 1, 1] = m
    y = oc.conv3d(x, w)
    np.testing.assert_allclose(y, np.einsum("oc,czyx->ozyx", m, x), rtol=1e-13, atol=1e-13)


def test_conv_adjoints():
    r = _rng(4)
    cin, cout, D, H, W = 3, 5, 4, 6, 5
    x = r.normal(size=(cin, D, H, W))
    w = r.normal(size=(cout, cin, 3, 3, 3))
    g = r.normal(size=(cout, D, H, W))
    # <conv(x), g> = <x, conv^T g>
    lhs = np.vdot(oc.conv3d(x, w), g)
    rhs = np.vdot(x, oc.conv3d_bwd_data(g, w))
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)
    # the convolution is linear in w: <conv(x; w), g> = <w, dW(x, g)>; bias: <b 1, g> = <b, db>
    dw, db = oc.conv3d_bwd_weight(x, g)
    assert abs(lhs - np.vdot(w, dw)) <= 1e-11 * abs(lhs)
    b = r.normal(size=cout)
    assert abs(np.vdot(oc.conv3d(x, w, b) - oc.conv3d(x, w), g) - np.vdot(b, db)) <= 1e-11 * np.abs(b).sum() * np.abs(g).sum()


def test_pool_and_upsample():
    r = _rng(5)
    x = r.normal(size=(2, 4, 6, 8))
    p = oc.pool(x)
    assert p.shape == (2, 2, 3, 4)
    # mean of a constant block is the constant; the mean over the whole volume is kept
    np.testing.assert_allclose(oc.pool(np.full((1, 2, 2, 2), 3.5)), [[[[3.5]]]])
    np.testing.assert_allclose(p.mean(axis=(1, 2, 3)), x.mean(axis=(1, 2, 3)), rtol=1e-13)
    # a brute-force voxel of the pooled volume
    assert abs(p[1, 1, 2, 3] - x[1, 2:4, 4:6, 6:8].sum() / 8) < 1e-14
    u = oc.upsample(p)
    assert u.shape == x.shape and u[0, 3, 5, 7] == p[0, 1, 2, 3]
    # pooling after upsampling gives back the coarse volume
    np.testing.assert_allclose(oc.pool(u), p, rtol=1e-14)
    # adjoints
    gy = r.normal(size=p.shape)
    assert abs(np.vdot(p, gy) - np.vdot(x, oc.pool_bwd(gy))) < 1e-12
    gx = r.normal(size=x.shape)
    assert abs(np.vdot(oc.upsample(gy), gx) - np.vdot(gy, oc.upsample_bwd(gx))) < 1e-12


def test_mse_gradient_finite_difference():
    r = _rng(6)
    y = r.normal(size=(1, 3, 4, 5))
    t = r.normal(size=y.shape)
    loss, g = oc.mse(y, t)
    assert abs(loss - ((y - t) ** 2).sum() / y.size) < 1e-14
    h = 1e-6
    for idx in [(0, 0, 0, 0), (0, 2, 3, 4), (0, 1, 2, 1)]:
        yp, ym = y.copy(), y.copy()
        yp[idx] += h
        ym[idx] -= h
        fd = (oc.mse(yp, t)[0] - oc.mse(ym, t)[0]) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * abs(g[idx])


def test_adam_bias_correction():
    # with a constant gradient the bias-corrected moments are exactly g and
    # g^2 at every step, so every step moves w by lr * g / (|g| + eps)
    r = _rng(7)
    g = r.normal(size=10)
    w = np.zeros(10)
    m = np.zeros(10)
    v = np.zeros(10)
    lr, eps = 1e-2, 1e-8
    for step in range(1, 6):
        w_prev = w
        w, m, v = oc.adam(w, g, m, v, lr, 0.9, 0.999, eps, step)
        np.testing.assert_allclose(w_prev - w, lr * g / (np.abs(g) + eps), rtol=1e-12)
    # the raw moments are the geometric sums of the constant gradient
    np.testing.assert_allclose(m, (1 - 0.9 ** 5) * g, rtol=1e-13)
    np.testing.assert_allclose(v, (1 - 0.999 ** 5) * g * g, rtol=1e-12)


def test_unet_layer_shapes():
    assert oc.unet_layers([16, 32, 64, 64]) == [(1, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64),
                                                (64, 64), (64, 64), (64, 64), (64, 32), (32, 32), (32, 16),
                                                (16, 16), (16, 1)]
    assert oc.unet_layers([4, 8], in_ch=2) == [(2, 4), (4, 4), (4, 8), (8, 4), (4, 4), (4, 1)]


def _loss(params, x, t, ch):
    y, _ = oc.unet_forward(params, x, ch)
    return oc.mse(y, t)[0]


@pytest.mark.parametrize("ch,in_ch", [([2, 3], 1), ([2, 3, 4, 4], 1), ([2, 3, 3], 2)])
def test_unet_gradients_finite_difference(ch, in_ch):
    """Analytic gradients of the whole network against central differences
    (h = 1e-6), relative error <= 1e-6 on every checked component."""
    r = _rng(8)
    params = oc.unet_init(ch, seed=9, in_ch=in_ch)
    # non-zero biases so that every bias gradient path is exercised
    params = [(w, r.normal(0, 0.1, size=b.shape)) for w, b in params]
    x = r.uniform(0.0, 1.5, size=(in_ch, 8, 8, 8))
    t = x[-1:] + r.normal(0, 0.1, size=(1,) + x.shape[1:])
    y, tape = oc.unet_forward(params, x, ch)
    _, dy = oc.mse(y, t)
    grads = oc.unet_backward(params, x, ch, tape, dy)
    h = 1e-6
    checked = 0
    for k, ((w, b), (dw, db)) in enumerate(zip(params, grads)):
        assert dw.shape == w.shape and db.shape == b.shape
        cand = [("w", np.unravel_index(int(np.argmax(np.abs(dw))), w.shape)),
                ("w", tuple(r.integers(0, s) for s in w.shape)), ("b", (int(np.argmax(np.abs(db))),))]
        for which, idx in cand:
            arr, g = (w, dw) if which == "w" else (b, db)
            if abs(g[idx]) < 1e-9:
                continue
            old = arr[idx]
            arr[idx] = old + h
            lp = _loss(params, x, t, ch)
            arr[idx] = old - h
            lm = _loss(params, x, t, ch)
            arr[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[idx]) <= 1e-6 * abs(g[idx]) + 1e-12, (k, which, idx, fd, g[idx])
            checked += 1
    assert checked >= 2 * len(params)


def test_unet_zero_last_layer_is_identity():
    # the network adds its output to the input: a zero last convolution returns the input
    ch = [2, 3, 4]
    params = oc.unet_init(ch, seed=1)
    w, b = params[-1]
    params[-1] = (np.zeros_like(w), np.zeros_like(b))
    x = _rng(10).normal(size=(1, 8, 8, 8))
    y, _ = oc.unet_forward(params, x, ch)
    np.testing.assert_array_equal(y, x)


def test_bf16_round_known_values_and_nearest():
    """bfloat16 keeps 8 significant bits: near 1 its spacing is 2^-7.
    Halfway cases go to the even neighbour; otherwise the nearest neighbour,
    checked against a direct search over the two candidates."""
    h = 2.0 ** -8
    vals = np.array([1.0, 1 + h, 1 + 3 * h, 1 + h + 2.0 ** -20, -(1 + 3 * h), 3.0, 2.0 ** -130, 65504.0])
    want = np.array([1.0, 1.0, 1 + 2 * 2 * h, 1 + 2 * h, -(1 + 4 * h), 3.0, 2.0 ** -130, 65536.0])
    assert np.array_equal(oc.bf16_round(vals), want)
    r = np.random.default_rng(5)
    x = (r.standard_normal(100_000) * np.exp(r.uniform(-20, 20, 100_000))).astype(np.float32)
    got = oc.bf16_round(x)
    u = x.view(np.uint32)
    lo = (u & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)  # truncation toward zero
    step = np.ldexp(1.0, np.frexp(np.abs(lo))[1] - 8)                    # spacing at |lo| (8 significant bits)
    hi = lo + np.sign(x) * step                                          # next bfloat16 away from zero
    d_lo, d_hi = np.abs(x.astype(np.float64) - lo), np.abs(hi - x.astype(np.float64))
    lo_even = ((u >> 16) & 1) == 0
    pick_lo = (d_lo < d_hi) | ((d_lo == d_hi) & lo_even)
    assert np.array_equal(got, np.where(pick_lo, lo, hi))
    # the rounded values are bfloat16 numbers: low 16 bits of their float32 zero
    assert not (got.astype(np.float32).view(np.uint32) & 0xFFFF).any()


def test_bf16_weight_gradient_reading():
    """The matrix-core weight gradient's reading: its operands x and g are
    rounded to bfloat16 where the shape has channel tiles of sixteen, and
    only there.  Inputs that are bfloat16 numbers already (small integers)
    give the exact gradients; a shape the form does not take gives them for
    any input; otherwise the result moves by about the rounding (2^-9
    relative per operand), and the bias gradient never moves."""
    r = _rng(12)
    ints = lambda *sh: r.integers(-8, 9, size=sh).astype(np.float64)
    x, g = ints(16, 3, 4, 5), ints(32, 3, 4, 5)
    exact = oc.conv3d_bwd_weight(x, g)
    got = oc._conv_bwd_weight(x, g, True)
    np.testing.assert_array_equal(got[0], exact[0])
    np.testing.assert_array_equal(got[1], exact[1])
    x8 = r.normal(size=(8, 3, 4, 5))
    g16 = r.normal(size=(16, 3, 4, 5))
    for a, b in zip(oc._conv_bwd_weight(x8, g16, True), oc.conv3d_bwd_weight(x8, g16)):
        np.testing.assert_array_equal(a, b)
    xr, gr = r.normal(size=(16, 3, 4, 5)), r.normal(size=(16, 3, 4, 5))
    (dq, bq), (de, be) = oc._conv_bwd_weight(xr, gr, True), oc.conv3d_bwd_weight(xr, gr)
    np.testing.assert_array_equal(bq, be)
    dabs, _ = oc.conv3d_bwd_weight(np.abs(xr), np.abs(gr))
    err = np.abs(dq - de)
    assert err.max() > 0
    assert np.all(err <= 2 * 2.0 ** -8 * dabs + 1e-12)
