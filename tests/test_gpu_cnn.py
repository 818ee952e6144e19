"""Warm-start network kernels (pct_cnn_*) against the FP64 oracle (oracle.cnn).

Tolerances (FP32 storage and accumulation against FP64):
* normwise: ||gpu - oracle|| / ||oracle|| <= 1e-5 for every single operation;
* elementwise, for sums: |gpu - oracle| <= 3e-5 * (the same operation on the
  absolute values of its operands), the usual bound for a floating-point sum
  with sqrt(n) growth of the rounding error (n <= 64 * 27 terms here) and a
  margin of about 4 standard deviations;
* the whole network: output normwise <= 1e-5, every parameter gradient
  normwise <= 1e-4 (fourteen layers of FP32 rounding composed, and ReLU
  decisions on activations within rounding of zero may differ).
Shapes are ragged on purpose: voxel counts that are not multiples of the
256-thread workgroup, extents that leave partial weight-gradient tiles
(64 voxels along W x 16 rows x 16 planes), output channel counts that leave
partial channel blocks (1, 6, 17), and a volume one voxel thick.

The matrix-core (bfloat16) convolution is checked against the oracle applied
to the same operands rounded to bfloat16: products of bfloat16 values are
exact in FP32, so the same FP32-sum bounds apply.  Its shapes leave partial
16 x 4 x 2 voxel tiles along every axis, a last pass over fewer than 32
input channels (40 = 32 + 8), and one, two and four 16-channel output tiles
per workgroup.  The matrix-core weight gradient (32 x 4 x 2 voxel tiles,
16 x 16 channel tiles) is checked the same way, on shapes that leave
partial tiles along every axis, one to four channel tiles each way and a
volume one voxel thick; its bias gradient sums the unrounded dy.  A whole
network in bfloat16 cannot follow the oracle's
bfloat16 network bit for bit: the two round activations that differ in their
last FP32 bits, a rounding that lands on the other neighbour moves that
value by 2^-8, and the layers after it then round differently too.  So the
network is checked by its distance to the exact (FP64, unrounded) oracle
network: the bfloat16 network on the GPU must be no farther from it than
twice the oracle's own bfloat16-rounded network (plus 1e-4), output
correction and every parameter gradient normwise.  (The oracle's own
bfloat16 network is ~6e-3 from the exact one in its output correction and up
to ~4e-2 in the gradients of the deepest layers, whose gradients are small;
a wrong operand or index would put the GPU at O(1).)
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import cnn as oc  # noqa: E402
from paper_1707_05014_amd import _lib, cnn  # noqa: E402

NORM_TOL = 1e-5
ELEM_TOL = 3e-5
NET_GRAD_TOL = 1e-4


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().double().numpy()


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _check(got, ref, absref=None, tol=NORM_TOL, what=""):
    err = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)
    assert err <= tol, f"{what}: normwise error {err:.3e}"
    if absref is not None:
        bad = np.abs(got - ref) > ELEM_TOL * absref + 1e-30
        assert not bad.any(), f"{what}: {bad.sum()} elements outside the elementwise bound"


SHAPES = [(3, 1, 5, 7, 9), (3, 6, 17, 19, 13), (2, 17, 1, 9, 33), (16, 16, 8, 40, 40), (2, 5, 3, 18, 70)]


@pytest.mark.parametrize("shape", SHAPES)
def test_conv3d_forward(shape):
    cin, cout, D, H, W = shape
    _say(f"conv3d forward {shape}")
    r = np.random.default_rng(11)
    x, w, b = _f32(r.normal(size=(cin, D, H, W))), _f32(r.normal(size=(cout, cin, 3, 3, 3))), _f32(r.normal(size=cout))
    y = torch.empty((cout, D, H, W), dtype=torch.float32, device="cuda")
    cnn.conv3d(_dev(x), _dev(w), _dev(b), y)
    _check(_host(y), oc.conv3d(x, w, b), oc.conv3d(np.abs(x), np.abs(w), np.abs(b)), what="conv3d")
    # no bias
    cnn.conv3d(_dev(x), _dev(w), None, y)
    _check(_host(y), oc.conv3d(x, w), oc.conv3d(np.abs(x), np.abs(w)), what="conv3d (no bias)")


@pytest.mark.parametrize("shape", SHAPES)
def test_conv3d_backward_data(shape):
    cin, cout, D, H, W = shape
    _say(f"conv3d backward data {shape}")
    r = np.random.default_rng(12)
    g, w = _f32(r.normal(size=(cout, D, H, W))), _f32(r.normal(size=(cout, cin, 3, 3, 3)))
    dx = torch.empty((cin, D, H, W), dtype=torch.float32, device="cuda")
    wt = torch.empty(cin * cout * 27, dtype=torch.float32, device="cuda")
    cnn.conv3d_bwd_data(_dev(g), _dev(w), dx, wt)
    _check(_host(dx), oc.conv3d_bwd_data(g, w), oc.conv3d_bwd_data(np.abs(g), np.abs(w)), what="bwd data")


@pytest.mark.parametrize("shape", SHAPES)
def test_conv3d_backward_weight(shape):
    cin, cout, D, H, W = shape
    _say(f"conv3d backward weight {shape}")
    r = np.random.default_rng(13)
    x, g = _f32(r.normal(size=(cin, D, H, W))), _f32(r.normal(size=(cout, D, H, W)))
    dw = torch.empty((cout, cin, 3, 3, 3), dtype=torch.float32, device="cuda")
    db = torch.empty(cout, dtype=torch.float32, device="cuda")
    scratch = torch.empty(cnn.wgrad_scratch(cin, cout, D, H, W), dtype=torch.float32, device="cuda")
    cnn.conv3d_bwd_weight(_dev(x), _dev(g), dw, db, scratch)
    rw, rb = oc.conv3d_bwd_weight(x, g)
    aw, ab = oc.conv3d_bwd_weight(np.abs(x), np.abs(g))
    _check(_host(dw), rw, aw, what="dw")
    _check(_host(db), rb, ab, what="db")
    # a second call gives the same bits (fixed summation order)
    dw2 = torch.empty_like(dw)
    cnn.conv3d_bwd_weight(_dev(x), _dev(g), dw2, None, scratch)
    assert torch.equal(dw, dw2)


def test_elementwise_ops():
    _say("relu / add / mask / pool / upsample")
    r = np.random.default_rng(14)
    n = 100_003
    a, b = _f32(r.normal(size=n)), _f32(r.normal(size=n))
    ta, tb = _dev(a), _dev(b)
    y = torch.empty_like(ta)
    assert np.array_equal(_host(cnn.relu(ta, y)), oc.relu(a))
    dx = torch.empty_like(ta)
    relu_out = _f32(oc.relu(a))
    assert np.array_equal(_host(cnn.relu_bwd(_dev(relu_out), tb, dx)), oc.relu_bwd(relu_out, b))
    assert np.array_equal(_host(cnn.add(ta, tb, y)), _f32(a + b))
    z = ta.clone()
    _check(_host(cnn.axpy(-0.37, tb, z)), a + float(np.float32(-0.37)) * b, what="axpy")
    m = (r.random(n) < 0.4).astype(np.uint8)
    assert np.array_equal(_host(cnn.mask(ta, torch.from_numpy(m).cuda(), y)), np.where(m != 0, a, 0.0))
    # in place
    z = ta.clone()
    cnn.relu(z, z)
    assert np.array_equal(_host(z), oc.relu(a))
    for (C, D, H, W) in [(3, 6, 10, 14), (1, 2, 2, 2), (5, 8, 40, 50)]:
        x = _f32(r.normal(size=(C, D, H, W)))
        p = torch.empty((C, D // 2, H // 2, W // 2), dtype=torch.float32, device="cuda")
        _check(_host(cnn.pool(_dev(x), p)), oc.pool(x), oc.pool(np.abs(x)), what="pool")
        gp = _f32(r.normal(size=p.shape))
        gx = torch.empty((C, D, H, W), dtype=torch.float32, device="cuda")
        _check(_host(cnn.pool_bwd(_dev(gp), gx)), oc.pool_bwd(gp), what="pool bwd")
        u = torch.empty((C, D, H, W), dtype=torch.float32, device="cuda")
        assert np.array_equal(_host(cnn.upsample(_dev(gp), u)), oc.upsample(gp))
        gu = torch.empty_like(p)
        _check(_host(cnn.upsample_bwd(_dev(x), gu)), oc.upsample_bwd(x), oc.upsample_bwd(np.abs(x)),
               what="upsample bwd")


def test_mse_and_adam():
    _say("mse / adam")
    r = np.random.default_rng(15)
    n = 100_003
    y, t = _f32(r.normal(size=n)), _f32(r.normal(size=n))
    dy = torch.empty(n, dtype=torch.float32, device="cuda")
    loss = cnn.mse(_dev(y), _dev(t), dy)
    ref_loss, ref_dy = oc.mse(y, t)
    assert abs(float(loss.item()) - ref_loss) <= 3e-7 * ref_loss  # e = y - t rounds once in FP32
    _check(_host(dy), ref_dy, what="mse gradient")
    # Adam: five steps with changing gradients against the FP64 recursion
    nw = 10_007
    w = _f32(r.normal(size=nw))
    tw, tm, tv = _dev(w), torch.zeros(nw, dtype=torch.float32, device="cuda"), torch.zeros(nw, dtype=torch.float32,
                                                                                              device="cuda")
    rw, rm, rv = w.copy(), np.zeros(nw), np.zeros(nw)
    for step in range(1, 6):
        g = _f32(r.normal(size=nw))
        cnn.adam(tw, _dev(g), tm, tv, 1e-3, step)
        # the ABI takes the hyper-parameters as float32: the oracle gets the same values
        rw, rm, rv = oc.adam(rw, g, rm, rv, *(float(np.float32(q)) for q in (1e-3, 0.9, 0.999, 1e-8)), step)
    _check(_host(tm), rm, what="adam m")
    _check(_host(tv), rv, what="adam v")
    # the weights move by ~lr per step: compare the total displacement
    _check(_host(tw) - w, rw - w, tol=1e-4, what="adam w")


@pytest.mark.parametrize("channels,dims,in_ch", [([4, 8, 8], (8, 12, 16), 1), ([16, 32, 64, 64], (8, 16, 24), 1),
                                                 ([4, 8, 8], (4, 12, 72), 2)])
def test_network_forward_backward(channels, dims, in_ch):
    _say(f"network {channels} on {dims}, {in_ch} input channels")
    net = cnn.UNet3D(channels, seed=0, in_channels=in_ch)
    params = oc.unet_init(channels, seed=21, in_ch=in_ch)
    r = np.random.default_rng(22)
    params = [(_f32(w), _f32(r.normal(0, 0.05, size=b.shape))) for w, b in params]
    net.load_params(params)
    x = _f32(r.uniform(0.0, 1.8, size=(in_ch,) + dims))
    t = _f32(x[-1:] + r.normal(0, 0.1, size=(1,) + dims))
    y_ref, tape = oc.unet_forward(params, x, channels)
    y = net.forward(_dev(x), keep=True)
    _check(_host(y), y_ref, what="network output")
    _, dy_ref = oc.mse(y_ref, t)
    grads = oc.unet_backward(params, x, channels, tape, dy_ref)
    net.backward(_dev(dy_ref))
    for k, ((dw, db), gw, gb) in enumerate(zip(grads, net.dw, net.db)):
        _check(_host(gw), dw, tol=NET_GRAD_TOL, what=f"layer {k} dw")
        _check(_host(gb), db, tol=NET_GRAD_TOL, what=f"layer {k} db")


def test_training_reduces_loss():
    _say("training on a smoothing task")
    r = np.random.default_rng(23)
    net = cnn.UNet3D([8, 16], seed=1)
    xs, ts = [], []
    for _ in range(4):
        x = _f32(r.uniform(0, 1, size=(1, 8, 16, 16)))
        xs.append(_dev(x))
        ts.append(_dev(oc.pool_bwd(oc.pool(x)) * 8.0))  # 2x2x2 block means: a learnable local filter
    first = [float(net.loss_and_grad(xx, tt).item()) for xx, tt in zip(xs, ts)]
    for step in range(60):
        net.train_step(xs[step % 4], ts[step % 4], lr=3e-3)
    last = [float(net.loss_and_grad(xx, tt).item()) for xx, tt in zip(xs, ts)]
    assert np.mean(last) < 0.5 * np.mean(first), (first, last)


def test_coarse_loss_gradient():
    """The coarse term's gradient (two poolings, MSE, two pooling adjoints,
    axpy) against the oracle composition of the same definitions."""
    _say("coarse loss gradient")
    r = np.random.default_rng(24)
    channels, dims = [4, 8], (8, 8, 12)
    net = cnn.UNet3D(channels, seed=0)
    params = oc.unet_init(channels, seed=25)
    params = [(_f32(w), _f32(r.normal(0, 0.05, size=b.shape))) for w, b in params]
    net.load_params(params)
    x = _f32(r.uniform(0.0, 1.8, size=(1,) + dims))
    t = _f32(x + r.normal(0, 0.1, size=x.shape))
    wc = 3.0
    y_ref, tape = oc.unet_forward(params, x, channels)
    _, g = oc.mse(y_ref, t)
    _, gc = oc.mse(oc.pool(oc.pool(y_ref)), oc.pool(oc.pool(t)))
    g = g + wc * oc.pool_bwd(oc.pool_bwd(gc))
    grads = oc.unet_backward(params, x, channels, tape, g)
    net.loss_and_grad(_dev(x), _dev(t), coarse_weight=wc)
    for k, ((dw, db), gw, gb) in enumerate(zip(grads, net.dw, net.db)):
        _check(_host(gw), dw, tol=NET_GRAD_TOL, what=f"layer {k} dw")
        _check(_host(gb), db, tol=NET_GRAD_TOL, what=f"layer {k} db")


BF16_SHAPES = [(8, 16, 5, 7, 9), (16, 32, 3, 18, 70), (64, 64, 6, 20, 20), (32, 16, 2, 9, 33), (40, 48, 4, 5, 17)]


@pytest.mark.parametrize("shape", BF16_SHAPES)
def test_conv3d_bf16_forward_and_backward_data(shape):
    cin, cout, D, H, W = shape
    _say(f"bf16 conv3d {shape}")
    r = np.random.default_rng(31)
    x, w, b = _f32(r.normal(size=(cin, D, H, W))), _f32(r.normal(size=(cout, cin, 3, 3, 3))), _f32(r.normal(size=cout))
    xq, wq = oc.bf16_round(x), oc.bf16_round(w)
    y = torch.empty((cout, D, H, W), dtype=torch.float32, device="cuda")
    wp = torch.empty(cnn.bf16_scratch(cin, cout), dtype=torch.uint8, device="cuda")
    cnn.conv3d(_dev(x), _dev(w), _dev(b), y, wpack=wp)
    _check(_host(y), oc.conv3d(xq, wq, b), oc.conv3d(np.abs(xq), np.abs(wq), np.abs(b)), what="bf16 conv3d")
    cnn.conv3d(_dev(x), _dev(w), None, y, wpack=wp)
    _check(_host(y), oc.conv3d(xq, wq), oc.conv3d(np.abs(xq), np.abs(wq)), what="bf16 conv3d (no bias)")
    # it is not the FP32 result: the roundings are there
    y32 = torch.empty_like(y)
    cnn.conv3d(_dev(x), _dev(w), None, y32)
    assert not torch.equal(y, y32)
    # input gradient (a convolution from cout to cin channels) where that shape is taken
    if cnn.bf16_scratch(cout, cin):
        g = _f32(r.normal(size=(cout, D, H, W)))
        gq = oc.bf16_round(g)
        dx = torch.empty((cin, D, H, W), dtype=torch.float32, device="cuda")
        wt = torch.empty(cin * cout * 27, dtype=torch.float32, device="cuda")
        wp2 = torch.empty(cnn.bf16_scratch(cout, cin), dtype=torch.uint8, device="cuda")
        cnn.conv3d_bwd_data(_dev(g), _dev(w), dx, wt, wpack=wp2)
        _check(_host(dx), oc.conv3d_bwd_data(gq, wq), oc.conv3d_bwd_data(np.abs(gq), np.abs(wq)),
               what="bf16 bwd data")


def test_conv3d_bf16_rejects_shapes():
    _say("bf16 conv3d shape checks")
    x = torch.zeros((12, 4, 4, 4), dtype=torch.float32, device="cuda")
    w = torch.zeros((16, 12, 3, 3, 3), dtype=torch.float32, device="cuda")
    y = torch.empty((16, 4, 4, 4), dtype=torch.float32, device="cuda")
    wp = torch.empty(1 << 16, dtype=torch.uint8, device="cuda")
    assert cnn.bf16_scratch(12, 16) == 0 and cnn.bf16_scratch(16, 24) == 0
    with pytest.raises(_lib.PctError) as ei:
        cnn.conv3d(x, w, None, y, wpack=wp)
    assert ei.value.code == _lib.PCT_EINVAL


BF16_WGRAD_SHAPES = [(16, 16, 5, 7, 9), (16, 32, 3, 18, 70), (64, 64, 6, 20, 20), (32, 16, 2, 9, 33),
                     (48, 32, 4, 5, 17), (16, 16, 1, 4, 200)]


@pytest.mark.parametrize("shape", BF16_WGRAD_SHAPES)
def test_conv3d_bf16_backward_weight(shape):
    cin, cout, D, H, W = shape
    _say(f"bf16 conv3d backward weight {shape}")
    r = np.random.default_rng(33)
    x, g = _f32(r.normal(size=(cin, D, H, W))), _f32(r.normal(size=(cout, D, H, W)))
    xq, gq = oc.bf16_round(x), oc.bf16_round(g)
    dw = torch.empty((cout, cin, 3, 3, 3), dtype=torch.float32, device="cuda")
    db = torch.empty(cout, dtype=torch.float32, device="cuda")
    scratch = torch.empty(cnn.wgrad_scratch(cin, cout, D, H, W), dtype=torch.float32, device="cuda")
    cnn.conv3d_bwd_weight(_dev(x), _dev(g), dw, db, scratch, bf16=True)
    rw, _ = oc.conv3d_bwd_weight(xq, gq)
    aw, _ = oc.conv3d_bwd_weight(np.abs(xq), np.abs(gq))
    _check(_host(dw), rw, aw, what="bf16 dw")
    _check(_host(db), g.sum(axis=(1, 2, 3)), np.abs(g).sum(axis=(1, 2, 3)), what="bf16 db")
    # the roundings are there: not the FP32 result
    dw32 = torch.empty_like(dw)
    cnn.conv3d_bwd_weight(_dev(x), _dev(g), dw32, None, scratch)
    assert not torch.equal(dw, dw32)
    # a second call gives the same bits (fixed summation order)
    dw2 = torch.empty_like(dw)
    cnn.conv3d_bwd_weight(_dev(x), _dev(g), dw2, None, scratch, bf16=True)
    assert torch.equal(dw, dw2)


def test_conv3d_bf16_backward_weight_rejects_shapes():
    _say("bf16 weight gradient shape checks")
    x = torch.zeros((8, 4, 4, 4), dtype=torch.float32, device="cuda")
    g = torch.zeros((16, 4, 4, 4), dtype=torch.float32, device="cuda")
    dw = torch.empty((16, 8, 3, 3, 3), dtype=torch.float32, device="cuda")
    scratch = torch.empty(cnn.wgrad_scratch(8, 16, 4, 4, 4), dtype=torch.float32, device="cuda")
    assert not cnn.bf16_wgrad_ok(8, 16) and not cnn.bf16_wgrad_ok(16, 24) and cnn.bf16_wgrad_ok(32, 48)
    with pytest.raises(_lib.PctError) as ei:
        cnn.conv3d_bwd_weight(x, g, dw, None, scratch, bf16=True)
    assert ei.value.code == _lib.PCT_EINVAL


def _rel_err(a, ref):
    return float(np.linalg.norm(a - ref) / max(np.linalg.norm(ref), 1e-300))


@pytest.mark.parametrize("channels,dims", [([16, 32, 64, 64], (8, 16, 24)), ([16, 32], (6, 10, 34))])
def test_network_bf16_forward_backward(channels, dims):
    _say(f"bf16 network {channels} on {dims}")
    net = cnn.UNet3D(channels, seed=0, precision="bf16")
    params = oc.unet_init(channels, seed=41)
    r = np.random.default_rng(42)
    params = [(_f32(w), _f32(r.normal(0, 0.05, size=b.shape))) for w, b in params]
    net.load_params(params)
    x = _f32(r.uniform(0.0, 1.8, size=(1,) + dims))
    t = _f32(x + r.normal(0, 0.1, size=(1,) + dims))
    y64, tape64 = oc.unet_forward(params, x, channels)
    yq, tapeq = oc.unet_forward(params, x, channels, bf16=True)
    y = _host(net.forward(_dev(x), keep=True))
    e_ref, e_gpu = _rel_err(yq - x, y64 - x), _rel_err(y - x, y64 - x)
    _say(f"  output correction vs exact: oracle bf16 {e_ref:.2e}, GPU bf16 {e_gpu:.2e}, "
         f"GPU vs oracle bf16 {_rel_err(y - x, yq - x):.2e}")
    assert e_gpu <= 2 * e_ref + 1e-4
    _, dy = oc.mse(y64, t)
    g64 = oc.unet_backward(params, x, channels, tape64, dy)
    gq = oc.unet_backward(params, x, channels, tapeq, dy, bf16=True)
    net.backward(_dev(dy))
    worst = 0.0
    for k, ((dw, db), (qw, qb), gw, gb) in enumerate(zip(g64, gq, net.dw, net.db)):
        for got, q, ref, what in ((_host(gw), qw, dw, "dw"), (_host(gb), qb, db, "db")):
            er, eg = _rel_err(q, ref), _rel_err(got, ref)
            worst = max(worst, eg)
            assert eg <= 2 * er + 1e-4, f"layer {k} {what}: GPU {eg:.2e}, oracle bf16 {er:.2e}"
    _say(f"  worst parameter-gradient error vs exact: {worst:.2e}")
