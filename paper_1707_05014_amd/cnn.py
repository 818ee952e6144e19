"""Learned warm start: a small 3D U-Net that maps the image after a few
sweeps to an estimate of the image after many sweeps, used as the initial
guess x0 of the row-action sweeps (the paper leaves x0 open, Sec. 2.1).

Every operation runs in the pct_cnn_* HIP kernels of libpct.so; torch only
supplies device memory and the stream.  Tensors are float32 [C][D][H][W]
(W fastest), one volume at a time.

Network (channels c_0..c_{L-1}, default 16, 32, 64, 64):
  encoder level l: conv(3x3x3) + ReLU, conv + ReLU; 2x2x2 average pooling to
  level l+1; the deepest level's second convolution maps back to c_{L-2};
  decoder level l (L-2 .. 0): nearest 2x upsampling, plus the encoder's level-l
  features, conv + ReLU, conv (+ ReLU, except at level 0, which maps to one
  channel); output = input + network (a learned correction of the image).
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib
from ._lib import check


def _s(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dev(t: torch.Tensor, name: str) -> int:
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 device tensor")
    return int(t.data_ptr())


def _dhw(t: torch.Tensor):
    return int(t.shape[-3]), int(t.shape[-2]), int(t.shape[-1])


# ----------------------------------------------------------- entry points
def bf16_scratch(cin, cout) -> int:
    """Bytes of packed-weight scratch the bfloat16 matrix-core convolution
    needs for (cin, cout); 0 when it does not take that shape (cin % 8 or
    cout % 16 not 0)."""
    return int(_lib.load().pct_cnn_conv3d_bf16_scratch(int(cin), int(cout)))


def _scratch(t: torch.Tensor, nbytes: int, name: str) -> int:
    if not (t.is_cuda and t.is_contiguous()) or t.numel() * t.element_size() < nbytes:
        raise ValueError(f"{name} must be a contiguous device tensor of at least {nbytes} bytes")
    return int(t.data_ptr())


def conv3d(x, w, b, y, stream=None, wpack=None):
    """y = b + w (*) x (3x3x3, zero padding); x [cin][D][H][W], w [cout][cin][3][3][3].
    With wpack (device scratch of bf16_scratch(cin, cout) bytes) the matrix
    cores compute it from bfloat16-rounded x and w, accumulating in FP32."""
    cout, cin = int(w.shape[0]), int(w.shape[1])
    D, H, W = _dhw(x)
    if x.shape != (cin, D, H, W) or y.shape != (cout, D, H, W) or (b is not None and b.numel() != cout):
        raise ValueError("conv3d: shapes do not match")
    bp = None if b is None else _dev(b, "b")
    if wpack is not None:
        check(_lib.load().pct_cnn_conv3d_bf16(_dev(x, "x"), _dev(w, "w"), bp, _dev(y, "y"),
                                              _scratch(wpack, bf16_scratch(cin, cout), "wpack"), cin, cout, D, H, W,
                                              _s(stream)))
    else:
        check(_lib.load().pct_cnn_conv3d(_dev(x, "x"), _dev(w, "w"), bp, _dev(y, "y"), cin, cout, D, H, W, _s(stream)))
    return y


def conv3d_bwd_data(dy, w, dx, wt, stream=None, wpack=None):
    """dx [cin] = adjoint of the convolution applied to dy [cout]; wt: cin*cout*27 floats of scratch.
    With wpack (bf16_scratch(cout, cin) bytes) on the matrix cores, as conv3d."""
    cout, cin = int(w.shape[0]), int(w.shape[1])
    D, H, W = _dhw(dy)
    if dy.shape != (cout, D, H, W) or dx.shape != (cin, D, H, W) or wt.numel() < cin * cout * 27:
        raise ValueError("conv3d_bwd_data: shapes do not match")
    if wpack is not None:
        check(_lib.load().pct_cnn_conv3d_bwd_data_bf16(_dev(dy, "dy"), _dev(w, "w"), _dev(dx, "dx"), _dev(wt, "wt"),
                                                       _scratch(wpack, bf16_scratch(cout, cin), "wpack"), cin, cout,
                                                       D, H, W, _s(stream)))
    else:
        check(_lib.load().pct_cnn_conv3d_bwd_data(_dev(dy, "dy"), _dev(w, "w"), _dev(dx, "dx"), _dev(wt, "wt"), cin,
                                                  cout, D, H, W, _s(stream)))
    return dx


def wgrad_scratch(cin, cout, D, H, W) -> int:
    return int(_lib.load().pct_cnn_wgrad_scratch(cin, cout, D, H, W))


def bf16_wgrad_ok(cin, cout) -> bool:
    """Shapes the matrix-core weight gradient takes."""
    return cin > 0 and cout > 0 and cin % 16 == 0 and cout % 16 == 0


def conv3d_bwd_weight(x, dy, dw, db, scratch, stream=None, bf16=False):
    """dw [cout][cin][27], db [cout] (or None) from the layer input x [cin] and
    dy [cout]; bf16=True: on the matrix cores (operands rounded to bfloat16,
    cin and cout multiples of 16)."""
    cin, cout = int(x.shape[0]), int(dy.shape[0])
    D, H, W = _dhw(x)
    if dy.shape[1:] != x.shape[1:] or dw.numel() != cout * cin * 27 or (db is not None and db.numel() != cout):
        raise ValueError("conv3d_bwd_weight: shapes do not match")
    if scratch.numel() < wgrad_scratch(cin, cout, D, H, W):
        raise ValueError("conv3d_bwd_weight: scratch too small")
    fn = _lib.load().pct_cnn_conv3d_bwd_weight_bf16 if bf16 else _lib.load().pct_cnn_conv3d_bwd_weight
    check(fn(_dev(x, "x"), _dev(dy, "dy"), _dev(dw, "dw"), None if db is None else _dev(db, "db"),
             _dev(scratch, "scratch"), cin, cout, D, H, W, _s(stream)))
    return dw


def relu(x, y, stream=None):
    if x.numel() != y.numel():
        raise ValueError("relu: sizes differ")
    check(_lib.load().pct_cnn_relu(_dev(x, "x"), _dev(y, "y"), x.numel(), _s(stream)))
    return y


def relu_bwd(y, dy, dx, stream=None):
    if not (y.numel() == dy.numel() == dx.numel()):
        raise ValueError("relu_bwd: sizes differ")
    check(_lib.load().pct_cnn_relu_bwd(_dev(y, "y"), _dev(dy, "dy"), _dev(dx, "dx"), y.numel(), _s(stream)))
    return dx


def pool(x, y, stream=None):
    C = int(x.shape[0])
    D, H, W = _dhw(x)
    if y.shape != (C, D // 2, H // 2, W // 2) or D % 2 or H % 2 or W % 2:
        raise ValueError("pool: shapes do not match (D, H, W must be even)")
    check(_lib.load().pct_cnn_pool(_dev(x, "x"), _dev(y, "y"), C, D, H, W, _s(stream)))
    return y


def pool_bwd(dy, dx, stream=None):
    C = int(dx.shape[0])
    D, H, W = _dhw(dx)
    if dy.shape != (C, D // 2, H // 2, W // 2) or D % 2 or H % 2 or W % 2:
        raise ValueError("pool_bwd: shapes do not match")
    check(_lib.load().pct_cnn_pool_bwd(_dev(dy, "dy"), _dev(dx, "dx"), C, D, H, W, _s(stream)))
    return dx


def upsample(x, y, stream=None):
    C = int(x.shape[0])
    d, h, w = _dhw(x)
    if y.shape != (C, 2 * d, 2 * h, 2 * w):
        raise ValueError("upsample: shapes do not match")
    check(_lib.load().pct_cnn_upsample(_dev(x, "x"), _dev(y, "y"), C, d, h, w, _s(stream)))
    return y


def upsample_bwd(dy, dx, stream=None):
    C = int(dx.shape[0])
    d, h, w = _dhw(dx)
    if dy.shape != (C, 2 * d, 2 * h, 2 * w):
        raise ValueError("upsample_bwd: shapes do not match")
    check(_lib.load().pct_cnn_upsample_bwd(_dev(dy, "dy"), _dev(dx, "dx"), C, d, h, w, _s(stream)))
    return dx


def add(a, b, y, stream=None):
    if not (a.numel() == b.numel() == y.numel()):
        raise ValueError("add: sizes differ")
    check(_lib.load().pct_cnn_add(_dev(a, "a"), _dev(b, "b"), _dev(y, "y"), a.numel(), _s(stream)))
    return y


def axpy(a: float, x, y, stream=None):
    """y += a * x."""
    if x.numel() != y.numel():
        raise ValueError("axpy: sizes differ")
    check(_lib.load().pct_cnn_axpy(float(a), _dev(x, "x"), _dev(y, "y"), x.numel(), _s(stream)))
    return y


def mask(x, m, y, stream=None):
    """y = x inside the hull mask m (uint8, same size), 0 outside."""
    if not (x.numel() == m.numel() == y.numel()) or m.dtype != torch.uint8 or not (m.is_cuda and m.is_contiguous()):
        raise ValueError("mask: sizes differ or mask is not a contiguous uint8 device tensor")
    check(_lib.load().pct_cnn_mask(_dev(x, "x"), int(m.data_ptr()), _dev(y, "y"), x.numel(), _s(stream)))
    return y


def mse(y, t, dy=None, scratch=None, loss=None, stream=None):
    """Mean squared error into a device float64 scalar `loss` (returned);
    dy = 2 (y - t) / n when given."""
    n = y.numel()
    if t.numel() != n or (dy is not None and dy.numel() != n):
        raise ValueError("mse: sizes differ")
    lib = _lib.load()
    need = int(lib.pct_cnn_mse_scratch(n))
    if scratch is None:
        scratch = torch.empty(max(need, 1), dtype=torch.float64, device=y.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device=y.device)
    if scratch.dtype != torch.float64 or scratch.numel() < need or loss.dtype != torch.float64:
        raise ValueError("mse: scratch / loss must be float64 device tensors")
    check(lib.pct_cnn_mse(_dev(y, "y"), _dev(t, "t"), None if dy is None else _dev(dy, "dy"), int(scratch.data_ptr()),
                          int(loss.data_ptr()), n, _s(stream)))
    return loss


def adam(w, g, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    n = w.numel()
    if not (g.numel() == m.numel() == v.numel() == n) or step < 1:
        raise ValueError("adam: sizes differ or step < 1")
    check(_lib.load().pct_cnn_adam(_dev(w, "w"), _dev(g, "g"), _dev(m, "m"), _dev(v, "v"), n, float(lr), float(beta1),
                                   float(beta2), float(eps), int(step), _s(stream)))
    return w


# ----------------------------------------------------------- network
def layer_shapes(channels, in_channels=1):
    """(cin, cout) of every convolution in execution order."""
    L = len(channels)
    out = []
    prev = in_channels
    for l, c in enumerate(channels):
        last = channels[L - 2] if (l == L - 1 and L > 1) else c
        out.append((prev, c))
        out.append((c, last))
        prev = c
    for l in range(L - 2, -1, -1):
        out.append((channels[l], channels[l]))
        out.append((channels[l], channels[l - 1] if l > 0 else 1))
    return out


class UNet3D:
    """Parameters live in one flat float32 device buffer (weights then bias
    per layer), so gradients and the Adam moments are single buffers too.
    precision "bf16": the convolutions and their input gradients that the
    matrix-core kernels take (cin % 8 == 0, cout % 16 == 0), and the weight
    gradients they take (cin % 16 == 0, cout % 16 == 0), run there on
    bfloat16-rounded operands with FP32 accumulation; bias gradients,
    activations and parameters stay FP32."""

    def __init__(self, channels=(16, 32, 64, 64), device="cuda", seed: int = 0, in_channels: int = 1,
                 precision: str = "f32"):
        if precision not in ("f32", "bf16"):
            raise ValueError("precision is 'f32' or 'bf16'")
        self.precision = precision
        self._wpack = None
        self.channels = tuple(int(c) for c in channels)
        if len(self.channels) < 2 or min(self.channels) < 1 or in_channels < 1:
            raise ValueError("the network needs at least two levels of positive channel counts")
        self.L = len(self.channels)
        self.in_channels = int(in_channels)
        self.shapes = layer_shapes(self.channels, self.in_channels)
        self.device = torch.device(device)
        sizes = []
        for cin, cout in self.shapes:
            sizes += [cout * cin * 27, cout]
        self.n_params = int(sum(sizes))
        self.flat = torch.zeros(self.n_params, dtype=torch.float32, device=self.device)
        self.grad = torch.zeros_like(self.flat)
        self.m = torch.zeros_like(self.flat)
        self.v = torch.zeros_like(self.flat)
        self.step_count = 0
        self.w, self.b, self.dw, self.db = [], [], [], []
        off = 0
        for cin, cout in self.shapes:
            nw = cout * cin * 27
            self.w.append(self.flat[off:off + nw].view(cout, cin, 3, 3, 3))
            self.dw.append(self.grad[off:off + nw].view(cout, cin, 3, 3, 3))
            off += nw
            self.b.append(self.flat[off:off + cout])
            self.db.append(self.grad[off:off + cout])
            off += cout
        self.init(seed)
        self._tape = None

    # -- parameters
    def init(self, seed: int):
        """He-normal weights (std sqrt(2 / (27 cin))), zero biases; the last
        convolution starts at zero so the untrained network is the identity."""
        rng = np.random.default_rng(seed)
        host = np.zeros(self.n_params, dtype=np.float32)
        off = 0
        for k, (cin, cout) in enumerate(self.shapes):
            nw = cout * cin * 27
            if k < len(self.shapes) - 1:
                host[off:off + nw] = rng.normal(0.0, np.sqrt(2.0 / (27 * cin)), nw)
            off += nw + cout
        self.flat.copy_(torch.from_numpy(host))
        self.m.zero_()
        self.v.zero_()
        self.step_count = 0

    def params_numpy(self):
        """[(w [cout][cin][3][3][3], b [cout]), ...] as float64 host arrays."""
        return [(w.detach().cpu().double().numpy(), b.detach().cpu().double().numpy()) for w, b in zip(self.w, self.b)]

    def load_params(self, params):
        for (w, b), (wd, bd) in zip(params, zip(self.w, self.b)):
            wd.copy_(torch.as_tensor(np.asarray(w), dtype=torch.float32))
            bd.copy_(torch.as_tensor(np.asarray(b), dtype=torch.float32))

    def save(self, path: str):
        np.savez(path, channels=np.array(self.channels), in_channels=np.array(self.in_channels),
                 flat=self.flat.cpu().numpy(), m=self.m.cpu().numpy(), v=self.v.cpu().numpy(),
                 step=np.array(self.step_count))

    @classmethod
    def load(cls, path: str, device="cuda") -> "UNet3D":
        z = np.load(path)
        net = cls(tuple(int(c) for c in z["channels"]), device=device, in_channels=int(z["in_channels"]))
        net.flat.copy_(torch.from_numpy(z["flat"]))
        net.m.copy_(torch.from_numpy(z["m"]))
        net.v.copy_(torch.from_numpy(z["v"]))
        net.step_count = int(z["step"])
        return net

    # -- passes
    def _check_input(self, x):
        if x.dim() != 4 or x.shape[0] != self.in_channels:
            raise ValueError(f"input must be [{self.in_channels}][D][H][W]")
        f = 1 << (self.L - 1)
        if any(int(s) % f for s in x.shape[1:]):
            raise ValueError(f"D, H, W must be multiples of {f}")
        _dev(x, "x")

    def _empty(self, c, dhw):
        return torch.empty((c,) + tuple(dhw), dtype=torch.float32, device=self.device)

    def _pack(self, cin, cout):
        """Packed-weight scratch for a matrix-core convolution of (cin, cout),
        or None (FP32 kernels) in FP32 precision or for a shape they do not take."""
        if self.precision != "bf16" or bf16_scratch(cin, cout) == 0:
            return None
        if self._wpack is None:
            need = max([bf16_scratch(ci, co) for ci, co in self.shapes] +
                       [bf16_scratch(co, ci) for ci, co in self.shapes])
            self._wpack = torch.empty(max(need, 1), dtype=torch.uint8, device=self.device)
        return self._wpack

    def forward(self, x: torch.Tensor, keep: bool = False, stream=None) -> torch.Tensor:
        """Output [1][D][H][W] = last input channel + network; with keep=True
        the activations are kept for backward()."""
        self._check_input(x)
        k = 0
        h = x
        dims = tuple(int(s) for s in x.shape[1:])
        enc = []
        for l in range(self.L):
            c1 = self.shapes[k][1]
            z1 = self._empty(c1, dims)
            conv3d(h, self.w[k], self.b[k], z1, stream, wpack=self._pack(*self.shapes[k]))
            relu(z1, z1, stream)
            c2 = self.shapes[k + 1][1]
            z2 = self._empty(c2, dims)
            conv3d(z1, self.w[k + 1], self.b[k + 1], z2, stream, wpack=self._pack(*self.shapes[k + 1]))
            relu(z2, z2, stream)
            enc.append((h, z1, z2))
            k += 2
            if l < self.L - 1:
                dims = tuple(d // 2 for d in dims)
                p = self._empty(c2, dims)
                pool(z2, p, stream)
                h = p
            else:
                h = z2
        dec = []
        for l in range(self.L - 2, -1, -1):
            skip = enc[l][2]
            dims = tuple(int(s) for s in skip.shape[1:])
            s = self._empty(int(skip.shape[0]), dims)
            upsample(h, s, stream)
            add(s, skip, s, stream)
            c1 = self.shapes[k][1]
            z1 = self._empty(c1, dims)
            conv3d(s, self.w[k], self.b[k], z1, stream, wpack=self._pack(*self.shapes[k]))
            relu(z1, z1, stream)
            c2 = self.shapes[k + 1][1]
            z2 = self._empty(c2, dims)
            conv3d(z1, self.w[k + 1], self.b[k + 1], z2, stream, wpack=self._pack(*self.shapes[k + 1]))
            if l > 0:
                relu(z2, z2, stream)
            dec.append((s, z1, z2))
            k += 2
            h = z2
        out = self._empty(1, dims)
        add(x[self.in_channels - 1:], h, out, stream)
        self._tape = (enc, dec) if keep else None
        return out

    def backward(self, dout: torch.Tensor, stream=None):
        """Gradients of every parameter into self.grad, given dL/d(output)."""
        if self._tape is None:
            raise RuntimeError("backward() needs forward(..., keep=True) first")
        enc, dec = self._tape
        maxw = max(cin * cout for cin, cout in self.shapes) * 27
        wt = torch.empty(maxw, dtype=torch.float32, device=self.device)
        full = tuple(int(s) for s in dout.shape[1:])
        maxs = max(wgrad_scratch(cin, cout, *full) for cin, cout in self.shapes)
        scratch = torch.empty(max(maxs, 1), dtype=torch.float32, device=self.device)

        def conv_back(k, inp, act, g, relu_out):
            # g: gradient of the layer's output (after its ReLU when relu_out);
            # returns the gradient of its input (none for the first layer)
            cin, cout = self.shapes[k]
            if relu_out:
                relu_bwd(act, g, g, stream)
            conv3d_bwd_weight(inp, g, self.dw[k], self.db[k], scratch, stream,
                              bf16=self.precision == "bf16" and bf16_wgrad_ok(cin, cout))
            if k == 0:
                return None
            gi = self._empty(cin, tuple(int(s) for s in inp.shape[1:]))
            conv3d_bwd_data(g, self.w[k], gi, wt, stream, wpack=self._pack(cout, cin))
            return gi

        k = len(self.shapes)
        g = dout.clone()  # the ReLU gradients are applied in place
        dskip = [None] * self.L
        for i, l in enumerate(range(0, self.L - 1)):
            s, z1, z2 = dec[len(dec) - 1 - i]
            k -= 2
            g1 = conv_back(k + 1, z1, z2, g, relu_out=l > 0)
            gs = conv_back(k, s, z1, g1, relu_out=True)
            dskip[l] = gs
            # gradient of the deeper level's output (the upsampled tensor)
            coarse = tuple(int(q) for q in enc[l + 1][2].shape[1:])
            gd = self._empty(int(gs.shape[0]), coarse)
            upsample_bwd(gs, gd, stream)
            g = gd
        for l in range(self.L - 1, -1, -1):
            h, z1, z2 = enc[l]
            if l < self.L - 1:
                gp = self._empty(int(z2.shape[0]), tuple(int(q) for q in z2.shape[1:]))
                pool_bwd(g, gp, stream)
                add(gp, dskip[l], gp, stream)
                g = gp
            k -= 2
            g1 = conv_back(k + 1, z1, z2, g, relu_out=True)
            g = conv_back(k, h, z1, g1, relu_out=True)
        assert k == 0
        return self.grad

    def loss_and_grad(self, x, target, coarse_weight: float = 0.0, stream=None) -> torch.Tensor:
        """Forward, loss against target and backward; returns MSE(y, t)
        (device float64 [1]).  The gradient is that of
        MSE(y, t) + coarse_weight * MSE(P(y), P(t))
        with P = two 2x2x2 average poolings (4x4x4 block means): the coarse
        term weighs the slowly converging low-frequency part of the error,
        which voxel noise in the target hides from the plain MSE."""
        y = self.forward(x, keep=True, stream=stream)
        dy = torch.empty_like(y)
        loss = mse(y, target, dy, stream=stream)
        if coarse_weight > 0.0:
            dims = [tuple(int(s) for s in y.shape[1:])]
            for _ in range(2):
                dims.append(tuple(d // 2 for d in dims[-1]))
            if any(d % 4 for d in dims[0]):
                raise ValueError("the coarse loss needs D, H, W divisible by 4")
            yc, tc = y, target
            for k in (1, 2):
                yc = pool(yc, self._empty(1, dims[k]), stream)
                tc = pool(tc, self._empty(1, dims[k]), stream)
            gc = self._empty(1, dims[2])
            mse(yc, tc, gc, stream=stream)
            # d/dy of w * MSE(P(y), P(t)): the coarse gradient spread back by the pooling adjoints
            g1 = pool_bwd(gc, self._empty(1, dims[1]), stream)
            g0 = pool_bwd(g1, self._empty(1, dims[0]), stream)
            axpy(float(coarse_weight), g0, dy, stream)
        self.backward(dy, stream)
        self._tape = None
        return loss

    def adam_step(self, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self.step_count += 1
        adam(self.flat, self.grad, self.m, self.v, lr, self.step_count, beta1, beta2, eps, stream)

    def train_step(self, x, target, lr: float, stream=None) -> torch.Tensor:
        loss = self.loss_and_grad(x, target, stream=stream)
        self.adam_step(lr, stream=stream)
        return loss

    def predict(self, x, stream=None) -> torch.Tensor:
        return self.forward(x, keep=False, stream=stream)
