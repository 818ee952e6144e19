"""FP64 NumPy oracle of the warm-start network.

TEST INFRASTRUCTURE ONLY: the tests and the smoke check use it; the product
path never imports or calls it.  The paper leaves the initial guess x0 of the
row-action sweeps open (Sec. 2.1); the learned warm start that fills it is an
addition, so this module follows the textbook definitions below, not the paper.

Plain, slow, written from the definitions: 3x3x3 cross-correlation with zero
padding over [C][D][H][W] volumes, its adjoints, ReLU, 2x2x2 average pooling,
nearest 2x upsampling, mean squared error, Adam (Kingma & Ba 2015) and the
small 3D U-Net built from them (encoder: two convolutions + ReLU per level,
average pooling between levels; decoder: nearest upsampling, addition of the
encoder's features of that level, two convolutions; output = input + net).
Nothing here is shared with the HIP library; the tests compare the two.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _shift(x, dz, dy, dx):
    """x shifted so that out[z, y, x] = x[z + dz, y + dy, x + dx] (zero outside)."""
    D, H, W = x.shape[-3:]
    out = np.zeros_like(x)
    zs, ys, xs = slice(max(0, -dz), min(D, D - dz)), slice(max(0, -dy), min(H, H - dy)), slice(max(0, -dx), min(W, W - dx))
    zt, yt, xt = slice(max(0, dz), min(D, D + dz)), slice(max(0, dy), min(H, H + dy)), slice(max(0, dx), min(W, W + dx))
    out[..., zs, ys, xs] = x[..., zt, yt, xt]
    return out


def conv3d(x, w, b=None):
    """y[co] = b[co] + sum_ci sum_taps w[co, ci, tz, ty, tx] x[ci, z+tz-1, y+ty-1, x+tx-1]."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    cout = w.shape[0]
    y = np.zeros((cout,) + x.shape[1:])
    for t, (dz, dy, dx) in enumerate(TAPS):
        xs = _shift(x, dz, dy, dx)  # [cin][D][H][W]
        wt = w.reshape(cout, w.shape[1], 27)[:, :, t]  # [cout][cin]
        y += np.tensordot(wt, xs, axes=([1], [0]))
    if b is not None:
        y += np.asarray(b, np.float64)[:, None, None, None]
    return y


def conv3d_bwd_data(dy, w):
    """dx = conv3d^T(dy): dx[ci] = sum_co sum_taps w[co, ci, t] dy[co] shifted by -t."""
    dy = np.asarray(dy, np.float64)
    w = np.asarray(w, np.float64)
    cin = w.shape[1]
    dx = np.zeros((cin,) + dy.shape[1:])
    for t, (dz, ddy, ddx) in enumerate(TAPS):
        gs = _shift(dy, -dz, -ddy, -ddx)
        wt = w.reshape(w.shape[0], cin, 27)[:, :, t]  # [cout][cin]
        dx += np.tensordot(wt.T, gs, axes=([1], [0]))
    return dx


def conv3d_bwd_weight(x, dy):
    """dw[co, ci, t] = sum_p dy[co, p] x[ci, p + t]; db[co] = sum_p dy[co, p]."""
    x = np.asarray(x, np.float64)
    dy = np.asarray(dy, np.float64)
    cout, cin = dy.shape[0], x.shape[0]
    dw = np.zeros((cout, cin, 27))
    for t, (dz, ddy, ddx) in enumerate(TAPS):
        xs = _shift(x, dz, ddy, ddx)
        dw[:, :, t] = np.tensordot(dy, xs, axes=([1, 2, 3], [1, 2, 3]))
    return dw.reshape(cout, cin, 3, 3, 3), dy.sum(axis=(1, 2, 3))


def relu(x):
    return np.maximum(x, 0.0)


def relu_bwd(y, dy):
    return np.where(y > 0, dy, 0.0)


def pool(x):
    C, D, H, W = x.shape
    return x.reshape(C, D // 2, 2, H // 2, 2, W // 2, 2).mean(axis=(2, 4, 6))


def pool_bwd(dy):
    return upsample(dy) / 8.0


def upsample(x):
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)


def upsample_bwd(dy):
    C, D, H, W = dy.shape
    return dy.reshape(C, D // 2, 2, H // 2, 2, W // 2, 2).sum(axis=(2, 4, 6))


def mse(y, t):
    e = np.asarray(y, np.float64) - np.asarray(t, np.float64)
    return float(np.mean(e * e)), 2.0 * e / e.size


def adam(w, g, m, v, lr, b1, b2, eps, step):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------- network
def bf16_round(a):
    """a rounded to float32, then to bfloat16 (round to nearest, ties to even:
    the high 16 bits of the float32 after adding 0x7fff plus the lowest kept
    bit), returned as float64.  The matrix-core form of the convolution takes
    its operands at this precision (finite values only here)."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def mfma_forward_ok(cin, cout):
    """Shapes the matrix-core convolution takes (input channels in groups of
    eight, output channels in tiles of sixteen)."""
    return cin % 8 == 0 and cout % 16 == 0


def mfma_wgrad_ok(cin, cout):
    """Shapes the matrix-core weight gradient takes (input and output
    channels in tiles of sixteen)."""
    return cin % 16 == 0 and cout % 16 == 0


def _conv(x, w, b, bf16):
    cout, cin = w.shape[0], w.shape[1]
    if bf16 and mfma_forward_ok(cin, cout):
        return conv3d(bf16_round(x), bf16_round(w), b)
    return conv3d(x, w, b)


def _conv_bwd_data(g, w, bf16):
    cout, cin = w.shape[0], w.shape[1]
    if bf16 and mfma_forward_ok(cout, cin):  # the adjoint is a convolution from cout to cin channels
        return conv3d_bwd_data(bf16_round(g), bf16_round(w))
    return conv3d_bwd_data(g, w)


def _conv_bwd_weight(x, g, bf16):
    """Weight and bias gradients; bf16: where the matrix-core form takes the
    shape, the weight gradient sees x and g rounded to bfloat16 (the bias
    gradient sums g unrounded)."""
    if bf16 and mfma_wgrad_ok(x.shape[0], g.shape[0]):
        dw, _ = conv3d_bwd_weight(bf16_round(x), bf16_round(g))
        return dw, np.asarray(g, np.float64).sum(axis=(1, 2, 3))
    return conv3d_bwd_weight(x, g)


def unet_layers(channels, in_ch=1):
    """Convolution shapes (cin, cout) in order: encoder levels 0..L-1 (two
    each; the second one of the deepest level maps back to channels[L-2]),
    then decoder levels L-2..0 (two each; the second one maps to the next
    shallower level's channels, at level 0 to 1 channel)."""
    L = len(channels)
    shapes = []
    cin = in_ch
    for lvl, c in enumerate(channels):
        # the deepest level hands channels[L-2] features up to the decoder
        cout2 = channels[L - 2] if (lvl == L - 1 and L > 1) else c
        shapes += [(cin, c), (c, cout2)]
        cin = c
    for lvl in range(L - 2, -1, -1):
        c = channels[lvl]
        nxt = channels[lvl - 1] if lvl > 0 else 1
        shapes += [(c, c), (c, nxt)]
    return shapes


def unet_init(channels, seed, in_ch=1):
    rng = np.random.default_rng(seed)
    params = []
    for cin, cout in unet_layers(channels, in_ch):
        std = np.sqrt(2.0 / (27 * cin))
        params.append((rng.normal(0, std, (cout, cin, 3, 3, 3)), np.zeros(cout)))
    return params


def unet_forward(params, x, channels, bf16=False):
    """x [in_ch][D][H][W] -> (output [1][D][H][W], tape).  Encoder level l:
    conv, relu, conv, relu (kept for the skip), pool to the next level.
    Decoder level l (from L-2 down to 0): upsample, add the level's encoder
    output, conv, relu, conv (+ relu except at level 0).  Output = the last
    input channel + last conv.  bf16: the convolutions that the matrix-core
    form takes see their operands rounded to bfloat16."""
    L = len(channels)
    tape = {}
    h = x
    skips = []
    k = 0
    for lvl in range(L):
        a1 = relu(_conv(h, *params[k], bf16)); k += 1
        a2 = relu(_conv(a1, *params[k], bf16)); k += 1
        tape[("enc", lvl)] = (h, a1, a2)
        skips.append(a2)
        h = pool(a2) if lvl < L - 1 else a2
    for lvl in range(L - 2, -1, -1):
        u = upsample(h)
        s = u + skips[lvl]
        a1 = relu(_conv(s, *params[k], bf16)); k += 1
        z2 = _conv(a1, *params[k], bf16); k += 1
        a2 = relu(z2) if lvl > 0 else z2
        tape[("dec", lvl)] = (s, a1, a2)
        h = a2
    return x[-1:] + h, tape


def unet_backward(params, x, channels, tape, dout, bf16=False):
    """Gradients of the parameters (list of (dw, db)) given dL/d(output).
    bf16: the input and weight gradients that the matrix-core forms take see
    their operands rounded to bfloat16 (bias gradients stay exact)."""
    L = len(channels)
    grads = [None] * len(params)
    k = len(params)
    g = dout  # d/d(last decoder output)
    dskips = [np.zeros_like(tape[("enc", l)][2]) for l in range(L)]
    for lvl in range(0, L - 1):
        s, a1, a2 = tape[("dec", lvl)]
        k -= 2
        gz2 = relu_bwd(a2, g) if lvl > 0 else g
        grads[k + 1] = _conv_bwd_weight(a1, gz2, bf16)
        ga1 = relu_bwd(a1, _conv_bwd_data(gz2, params[k + 1][0], bf16))
        grads[k] = _conv_bwd_weight(s, ga1, bf16)
        gs = _conv_bwd_data(ga1, params[k][0], bf16)
        dskips[lvl] += gs
        g = upsample_bwd(gs)  # gradient of the deeper level's output
    # g now is the gradient of the bottleneck output (encoder level L-1's a2)
    for lvl in range(L - 1, -1, -1):
        h, a1, a2 = tape[("enc", lvl)]
        if lvl < L - 1:
            g = dskips[lvl] + pool_bwd(g)
        k -= 2
        gz2 = relu_bwd(a2, g)
        grads[k + 1] = _conv_bwd_weight(a1, gz2, bf16)
        ga1 = relu_bwd(a1, _conv_bwd_data(gz2, params[k + 1][0], bf16))
        grads[k] = _conv_bwd_weight(h, ga1, bf16)
        g = _conv_bwd_data(ga1, params[k][0], bf16)  # gradient of this level's input
    return grads
