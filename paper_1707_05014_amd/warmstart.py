"""Learned warm start of the row-action sweeps.

The paper starts its block-iterative sweeps from an initial guess x0 that it
leaves to the user (Sec. 2.1).  Here x0 can come from a 3D U-Net
(``cnn.UNet3D``) that maps the image after a few sweeps from the hull start
to an estimate of the image after many sweeps; the plain sweeps then
continue from it.  Training pairs come from the solver itself on seeded
phantoms.  Everything runs in the library's kernels: the sweeps in the plan
kernels, the network in the pct_cnn_* kernels; torch provides memory.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import api, cnn


def volume(x: torch.Tensor, grid) -> torch.Tensor:
    """[M] image -> [1][nz][ny][nx] view (x fastest, as the grid's linear index)."""
    return x.view(1, grid.nz, grid.ny, grid.nx)


def sweep_snapshots(grid, plan, x: torch.Tensor, params_one: "api.SweepParams", snapshots, stream=None):
    """Run max(snapshots) sweeps on x in place; return copies of x after each
    sweep count listed in snapshots (a dict count -> [M] tensor)."""
    want = sorted(set(int(s) for s in snapshots))
    out = {}
    for s in range(1, want[-1] + 1):
        api.plan_sweep(grid, plan, x, params_one, stream=stream)
        if s in want:
            out[s] = x.clone()
    return out


def net_input(snapshots: dict, sweeps, grid) -> torch.Tensor:
    """[len(sweeps)][nz][ny][nx] network input from the images after the
    listed sweep counts (the last one is the image the network corrects)."""
    vols = [volume(snapshots[s], grid) for s in sweeps]
    return vols[0].clone() if len(vols) == 1 else torch.cat(vols, dim=0)


def train(net: "cnn.UNet3D", pairs, steps: int, lr: float = 1e-3, seed: int = 0, coarse_weight: float = 0.0,
          log=None, log_every: int = 100, warmup: int | None = None):
    """Adam on the network's loss (MSE plus coarse_weight times the MSE of
    4x4x4 block means) between net(input) and target over `pairs` (list of
    ([in][D][H][W] input, [1][D][H][W] target) device tensors), one pair per
    step in a seeded shuffled order, learning rate ramped up linearly over
    the first warmup steps, then with cosine decay (without the ramp, Adam's
    first full-size steps now and then leave a network stuck at its identity
    start).  Returns the per-step voxel MSEs (host floats) and the wall time
    (s)."""
    rng = np.random.default_rng(seed)
    warm = max(1, steps // 20) if warmup is None else max(int(warmup), 1)
    order = []
    losses = []
    t0 = time.perf_counter()
    for k in range(steps):
        if not order:
            order = list(rng.permutation(len(pairs)))
        i = order.pop()
        lr_k = lr * 0.5 * (1.0 + math.cos(math.pi * k / max(steps, 1)))
        if k < warm:
            lr_k *= (k + 1) / warm
        losses.append(net.loss_and_grad(pairs[i][0], pairs[i][1], coarse_weight))
        net.adam_step(max(lr_k, 1e-3 * lr))
        if log is not None and (k + 1) % log_every == 0:
            log(f"train step {k + 1}/{steps}: loss {float(losses[-1].item()):.4e}")
    torch.cuda.synchronize()
    return [float(v.item()) for v in losses], time.perf_counter() - t0


def warm_start(net, inp: torch.Tensor, hull_mask: torch.Tensor, stream=None) -> torch.Tensor:
    """x0 = net(inp) restricted to the hull (a new [M] tensor); inp is the
    network input built by net_input().  net may also be a list of networks
    (an ensemble trained from different seeds): x0 is then the mean of their
    outputs."""
    nets = list(net) if isinstance(net, (list, tuple)) else [net]
    if len(nets) == 1:
        y = nets[0].predict(inp, stream=stream).view(-1)
    else:
        y = torch.zeros(hull_mask.numel(), dtype=torch.float32, device=inp.device)
        for k in nets:
            cnn.axpy(1.0 / len(nets), k.predict(inp, stream=stream).view(-1), y, stream=stream)
    cnn.mask(y, hull_mask, y, stream=stream)
    return y
