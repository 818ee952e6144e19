"""The device history generator against the host one: the same seeded
Philox counter stream and FP64 transport, so the float32 histories agree bit
for bit except where a device transcendental's last bit differs from the
host's (allowed on at most 1e-4 of the histories, and then only within a
few float32 ulps)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import synth  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("key,n,start", [(1, 100_000, 0), (2, 100_000, 7_654_321), (3, 50_000, 199_000_000)])
def test_gpu_generator_matches_host(key, n, start):
    cfg = synth.config(key)
    _say(f"generator: config {key}, histories [{start}, {start + n})")
    hc = synth.generate(cfg, n=n, start=start)
    hg = synth.generate_gpu(cfg, n=n, start=start)
    torch.cuda.synchronize()
    same = np.ones(n, bool)
    worst = 0.0
    for k in synth.HIST_FIELDS:
        a = hc[k]
        b = hg[k].cpu().numpy()
        same &= a.view(np.uint32) == b.view(np.uint32)
        d = np.abs(a.astype(np.float64) - b) / np.maximum(np.abs(a.astype(np.float64)), 1e-3)
        worst = max(worst, float(d.max()))
    frac = same.mean()
    _say(f"  bit-identical histories {frac:.6f}; worst relative field difference {worst:.2e}")
    assert frac >= 0.9999
    assert worst <= 1e-6


def test_gpu_generator_empty_and_rejects_bad_args():
    cfg = synth.config(1)
    h = synth.generate_gpu(cfg, n=0)
    assert all(v.numel() == 0 for v in h.values())
    with pytest.raises(RuntimeError):
        synth.generate_gpu(cfg, n=10, start=-1)
