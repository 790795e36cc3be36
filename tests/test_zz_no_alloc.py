"""The allocation-free forward entry point (wn_forward_noalloc) against the
scratch-buffer one (wn_forward): two calls in a row through the C ABI, the
second on a smaller input, each bitwise equal to wn_forward on the same
input, and a batch of several full-size images.  (The launch limit is
checked on the CPU.)"""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _params(seed):
    from oracle import cnn
    rng = np.random.default_rng(seed)
    out = []
    for ci, co in cnn.LAYERS:
        out.append(rng.normal(size=co * ci * 9) * np.sqrt(2.0 / (9 * ci)))
        out.append(rng.normal(size=co) * 0.1)
    return np.concatenate(out)


def test_forward_noalloc_matches_forward_twice():
    from paper_0811_4446_amd import mgfluid as M
    net = M.Net(_params(21))
    rng = np.random.default_rng(22)
    for (B, H, W) in ((1, 257, 257), (2, 33, 40)):
        _say("wn_forward_noalloc", B, H, W)
        x = torch.tensor(rng.normal(size=(B, 7, H, W)), dtype=torch.float32, device="cuda")
        want = net.forward(x)
        got = torch.full((B, 3, H, W), float("nan"), dtype=torch.float32, device="cuda")
        net.forward_noalloc(x, got)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (B, H, W, float((got - want).abs().max()))


def test_forward_noalloc_takes_batches_beyond_one_image():
    """The static array holds only the packed weights, so a batch of several
    257 x 257 images (which no fixed activation buffer would hold) runs too,
    bitwise equal to wn_forward."""
    from paper_0811_4446_amd import mgfluid as M
    net = M.Net(_params(23))
    rng = np.random.default_rng(24)
    _say("wn_forward_noalloc", 3, 257, 257)
    x = torch.tensor(rng.normal(size=(3, 7, 257, 257)), dtype=torch.float32, device="cuda")
    want = net.forward(x)
    got = torch.full((3, 3, 257, 257), float("nan"), dtype=torch.float32, device="cuda")
    net.forward_noalloc(x, got)
    torch.cuda.synchronize()
    assert torch.equal(got, want), float((got - want).abs().max())
