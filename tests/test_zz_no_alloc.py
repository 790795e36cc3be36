"""The allocation-free forward entry point (wn_forward_noalloc) against the
scratch-buffer one (wn_forward): two calls in a row through the C ABI, the
second on a smaller input, each bitwise equal to wn_forward on the same
input; sizes beyond its static array are refused on the host."""
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


def test_forward_noalloc_refuses_oversized_input():
    from paper_0811_4446_amd import mgfluid as M
    net = M.Net(_params(23))
    x = torch.zeros((2, 7, 257, 257), dtype=torch.float32, device="cuda")
    out = torch.zeros((2, 3, 257, 257), dtype=torch.float32, device="cuda")
    with pytest.raises(M.MGError) as ei:
        net.forward_noalloc(x, out)
    assert ei.value.code == -1 and "static scratch" in str(ei.value)
