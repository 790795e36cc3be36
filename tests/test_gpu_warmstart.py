"""The warm-start network's hand-written kernels against the CPU reference
(bf16 inputs/weights/activations emulated on the CPU, FP64 accumulation):
forward pass, loss and gradient, training progress, and the exactness of
the feature / target / apply kernels."""
import sys

import numpy as np
import pytest
import torch

from oracle import cnn
from paper_0811_4446_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def M():
    from paper_0811_4446_amd import mgfluid
    return mgfluid


def _params(seed):
    rng = np.random.default_rng(seed)
    out = []
    for ci, co in cnn.LAYERS:
        out.append(rng.normal(size=co * ci * 9) * np.sqrt(2.0 / (9 * ci)))
        out.append(rng.normal(size=co) * 0.1)
    return np.concatenate(out)


@pytest.mark.parametrize("B,H,W", [(2, 9, 20), (1, 17, 33), (1, 5, 3), (3, 40, 17), (1, 257, 257)])
def test_forward_matches_cpu_reference(B, H, W):
    _say("wn forward", B, H, W)
    m = M()
    p = _params(0)
    rng = np.random.default_rng(1)
    x = rng.normal(size=(B, 7, H, W))
    net = m.Net(p)
    out = net.forward(torch.tensor(x, dtype=torch.float32, device="cuda")).cpu().numpy()
    ref = cnn.forward(p.astype(np.float32).astype(np.float64), x.astype(np.float32).astype(np.float64), bf16=True)
    err = np.abs(out - ref).max() / np.abs(ref).max()
    print("forward rel err %.2e" % err)
    assert err <= 1e-2


@pytest.mark.parametrize("B,H,W", [(2, 9, 20), (1, 33, 40)])
def test_gradient_matches_cpu_reference(B, H, W):
    _say("wn grad", B, H, W)
    m = M()
    p = _params(2)
    rng = np.random.default_rng(3)
    x = rng.normal(size=(B, 7, H, W))
    t = rng.normal(size=(B, 3, H, W))
    net = m.Net(p)
    loss, g = net.grad(torch.tensor(x, dtype=torch.float32, device="cuda"),
                       torch.tensor(t, dtype=torch.float32, device="cuda"))
    g = g.cpu().numpy()
    lref, gref = cnn.loss_and_grad(p.astype(np.float32).astype(np.float64), x.astype(np.float32).astype(np.float64),
                                   t.astype(np.float32).astype(np.float64), bf16=True)
    assert abs(loss - lref) <= 1e-2 * abs(lref)
    off = 0
    for ci, co in cnn.LAYERS:
        for n in (co * ci * 9, co):
            a, b = g[off:off + n], gref[off:off + n]
            err = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
            print("grad block size %d rel err %.2e" % (n, err))
            assert err <= 2e-2
            off += n


def test_train_steps_match_oracle_adam():
    """Three wn_train_step calls (gradient + Adam, step counter 1..3) against
    the oracle: the gradient of the bf16-emulated network (FP64) and the
    oracle's Adam recurrences.  The first moment is linear in the gradients
    (held to the gradient tolerance), the second moment quadratic; each
    parameter's total move is compared wherever its gradient is not lost in
    the bf16 noise."""
    _say("wn train step vs oracle adam")
    m = M()
    p = _params(8)
    rng = np.random.default_rng(9)
    B, H, W = 1, 17, 24
    x = rng.normal(size=(B, 7, H, W))
    t = rng.normal(size=(B, 3, H, W))
    x32, t32 = x.astype(np.float32), t.astype(np.float32)
    lr = 1e-3
    net = m.Net(p)
    xt, tt = torch.tensor(x32, device="cuda"), torch.tensor(t32, device="cuda")
    for _ in range(3):
        net.train_step(xt, tt, lr=lr)
    got_p = net.params.cpu().numpy().astype(np.float64)
    got_m = net.m.cpu().numpy().astype(np.float64)
    got_v = net.v.cpu().numpy().astype(np.float64)
    p0 = p.astype(np.float32).astype(np.float64)
    pr, mr, vr = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    gs = []
    for step in (1, 2, 3):
        _, g = cnn.loss_and_grad(pr, x32.astype(np.float64), t32.astype(np.float64), bf16=True)
        gs.append(g)
        cnn.adam(pr, g, mr, vr, step, lr=lr)
    em = np.linalg.norm(got_m - mr) / np.linalg.norm(mr)
    ev = np.linalg.norm(got_v - vr) / np.linalg.norm(vr)
    big = np.min([np.abs(g) for g in gs], axis=0) >= 0.05 * np.max([np.abs(g).max() for g in gs])
    ep = np.abs((got_p - p0) - (pr - p0))[big].max() / lr
    print("adam x3: m rel %.2e, v rel %.2e, move err %.2e lr on %d params" % (em, ev, ep, big.sum()))
    assert em <= 2e-2 and ev <= 4e-2
    assert big.sum() >= 100 and ep <= 5e-2
    assert np.abs(got_p - p0).max() <= 3 * lr * 1.01


def test_training_reduces_loss():
    _say("wn train")
    m = M()
    rng = np.random.default_rng(5)
    B, H, W = 4, 33, 33
    x = rng.normal(size=(B, 7, H, W)).astype(np.float32)
    # a smooth target the network can represent: a linear map of the inputs
    t = np.stack([x[:, 0] * 0.5 - x[:, 3], x[:, 1] + 0.2 * x[:, 4], -x[:, 2]], axis=1).astype(np.float32)
    net = m.Net(_params(6) * 0.5)
    xt, tt = torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda")
    losses = [net.train_step(xt, tt, lr=3e-3) for _ in range(150)]
    print("loss %.4f -> %.4f" % (losses[0], losses[-1]))
    assert losses[-1] < 0.2 * losses[0]


def test_features_targets_apply_roundtrip():
    """apply(up, targets(up, steady)) reproduces steady to FP32 rounding."""
    _say("wn roundtrip")
    m = M()
    N = 64
    z = I.z_cos(N)
    sol = m.Solver(N, N, z)
    rng = np.random.default_rng(7)
    up = [I.initial_potential(N, N, z), 10 + rng.random((N + 1, N + 1)), 10 + rng.random((N + 1, N + 1))]
    st = [up[0] + 0.01 * rng.random(up[0].shape), up[1] * 1.01, up[2] * 0.99]
    for a in up[1:] + st[1:]:
        a[:, 0] = a[:, -1] = 0.0
    for a in (up[0], st[0]):
        a[:, 0], a[:, -1] = 0.0, 1.0
    tu = [sol.upload(a) for a in up]
    ts = [sol.upload(a) for a in st]
    dst = [sol.field() for _ in range(3)]
    S = sol.upload(I.source(N, N, z))
    su = sol.state(tu[0], tu[1], tu[2], S, S)
    ss = sol.state(ts[0], ts[1], ts[2], S, S)
    sd = sol.state(dst[0], dst[1], dst[2], S, S)
    f, ns = m.features(sol, su, 1.0, 100.0)
    assert abs(float(ns.cpu()[0]) - max(up[1].max(), up[2].max())) == 0.0
    fc = f.cpu().numpy()
    assert np.allclose(fc[1], (up[1] / ns.cpu().numpy()[0]).astype(np.float32), rtol=1e-6)
    tg = m.targets(sol, su, ss, 1.0, ns)
    m.apply_prediction(sol, su, tg, 1.0, ns, m.Physics.of(I.PHYS), sd)
    for k in range(3):
        got = sol.download(dst[k])
        assert np.abs(got - st[k]).max() <= 1e-6 * np.abs(st[k]).max()


@pytest.fixture(scope="module")
def small_warmstart():
    """A network trained on the 33 -> 65 -> 129 chain (few draws, few
    epochs) and held-out test data: enough to show the mechanism."""
    _say("warm start: data 129x129 + training")
    from paper_0811_4446_amd import warmstart as WS
    log = lambda *a: print(*a)
    tr = WS.generate(WS.draws(24, 2024), log=log, N=128)
    va = WS.generate(WS.draws(4, 7), log=log, N=128)
    te = WS.generate(WS.draws(6, 8), log=log, N=128)
    net, hist = WS.train(tr, va, epochs=40, log=log)
    return WS, net, te, hist


def test_warm_start_gain_on_held_out_draws(small_warmstart):
    """The network's start needs fewer time steps than the plain
    prolongation on most held-out draws, and both runs end at the same
    discrete steady solution once polished by steady Newton."""
    _say("warm start gain 129x129")
    WS, net, te, hist = small_warmstart
    assert hist[-1][2] < 0.5 * hist[0][2]
    s = WS.compare(net, te, timed=0, log=lambda *a: print(*a))
    print({k: v for k, v in s.items() if not k.startswith("_")})
    assert s["fallbacks"] == 0
    assert s["network_start_steps_ratio_median"] < 1.0
    assert s["steps_learned_mean"] < s["steps_plain_mean"]
    assert s["polished_states_maxrel_diff_max"] < 1e-9


def test_warm_start_forced_fallback(small_warmstart):
    """A run from the network's start that cannot finish (step cap of 3)
    falls back to the plain prolongation, whose result it then returns
    bitwise."""
    _say("warm start forced fallback 129x129")
    WS, net, te, hist = small_warmstart
    s = WS.compare(net, te, timed=0, attempt_steps=3, log=lambda *a: print(*a))
    assert s["fallbacks"] == len(te["draws"])
    for a, b in zip(s["_chosen_finals"], s["_plain_finals"]):
        for k in ("V", "ne", "np"):
            assert torch.equal(a[k], b[k])
