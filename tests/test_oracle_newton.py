"""Pins of the oracle's coupled Newton step (Sec. 2, Eq. 14) and steady
driver.  The Jacobian blocks are checked against central finite
differences of the residual; the steady state against global particle
balance and the fixed-point property."""
import numpy as np
import pytest

import oracle as O
from oracle import newton as NW
from paper_0811_4446_amd import inputs as I


def _state(N, seed=0):
    z = I.z_cos(N)
    ne = I.initial_density(N, N, seed)
    rng = np.random.default_rng(seed + 7)
    ne[:, 1:-1] *= 1 + 200 * rng.random((N + 1, N - 1))
    np_ = ne * (1 + 0.3 * rng.random(ne.shape))
    V = I.initial_potential(N, N, z) + 0.02 * rng.normal(size=(N + 1, N + 1))
    V[:, 0], V[:, -1] = 0.0, 1.0
    return z, np.ascontiguousarray(V), ne, np_, I.source(N, N, z)


def test_bernoulli_derivative_vs_mpmath():
    import mpmath
    mpmath.mp.dps = 50
    for x in [0.0, 1e-9, -3e-4, 9e-4, 1.2e-3, 0.05, -0.0999, 0.1001, -0.7, 2.5, -15.0, 40.0, -300.0]:
        xm = mpmath.mpf(x)
        ref = mpmath.diff(lambda t: t / mpmath.expm1(t) if t != 0 else mpmath.mpf(1), xm) if x != 0 else -0.5
        assert abs(NW.bernoulli_dF(x) - float(ref)) <= 1e-14 * max(1.0, abs(float(ref)))


@pytest.mark.parametrize("N", [8, 16])
def test_jacobian_matches_finite_differences(N):
    """Every column of the 3x3-block Jacobian equals the central difference
    of the residual F(u) (h scaled per field)."""
    z, V, ne, np_, S = _state(N)
    ph = dict(I.PHYS)
    cp = NW.Coupled(N, N, 1.0, z, ph)
    nek, npk = ne.copy(), np_.copy()
    dt_inv = 1e2
    (Fe, Fp, FV), (Ae, Ap) = cp.residual(V, ne, np_, nek, npk, S, S, dt_inv)
    J = cp.jacobian(V, ne, np_, Ae, Ap).toarray()
    rng = np.random.default_rng(1)
    cols = rng.choice(J.shape[1], 40, replace=False)
    fields = [ne, np_, V]
    for col in cols:
        node, f = divmod(col, 3)
        i, j = divmod(node, N - 1)
        j += 1
        h = 1e-6 * max(1.0, abs(fields[f][i, j]))
        saved = fields[f][i, j]
        fields[f][i, j] = saved + h
        Fp_ = cp.pack(*cp.residual(V, ne, np_, nek, npk, S, S, dt_inv)[0])
        fields[f][i, j] = saved - h
        Fm_ = cp.pack(*cp.residual(V, ne, np_, nek, npk, S, S, dt_inv)[0])
        fields[f][i, j] = saved
        fd = (Fp_ - Fm_) / (2 * h)
        scale = np.abs(J[:, col]).max() + 1e-30
        assert np.abs(fd - J[:, col]).max() <= 1e-6 * scale, (col, f)


def test_newton_step_converges_quadratically_and_conserves():
    N = 16
    z = I.z_cos(N)
    ne = I.initial_density(N, N, 3)
    np_ = ne.copy()
    V = I.initial_potential(N, N, z)
    S = I.source(N, N, z)
    ph = dict(I.PHYS)
    cp = NW.Coupled(N, N, 1.0, z, ph)
    nek, npk = ne.copy(), np_.copy()
    hist = []
    ok, its = NW.newton_step(cp, V, ne, np_, S, S, 1e-4, max_newton=10, tol=1e-13, history=hist)
    assert ok and its <= 6
    # quadratic tail: the last corrections shrink much faster than linearly
    c = [max(h) for h in hist]
    assert c[-1] < 1e-13 and c[-2] < 1e-6 and c[-2] < c[-3] ** 1.5
    # the step solves the BE system: residual at the new state is tiny
    (Fe, Fp, FV), _ = cp.residual(V, ne, np_, nek, npk, S, S, 1e4)
    vol = cp.vol
    assert np.abs(Fe / np.where(vol > 0, vol, 1))[:, 1:-1].max() < 1e-12 * np.abs(ne).max() * 1e4


def test_steady_fixed_point_and_global_balance():
    """From the steady state a further step changes nothing, and at steady
    state the source integral equals the particle outflow through the
    electrodes for each species (r = 0 and r = R carry no flux)."""
    N = 8
    z = I.z_cos(N)
    ph = dict(I.PHYS)
    cp = NW.Coupled(N, N, 1.0, z, ph)
    ne = I.initial_density(N, N, 0)
    np_ = ne.copy()
    V = I.initial_potential(N, N, z)
    S = I.source(N, N, z)
    acc, rej, seq = NW.steady(cp, V, ne, np_, S, S, tol=1e-8)
    # drive to the exact steady state with dt = inf
    for _ in range(3):
        NW.newton_step(cp, V, ne, np_, S, S, np.inf, tol=1e-14)
    V0, ne0, np0 = V.copy(), ne.copy(), np_.copy()
    NW.newton_step(cp, V, ne, np_, S, S, 0.1, tol=1e-14)
    assert np.abs(ne - ne0).max() <= 1e-11 * ne0.max()
    assert np.abs(V - V0).max() <= 1e-11
    # global balance: sum of FV rows = vol*S integral minus electrode outflow
    (Fe, Fp, FV), (Ae, Ap) = cp.residual(V, ne, np_, ne, np_, S, S, 0.0)
    src = (cp.vol * S)[:, 1:-1].sum()
    for s, mu, D, n in ((-1, ph["mu_e"], ph["D_e"], ne), (1, ph["mu_p"], ph["D_p"], np_)):
        from tests.test_oracle_pins import _electrode_outflow
        out = _electrode_outflow(1.0, z, s, mu, D, V, n)
        assert abs(out - src) <= 1e-9 * src
