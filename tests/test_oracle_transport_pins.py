"""Pins of the oracle's node-wise transport (Sec. 2: mobilities and
diffusion coefficients as functions of the field, supplied by lookup
tables): constant node values reproduce the constant-coefficient operators
bit for bit; with the Einstein relation D = mu T the Boltzmann density of
the face-mean ratio stays in the null space; a BE step conserves particles
(face sums with 50-digit Bernoulli functions); the Jacobian equals finite
differences; the field strength is exact on linear potentials and on r^2,
and the table lookup is exact on linear tables and clamps outside."""
import mpmath
import numpy as np
import pytest

import oracle as O
from oracle import newton as NW
from paper_0811_4446_amd import inputs as I

mpmath.mp.dps = 50


def _fields(N, seed):
    z = I.z_cos(N)
    rng = np.random.default_rng(seed)
    V = np.ascontiguousarray(I.initial_potential(N, N, z) + 0.05 * rng.normal(size=(N + 1, N + 1)))
    mu = 50.0 * (1.0 + rng.random((N + 1, N + 1)))
    D = mu * (0.01 + 0.02 * rng.random((N + 1, N + 1)))
    return z, V, np.ascontiguousarray(mu), np.ascontiguousarray(D)


@pytest.mark.parametrize("s", [-1, 1])
def test_constant_node_transport_equals_constants(s):
    N = 16
    z, V, _, _ = _fields(N, 1)
    nk = np.random.default_rng(2).random((N + 1, N + 1))
    S = I.source(N, N, z)
    mu, D = 37.0, 0.9
    a = O.sg_assemble(N, N, 1.0, z, s, mu, D, 1e2, V, nk, S)
    b = O.sg_assemble(N, N, 1.0, z, s, 0.0, 1.0, 1e2, V, nk, S, mun=np.full_like(V, mu), Dn=np.full_like(V, D))
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
    da = NW._sg_dV(N, N, 1.0, z, s, mu, D, V, nk)
    db = NW._sg_dV(N, N, 1.0, z, s, 0.0, 1.0, V, nk, mun=np.full_like(V, mu), Dn=np.full_like(V, D))
    for x, y in zip(da, db):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("s", [-1, 1])
def test_einstein_relation_keeps_boltzmann_null_space(s):
    """D = mu T node by node: every face has mu/D = 1/T, so n = exp(-s V/T)
    carries no flux, whatever the mobility varies like."""
    N = 16
    z, V, mu, _ = _fields(N, 3)
    T = 0.02
    D = np.ascontiguousarray(mu * T)
    A = O.sg_assemble(N, N, 1.0, z, s, 0.0, 1.0, 0.0, V, mun=mu, Dn=D)
    n = np.exp(-s * (V - V.mean()) / T)
    res = O.apply(A, n)[:, 1:-1]
    assert np.abs(res).max() <= 1e-12 * np.abs(A[1] * n).max()
    # a mobility that is not proportional to D breaks it
    A2 = O.sg_assemble(N, N, 1.0, z, s, 0.0, 1.0, 0.0, V, mun=mu, Dn=np.ascontiguousarray(D * (1 + 0.5 * np.sin(mu))))
    assert np.abs(O.apply(A2, n)[:, 1:-1]).max() >= 1e-3 * np.abs(A2[1] * n).max()


@pytest.mark.parametrize("s", [-1, 1])
def test_node_transport_step_conserves_particles(s):
    N, dt = 16, 1e-3
    z, V, mu, D = _fields(N, 5)
    rng = np.random.default_rng(6)
    nk = rng.random((N + 1, N + 1))
    nk[:, 0] = nk[:, -1] = 0
    S = I.source(N, N, z)
    coef = O.sg_assemble(N, N, 1.0, z, s, 0.0, 1.0, 1.0 / dt, V, nk, S, mun=mu, Dn=D)
    n = nk.copy()
    O.direct_solve(coef, n)

    def Fm(x):
        x = mpmath.mpf(x)
        return float(x / mpmath.expm1(x)) if x != 0 else 1.0

    dr = 1.0 / N
    w = np.array([dr * dr / 8] + [i * dr * dr for i in range(1, N)] + [0.5 * dr * (1.0 - dr / 4)])
    out = 0.0
    for i in range(N + 1):
        for (jl, ju, sign) in ((0, 1, -1.0), (N - 1, N, 1.0)):
            Df = 0.5 * (D[i, jl] + D[i, ju])
            al = -s * 0.5 * (mu[i, jl] + mu[i, ju]) / Df * (V[i, ju] - V[i, jl])
            out += sign * w[i] * Df / (z[ju] - z[jl]) * (n[i, jl] * Fm(-al) - n[i, ju] * Fm(al))
    vol = O.volumes(N, N, 1.0, z)
    lhs = (vol * ((n - nk) / dt - S))[:, 1:N].sum()
    assert abs(lhs + out) <= 1e-10 * np.abs(vol * S).sum(), (lhs, out)
    fl = NW.boundary_flow(1.0, z, s, 0.0, 1.0, V, n, mun=mu, Dn=D)
    assert abs(fl[0] + fl[1] - out) <= 1e-12 * abs(out)


def test_node_transport_jacobian_matches_finite_differences():
    N = 8
    z, V, mu, D = _fields(N, 7)
    rng = np.random.default_rng(8)
    ne = 1e-3 * (1 + 100 * rng.random((N + 1, N + 1)))
    np_ = ne * (1 + 0.3 * rng.random(ne.shape))
    ne[:, 0] = ne[:, -1] = np_[:, 0] = np_[:, -1] = 0
    tr = dict(mue=mu, De=D, mup=np.ascontiguousarray(mu / 80), Dp=np.ascontiguousarray(D / 90))
    cp = NW.Coupled(N, N, 1.0, z, dict(I.PHYS), transport=tr)
    S = I.source(N, N, z)
    nek, npk = ne.copy(), np_.copy()
    (Fe, Fp, FV), (Ae, Ap) = cp.residual(V, ne, np_, nek, npk, S, S, 1e2)
    J = cp.jacobian(V, ne, np_, Ae, Ap).toarray()
    fields = [ne, np_, V]
    for col in np.random.default_rng(9).choice(J.shape[1], 40, replace=False):
        node, f = divmod(col, 3)
        i, j = divmod(node, N - 1)
        j += 1
        h = 1e-6 * max(1.0, abs(fields[f][i, j]))
        saved = fields[f][i, j]
        fields[f][i, j] = saved + h
        Fa = cp.pack(*cp.residual(V, ne, np_, nek, npk, S, S, 1e2)[0])
        fields[f][i, j] = saved - h
        Fb = cp.pack(*cp.residual(V, ne, np_, nek, npk, S, S, 1e2)[0])
        fields[f][i, j] = saved
        fd = (Fa - Fb) / (2 * h)
        assert np.abs(fd - J[:, col]).max() <= 1e-6 * (np.abs(J[:, col]).max() + 1e-30), (col, f)


def test_field_strength_exact_cases_and_table_lookup():
    N = 16
    z = I.z_cos(N)
    r = np.arange(N + 1) / N
    V = np.ascontiguousarray(np.repeat((3.0 * z)[None, :], N + 1, axis=0))
    np.testing.assert_allclose(NW.field_strength(1.0, z, V), 3.0, rtol=1e-14)
    V2 = np.ascontiguousarray(np.repeat((0.7 * r ** 2)[:, None], N + 1, axis=1))
    E2 = NW.field_strength(1.0, z, V2)
    np.testing.assert_allclose(E2[1:N], (1.4 * r[1:N, None]) * np.ones((1, N + 1)), rtol=1e-13)
    assert np.all(E2[0] == 0.0)
    Et = np.array([0.0, 1.0, 2.0, 5.0])
    mu, D = NW.transport_from_table(1.0, z, V, Et, 10.0 - Et, 1.0 + 0.5 * Et)
    np.testing.assert_allclose(mu, 7.0, rtol=1e-14)
    np.testing.assert_allclose(D, 2.5, rtol=1e-14)
    mu, D = NW.transport_from_table(1.0, z, np.ascontiguousarray(V * 10), Et, 10.0 - Et, 1.0 + 0.5 * Et)
    assert np.all(mu == 5.0) and np.all(D == 3.5)
