"""Pins of the oracle's Dirichlet wall at r = R (the paper's experiment,
Sec. 3: potential interpolated linearly along the wall, densities 0 there):
a manufactured cylindrical solution converges at second order, the rows of
the inner nodes are those of the zero-flux domain, the SG operator keeps the
Boltzmann null space up to the wall, one BE step conserves particles with the
wall outflow counted (fluxes from 50-digit Bernoulli functions), multigrid
equals a dense direct solve, the Newton Jacobian equals finite differences,
and a steady state balances sources against electrode plus wall outflow."""
import mpmath
import numpy as np
import pytest

import oracle as O
from oracle import newton as NW
from paper_0811_4446_amd import inputs as I

mpmath.mp.dps = 50


def _Fm(x):
    x = mpmath.mpf(x)
    return float(x / mpmath.expm1(x)) if x != 0 else 1.0


def _outflow(R, z, s, mu, D, V, n):
    """Net particle flow (per radian) out of the unknown cells i < nr through
    the electrode faces j = 1/2, nz - 1/2 and the wall face r_{nr-1/2}, from
    the SG flux of Eqs. (8)-(9) with 50-digit Bernoulli functions."""
    N, nz = V.shape[0] - 1, V.shape[1] - 1
    dr = R / N
    w = np.array([dr * dr / 8] + [i * dr * dr for i in range(1, N)])
    q = -s * mu / D
    out = 0.0
    for i in range(N):
        for (jl, ju, sign) in ((0, 1, -1.0), (nz - 1, nz, 1.0)):
            al = q * (V[i, ju] - V[i, jl])
            out += sign * w[i] * D / (z[ju] - z[jl]) * (n[i, jl] * _Fm(-al) - n[i, ju] * _Fm(al))
    for j in range(1, nz):
        dzc = 0.5 * (z[j + 1] - z[j - 1])
        al = q * (V[N, j] - V[N - 1, j])
        out += (N - 0.5) * dr * dzc * D / dr * (n[N - 1, j] * _Fm(-al) - n[N, j] * _Fm(al))
    return out


def test_poisson_wall_manufactured_second_order():
    """V = z + c cos(pi r / 2R) sin(pi z) satisfies the paper's wall condition
    (V(R, z) = z, linear between the electrodes 0 and 1) and dV/dr = 0 on the
    axis; with its Laplacian as the charge the discrete solution converges at
    second order on the cos-stretched grid."""
    c = 0.3
    errs = []
    Ns = [16, 32, 64, 128]
    for N in Ns:
        z = I.z_cos(N)
        r = np.arange(N + 1) / N
        rr, zz = np.meshgrid(r, z, indexing="ij")
        h = np.pi / 2
        with np.errstate(invalid="ignore", divide="ignore"):
            sr = np.where(rr > 0, np.sin(h * rr) / np.where(rr > 0, rr, 1.0), h)
        lap = c * np.sin(np.pi * zz) * (h * h * np.cos(h * rr) + h * sr + np.pi ** 2 * np.cos(h * rr))
        exact = zz + c * np.cos(h * rr) * np.sin(np.pi * zz)
        Vw = O.wall_values(z, 0.0, 1.0)
        coef = O.poisson_assemble(N, N, 1.0, z, 1.0, np.zeros_like(lap), np.ascontiguousarray(lap), wall=1, Vwall=Vw)
        x = np.zeros((N + 1, N + 1))
        x[:, -1] = 1.0
        mg = O.MG(N, N, 1.0, z, coarsest=8, smoother=O.SMOOTH_RB, wall=1)
        mg.assemble_poisson(1.0, np.zeros_like(lap), np.ascontiguousarray(lap), Vwall=Vw)
        for k in range(6):
            np.testing.assert_array_equal(mg.coef(0)[k], coef[k])
        st, cyc, rr_ = mg.solve(x, rtol=1e-13, max_cycles=200)
        assert st == 0, (N, cyc, rr_)
        assert np.abs(x[-1, :] - Vw).max() <= 1e-15
        errs.append(np.abs(x - exact).max())
    orders = [np.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert min(orders) > 1.8, (errs, orders)


@pytest.mark.parametrize("N", [8, 16])
def test_wall_rows_identity_inner_rows_unchanged(N):
    """With the wall the rows i < nr are those of the zero-flux operator (full
    control volumes, the face r_{nr-1/2} couples to the wall node) and the
    rows i = nr are identities (right-hand side: the wall potential on
    Poisson, 0 on the SG equations)."""
    z = I.z_cos(N)
    rng = np.random.default_rng(N)
    ne, np_ = rng.random((N + 1, N + 1)), rng.random((N + 1, N + 1))
    V = np.ascontiguousarray(I.initial_potential(N, N, z) + 0.05 * rng.normal(size=(N + 1, N + 1)))
    Vw = O.wall_values(z, 0.0, 1.0)
    for A0, A1, fw in ((O.poisson_assemble(N, N, 1.0, z, 7.0, ne, np_),
                        O.poisson_assemble(N, N, 1.0, z, 7.0, ne, np_, wall=1, Vwall=Vw), Vw),
                       (O.sg_assemble(N, N, 1.0, z, -1, 100.0, 1.0, 1e3, V, ne, np_),
                        O.sg_assemble(N, N, 1.0, z, -1, 100.0, 1.0, 1e3, V, ne, np_, wall=1), 0 * Vw)):
        for k in range(6):
            np.testing.assert_array_equal(A1[k][:N], A0[k][:N])
        assert np.all(A1[1][N, 1:-1] == 1.0)
        for k in (0, 2, 3, 4):
            assert np.all(A1[k][N] == 0.0)
        np.testing.assert_array_equal(A1[5][N, 1:-1], fw[1:-1])


@pytest.mark.parametrize("s,mu,D", [(-1, 100.0, 1.0), (1, 1.0, 0.01)])
def test_sg_wall_boltzmann_up_to_the_wall(s, mu, D):
    """n = exp(-s mu/D V) with the wall node holding that value as well: no
    face flux anywhere, so every inner row (i < nr) of the steady operator
    annihilates it, including the rows next to the wall."""
    N = 16
    z = I.z_cos(N)
    r = np.arange(N + 1) / N
    V = np.ascontiguousarray(z[None, :] + 0.07 * np.cos(2.1 * r[:, None]) * np.sin(2.9 * z[None, :]))
    q = -s * mu / D
    n = np.exp(q * (V - V.mean()))
    A = O.sg_assemble(N, N, 1.0, z, s, mu, D, 0.0, V, wall=1)
    res = O.apply(A, n)[:N, 1:-1]
    assert np.abs(res).max() <= 1e-13 * np.abs(A[1][:N] * n[:N]).max()


@pytest.mark.parametrize("s,mu,D", [(-1, 100.0, 1.0), (1, 1.0, 0.01)])
def test_sg_wall_step_conserves_particles(s, mu, D):
    """One BE step with the wall: sum over the unknown cells of
    vol ((n - n^k)/dt - S) = -(outflow through both electrodes and the wall)."""
    N, dt = 16, 1e-3
    z = I.z_cos(N)
    rng = np.random.default_rng(3)
    V = np.ascontiguousarray(I.initial_potential(N, N, z) + 0.05 * rng.normal(size=(N + 1, N + 1)))
    nk = rng.random((N + 1, N + 1))
    nk[:, 0] = nk[:, -1] = nk[-1, :] = 0.0
    S = I.source(N, N, z)
    coef = O.sg_assemble(N, N, 1.0, z, s, mu, D, 1.0 / dt, V, nk, S, wall=1)
    n = nk.copy()
    O.direct_solve(coef, n)
    assert np.all(n[-1, :] == 0.0)
    vol = O.volumes(N, N, 1.0, z)
    lhs = (vol * ((n - nk) / dt - S))[:N, 1:N].sum()
    out = _outflow(1.0, z, s, mu, D, V, n)
    assert abs(lhs + out) <= 1e-10 * np.abs(vol * S).sum(), (lhs, out)
    # the wall really takes particles: its share of the outflow is not small
    assert abs(_outflow(1.0, z, s, mu, D, V, n) - _outflow_electrodes_only(1.0, z, s, mu, D, V, n)) > 1e-3 * abs(out)


def _outflow_electrodes_only(R, z, s, mu, D, V, n):
    N, nz = V.shape[0] - 1, V.shape[1] - 1
    dr = R / N
    w = np.array([dr * dr / 8] + [i * dr * dr for i in range(1, N)])
    q = -s * mu / D
    out = 0.0
    for i in range(N):
        for (jl, ju, sign) in ((0, 1, -1.0), (nz - 1, nz, 1.0)):
            al = q * (V[i, ju] - V[i, jl])
            out += sign * w[i] * D / (z[ju] - z[jl]) * (n[i, jl] * _Fm(-al) - n[i, ju] * _Fm(al))
    return out


@pytest.mark.parametrize("smoother", [O.SMOOTH_RB, O.SMOOTH_ZEBRA])
@pytest.mark.parametrize("eq", ["poisson", "electron", "ion"])
def test_mg_with_wall_matches_dense_solve(smoother, eq):
    """Multigrid with the wall rows on every level converges to the dense
    direct solution of the same system (9x9 and 17x17 grids)."""
    for N in (8, 16):
        z = I.z_cos(N)
        rng = np.random.default_rng(N + len(eq))
        ne, np_ = rng.random((N + 1, N + 1)), rng.random((N + 1, N + 1))
        V = np.ascontiguousarray(I.initial_potential(N, N, z) + 0.02 * rng.normal(size=(N + 1, N + 1)))
        Vw = O.wall_values(z, 0.0, 1.0)
        mg = O.MG(N, N, 1.0, z, coarsest=4, smoother=smoother, wall=1)
        x = np.zeros((N + 1, N + 1))
        if eq == "poisson":
            mg.assemble_poisson(50.0, ne, np_, Vwall=Vw)
            x[:, -1] = 1.0
        else:
            s, mu, D = (-1, 100.0, 1.0) if eq == "electron" else (1, 1.0, 0.01)
            mg.assemble_sg(s, mu, D, 1e2, V, ne, I.source(N, N, z))
        ref = x.copy()
        O.direct_solve(mg.coef(0), ref)
        st, cyc, rr = mg.solve(x, rtol=1e-13, max_cycles=300)
        assert st == 0
        assert np.abs(x - ref).max() <= 1e-11 * np.abs(ref).max(), (N, eq)


def _wall_state(N, seed=0):
    z = I.z_cos(N)
    ne = I.initial_density(N, N, seed)
    rng = np.random.default_rng(seed + 7)
    ne[:, 1:-1] *= 1 + 200 * rng.random((N + 1, N - 1))
    np_ = ne * (1 + 0.3 * rng.random(ne.shape))
    V = I.initial_potential(N, N, z) + 0.02 * rng.normal(size=(N + 1, N + 1))
    cp = NW.Coupled(N, N, 1.0, z, dict(I.PHYS), wall=1)
    V = np.ascontiguousarray(V)
    cp.electrodes(V, ne, np_)
    return z, cp, V, ne, np_, I.source(N, N, z)


def test_newton_jacobian_with_wall_matches_finite_differences():
    """Every column of the Jacobian (Eq. 14) with the wall rows equals the
    central difference of the residual, including the columns of the nodes
    next to the wall and of the wall nodes themselves."""
    N = 8
    z, cp, V, ne, np_, S = _wall_state(N)
    nek, npk = ne.copy(), np_.copy()
    dt_inv = 1e2
    (Fe, Fp, FV), (Ae, Ap) = cp.residual(V, ne, np_, nek, npk, S, S, dt_inv)
    assert np.abs(Fe[-1]).max() == 0 and np.abs(Fp[-1]).max() == 0 and np.abs(FV[-1]).max() == 0
    J = cp.jacobian(V, ne, np_, Ae, Ap).toarray()
    fields = [ne, np_, V]
    cols = [3 * (i * (N - 1) + (j - 1)) + f for i in (N - 1, N) for j in range(1, N) for f in range(3)]
    rng = np.random.default_rng(2)
    cols += list(rng.choice(J.shape[1], 20, replace=False))
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
        assert np.abs(fd - J[:, col]).max() <= 1e-6 * scale, (col, i, j, f)


def test_steady_with_wall_balances_sources_against_electrode_and_wall_outflow():
    """A steady run with the wall (synthetic physics, 9x9): the wall rows keep
    their values, one more step changes nothing, and for each species the
    source integral equals the outflow through the electrodes and the wall."""
    N = 8
    z = I.z_cos(N)
    ph = dict(I.PHYS)
    cp = NW.Coupled(N, N, 1.0, z, ph, wall=1)
    ne = I.initial_density(N, N, 0)
    np_ = ne.copy()
    V = I.initial_potential(N, N, z)
    S = I.source(N, N, z)
    NW.steady(cp, V, ne, np_, S, S, tol=1e-8)
    for _ in range(3):
        NW.newton_step(cp, V, ne, np_, S, S, np.inf, tol=1e-14)
    # the sparse LU leaves rounding noise of the size of eps * |du| on the wall rows
    assert np.abs(ne[-1]).max() <= 1e-14 * ne.max() and np.abs(np_[-1]).max() <= 1e-14 * np_.max()
    assert np.abs(V[-1] - O.wall_values(z, 0.0, 1.0)).max() <= 1e-14
    V0, ne0 = V.copy(), ne.copy()
    NW.newton_step(cp, V, ne, np_, S, S, 0.1, tol=1e-14)
    assert np.abs(ne - ne0).max() <= 1e-11 * ne0.max() and np.abs(V - V0).max() <= 1e-11
    src = (cp.vol * S)[:N, 1:-1].sum()
    for s, mu, D, n in ((-1, ph["mu_e"], ph["D_e"], ne), (1, ph["mu_p"], ph["D_p"], np_)):
        out = _outflow(1.0, z, s, mu, D, V, n)
        assert abs(out - src) <= 1e-9 * src, (s, out, src)


@pytest.mark.parametrize("wall", [0, 1])
def test_boundary_flow_equals_independent_face_sums(wall):
    """newton.boundary_flow (cathode, anode, wall) equals the face sums
    written here with 50-digit Bernoulli functions, and a BE step's particle
    balance closes with it: sum vol ((n - n^k)/dt - S) = -(total outflow)."""
    N, dt = 16, 1e-3
    z = I.z_cos(N)
    rng = np.random.default_rng(11 + wall)
    V = np.ascontiguousarray(I.initial_potential(N, N, z) + 0.05 * rng.normal(size=(N + 1, N + 1)))
    nk = rng.random((N + 1, N + 1))
    nk[:, 0] = nk[:, -1] = 0.0
    if wall:
        nk[-1, :] = 0.0
    S = I.source(N, N, z)
    for s, mu, D in ((-1, 100.0, 1.0), (1, 1.0, 0.01)):
        coef = O.sg_assemble(N, N, 1.0, z, s, mu, D, 1.0 / dt, V, nk, S, wall=wall)
        n = nk.copy()
        O.direct_solve(coef, n)
        cath, anode, wflow = NW.boundary_flow(1.0, z, s, mu, D, V, n, wall)
        if wall:
            ref = _outflow(1.0, z, s, mu, D, V, n)
            ref_e = _outflow_electrodes_only(1.0, z, s, mu, D, V, n)
            assert abs((cath + anode) - ref_e) <= 1e-12 * abs(ref_e)
            assert abs((cath + anode + wflow) - ref) <= 1e-12 * abs(ref)
        else:
            assert wflow == 0.0
        vol = O.volumes(N, N, 1.0, z)
        cells = (slice(0, N if wall else N + 1), slice(1, N))
        lhs = (vol * ((n - nk) / dt - S))[cells].sum()
        assert abs(lhs + cath + anode + wflow) <= 1e-10 * np.abs(vol * S).sum()
