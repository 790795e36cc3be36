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


def _hier(N, dt, coarsest=4, seed=0):
    z, V, ne, np_ = _state(N, seed)[:4]
    return NW.block_hierarchy(N, N, 1.0, z, dict(I.PHYS), V, ne, np_, dt, coarsest=coarsest)


def test_block_colour_sweep_solves_its_nodes():
    """After a half-sweep the three equations of every node of that colour
    hold exactly (to rounding), and the other colour is untouched."""
    L = _hier(16, 1e-2)[0]
    rng = np.random.default_rng(3)
    f = rng.normal(size=L["J"].shape[0])
    x = rng.normal(size=f.size)
    for c in (0, 1):
        before = x.copy()
        NW.block_colour_sweep(L, f, x, c)
        r = f - L["J"] @ x
        ix, other = L["idx"][c], L["idx"][1 - c]
        assert np.abs(r[ix]).max() <= 1e-12 * np.abs(f).max() * 1e3
        assert np.array_equal(x[other], before[other])


def test_block_vcycle_single_level_is_the_exact_solve():
    """With one level the cycle is the coarsest-grid solve: x = J^-1 f."""
    levels = _hier(4, 1e-2, coarsest=4)
    assert len(levels) == 1
    f = np.random.default_rng(4).normal(size=levels[0]["J"].shape[0])
    x = NW.block_vcycle(levels, f)
    assert np.abs(levels[0]["J"] @ x - f).max() <= 1e-10 * np.abs(f).max()


@pytest.mark.parametrize("dt", [1e-4])
def test_block_vcycle_iteration_converges_to_the_solution(dt):
    """At a small step (diagonally strong Jacobian) x <- x + V(f - J x)
    converges to J^-1 f (a wrong sign, weight or transfer in the cycle would
    stall or diverge), and the cycle is a linear map of f.  At larger steps
    the stationary iteration need not converge (on this perturbed state it
    diverges from dt = 1e-3), which is why the cycle preconditions FGMRES."""
    levels = _hier(16, dt)
    J = levels[0]["J"]
    assert len(levels) == 3
    rng = np.random.default_rng(5)
    f = rng.normal(size=J.shape[0])
    exact = NW.spla.spsolve(J.tocsc(), f)
    x = np.zeros_like(f)
    errs = []
    for _ in range(25):
        x += NW.block_vcycle(levels, f - J @ x)
        errs.append(np.abs(x - exact).max() / np.abs(exact).max())
    assert errs[-1] <= 1e-10, errs
    g = rng.normal(size=f.size)
    lin = NW.block_vcycle(levels, 2.0 * f - 3.0 * g)
    assert np.abs(lin - (2.0 * NW.block_vcycle(levels, f) - 3.0 * NW.block_vcycle(levels, g))).max() \
        <= 1e-12 * np.abs(lin).max()


def test_block_transfers_are_adjoint_and_exact_on_bilinear():
    """Field by field, restriction is the transpose of prolongation, and
    prolongation reproduces functions bilinear in (r, z) at the fine nodes."""
    levels = _hier(16, 1e-2)
    L, Lc = levels[0], levels[1]
    rng = np.random.default_rng(6)
    u = rng.normal(size=Lc["J"].shape[0])
    v = rng.normal(size=L["J"].shape[0])
    lhs = np.dot(NW.block_prolong(L, Lc, u), v)
    rhs = np.dot(u, NW.block_restrict(L, Lc, v))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    zc, zf = Lc["z"], L["z"]
    rc = np.linspace(0.0, 1.0, 9)[:, None]
    rf = np.linspace(0.0, 1.0, 17)[:, None]
    # a field linear in r and constant in z (zero on the electrode rows, where corrections vanish)
    gc = (1.0 + 2.0 * rc) * np.ones((1, zc.size))
    gc[:, 0] = gc[:, -1] = 0.0
    pf = Lc["cp"].pack(gc, 2 * gc, 3 * gc)
    out = L["cp"].unpack(NW.block_prolong(L, Lc, pf))
    want = (1.0 + 2.0 * rf) * np.ones((1, zf.size))
    # away from the first and last fine interior nodes (their coarse neighbour is an electrode)
    for k, fac in enumerate((1, 2, 3)):
        assert np.abs(out[k][:, 2:-2] - fac * want[:, 2:-2]).max() <= 1e-13


def test_block_zebra_sweep_solves_its_lines():
    """Block zebra z-line half-sweep (all unknowns of the axial lines of one
    parity solved together): lines of one parity share no matrix entry (the
    five-point stencil reaches i +- 1 only), after the half-sweep every
    equation of those lines holds to rounding, and the other lines are
    untouched."""
    L = _hier(16, 1e-2)[0]
    cp = L["cp"]
    for c in (0, 1):
        sub = L["J"][L["lidx"][c]][:, L["lidx"][c]].tocoo()
        lines = cp.ii[L["lidx"][c] // 3]
        assert np.array_equal(lines[sub.row], lines[sub.col])
    rng = np.random.default_rng(13)
    f = rng.normal(size=L["J"].shape[0])
    x = rng.normal(size=f.size)
    for c in (0, 1):
        before = x.copy()
        NW.block_colour_sweep(L, f, x, c, lines=True)
        r = f - L["J"] @ x
        ix, other = L["lidx"][c], L["lidx"][1 - c]
        assert np.abs(r[ix]).max() <= 1e-12 * np.abs(f).max() * 1e3
        assert np.array_equal(x[other], before[other])


def test_block_zebra_sweep_is_exact_without_radial_coupling():
    """With the entries that couple different axial lines removed, the
    system splits into independent lines and one zebra sweep (both
    parities) from any start is its exact solution; the point red-black
    sweep is not."""
    import scipy.sparse as sps
    L = _hier(16, 1e-2)[0]
    cp = L["cp"]
    J = L["J"].tocoo()
    keep = cp.ii[J.row // 3] == cp.ii[J.col // 3]
    Jm = sps.csr_matrix((J.data[keep], (J.row[keep], J.col[keep])), shape=J.shape)
    Lm = dict(L, J=Jm, llu=[NW.spla.splu(Jm[ix][:, ix].tocsc()) for ix in L["lidx"]],
              lu=[NW.spla.splu(Jm[ix][:, ix].tocsc()) for ix in L["idx"]])
    rng = np.random.default_rng(14)
    f = rng.normal(size=J.shape[0])
    exact = NW.spla.spsolve(Jm.tocsc(), f)
    x = rng.normal(size=f.size)
    NW.block_colour_sweep(Lm, f, x, 0, lines=True)
    NW.block_colour_sweep(Lm, f, x, 1, lines=True)
    assert np.abs(x - exact).max() <= 1e-10 * np.abs(exact).max()
    y = rng.normal(size=f.size)
    NW.block_colour_sweep(Lm, f, y, 0)
    NW.block_colour_sweep(Lm, f, y, 1)
    assert np.abs(y - exact).max() > 1e-3 * np.abs(exact).max()


def test_block_zebra_vcycle_converges_and_beats_point_smoothing():
    """The zebra cycle is a linear map, its stationary iteration converges
    to J^-1 f, and on the cos-stretched axial grid (cells much shorter in z
    than in r near the electrodes) it reduces the error faster per cycle
    than the point red-black cycle."""
    levels = _hier(16, 1e-4)
    J = levels[0]["J"]
    rng = np.random.default_rng(15)
    f = rng.normal(size=J.shape[0])
    exact = NW.spla.spsolve(J.tocsc(), f)
    errs = {}
    for lines in (False, True):
        x = np.zeros_like(f)
        e = []
        for _ in range(16):
            x += NW.block_vcycle(levels, f - J @ x, lines=lines)
            e.append(np.abs(x - exact).max() / np.abs(exact).max())
        errs[lines] = e
    assert errs[True][-1] <= 1e-10, errs[True]
    assert errs[True][5] < 0.5 * errs[False][5], (errs[True][5], errs[False][5])
    g = rng.normal(size=f.size)
    lin = NW.block_vcycle(levels, 2.0 * f - 3.0 * g, lines=True)
    ref = 2.0 * NW.block_vcycle(levels, f, lines=True) - 3.0 * NW.block_vcycle(levels, g, lines=True)
    assert np.abs(lin - ref).max() <= 1e-12 * np.abs(lin).max()
