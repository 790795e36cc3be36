"""Pins of the oracle's composite steps against facts fixed by the paper and
by mathematics: the Scharfetter-Gummel operator with a potential that varies
in r and z (Boltzmann null space of the zero-flux condition, Eqs. 8-11), its
potential derivative (Eq. 14 blocks), the composition of the decoupled
backward-Euler step (Eq. 7 with Eqs. 12-13), the time-step rule with
rejections (Sec. 2), the Newton stop measure, the multilevel prolongation of
a state and its chain (Sec. 2), and Adam's moment recurrences beyond the
first step.
"""
import numpy as np
import pytest

import oracle as O
from oracle import cnn
from oracle import newton as NW
from paper_0811_4446_amd import inputs as I


def _smooth_potential(N, z, amp=0.08, seed=0):
    """A potential that varies in both r and z (no symmetry the pins could
    hide behind): linear drop plus products of sines/cosines and noise."""
    r = np.arange(N + 1) / N
    rng = np.random.default_rng(seed)
    V = (z[None, :] + amp * np.cos(2.3 * r[:, None] + 0.4) * np.sin(3.1 * z[None, :] + 0.2)
         + 0.3 * amp * r[:, None] ** 2 * z[None, :] + 0.02 * amp * rng.normal(size=(N + 1, N + 1)))
    return np.ascontiguousarray(V)


# ---------------------------------------------------------------------------
# SG operator with V(r, z): Boltzmann null space (Eqs. 8-11)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("s,mu,D", [(-1, 100.0, 1.0), (1, 1.0, 0.01), (-1, 30.0, 0.5)])
@pytest.mark.parametrize("N", [8, 16])
def test_sg_boltzmann_state_is_annihilated(s, mu, D, N):
    """Each SG face flux D/h [n_i G(a) - n_nb F(a)] = D/h F(a) [n_i e^a - n_nb]
    vanishes exactly when n_nb/n_i = e^a, a = -s mu/D (V_nb - V_i).  So the
    Boltzmann density n = exp(-s mu/D V) carries no flux through any face, in
    r as well as in z, and the steady operator (dt = inf, S = 0) maps it to
    zero on every unknown row.  The opposite drift sign leaves a residual of
    the size of the face terms, so a sign slip in either direction fails."""
    z = I.z_cos(N)
    V = _smooth_potential(N, z, seed=N)
    q = -s * mu / D
    n = np.exp(q * (V - V.mean()))
    A = O.sg_assemble(N, N, 1.0, z, s, mu, D, 0.0, V)
    scale = np.abs(A[1] * n).max()
    res = O.apply(A, n)[:, 1:-1]
    assert np.abs(res).max() <= 1e-13 * scale, np.abs(res).max() / scale
    wrong = np.exp(-q * (V - V.mean()))
    res_w = O.apply(A, wrong)[:, 1:-1]
    assert np.abs(res_w).max() >= 1e-3 * np.abs(A[1] * wrong).max()
    # a radial-only potential: the r faces alone decide (axial differences vanish)
    r = np.arange(N + 1) / N
    Vr = np.ascontiguousarray(np.repeat((0.05 * np.sin(2.0 * r) + 0.02 * r ** 3)[:, None], N + 1, axis=1))
    nr_ = np.exp(q * Vr)
    Ar = O.sg_assemble(N, N, 1.0, z, s, mu, D, 0.0, Vr)
    assert np.abs(O.apply(Ar, nr_)[:, 1:-1]).max() <= 1e-13 * np.abs(Ar[1] * nr_).max()
    wr = np.exp(-q * Vr)
    assert np.abs(O.apply(Ar, wr)[:, 1:-1]).max() >= 1e-3 * np.abs(Ar[1] * wr).max()


@pytest.mark.parametrize("s,mu,D", [(-1, 100.0, 1.0), (1, 1.0, 0.01)])
def test_sg_potential_derivative_along_boltzmann_family(s, mu, D):
    """Along V_t = V + t w, n_t = exp(q V_t) (q = -s mu/D) the steady SG
    residual A(V_t) n_t is zero for every t, so its t-derivative vanishes:
    (dA/dV . w) n + A(V) (q w n) = 0.  This fixes the potential blocks of the
    Newton Jacobian (Eq. 14) for potentials varying in r and z, independently
    of finite differences."""
    N = 16
    z = I.z_cos(N)
    V = _smooth_potential(N, z, seed=3)
    q = -s * mu / D
    n = np.exp(q * (V - V.mean()))
    A = O.sg_assemble(N, N, 1.0, z, s, mu, D, 0.0, V)
    dV = NW._sg_dV(N, N, 1.0, z, s, mu, D, V, n)
    rng = np.random.default_rng(11)
    w = rng.normal(size=V.shape)
    lhs = O.apply(dV, w)[:, 1:-1]
    rhs = -O.apply(A, np.ascontiguousarray(q * w * n))[:, 1:-1]
    scale = np.abs(rhs).max()
    assert np.abs(lhs - rhs).max() <= 1e-11 * scale, np.abs(lhs - rhs).max() / scale


# ---------------------------------------------------------------------------
# Decoupled backward-Euler step (Eq. 7; Poisson Eqs. 12-13 with n^k first)
# ---------------------------------------------------------------------------

def test_decoupled_step_solves_each_equation_with_the_right_state():
    """or_step_decoupled: V^{k+1} solves Poisson with the charge of n^k;
    n_e^{k+1} solves the electron SG-BE equation (s = -1, mu_e, D_e, S_e,
    n_e^k) with V^{k+1}; n_p^{k+1} the ion one (s = +1, mu_p, D_p, S_p, n_p^k)
    with V^{k+1}.  Each alternative (charge of n^{k+1}, potential V^k,
    swapped species parameters or sources) leaves a residual many orders
    larger; each species balance holds with V^{k+1}."""
    N, dt = 16, 1e-2
    z = I.z_cos(N)
    ph = dict(I.PHYS)
    rng = np.random.default_rng(4)
    ne_k = I.initial_density(N, N, 2) * (1 + 50 * rng.random((N + 1, N + 1)))
    np_k = ne_k * (1 + 0.5 * rng.random((N + 1, N + 1)))
    ne_k[:, 0] = ne_k[:, -1] = np_k[:, 0] = np_k[:, -1] = 0.0
    V_k = _smooth_potential(N, z, amp=0.05, seed=9)
    V_k[:, 0], V_k[:, -1] = 0.0, 1.0
    Se = I.source(N, N, z)
    Sp = 0.7 * I.source(N, N, z, zc=0.4)
    V, ne, np_ = V_k.copy(), ne_k.copy(), np_k.copy()
    code, cyc, rr = O.step_decoupled(1.0, z, O.Phys(**ph), V, ne, np_, Se, Sp, dt, coarsest=4, rtol=1e-12)
    assert code == 0, (code, cyc, rr)
    assert np.abs(V - V_k).max() > 1e-3  # the potential moved, so V^k and V^{k+1} are distinguishable

    def rr_poisson(nE, nP):
        return O.relres(1.0, z, O.poisson_assemble(N, N, 1.0, z, ph["k"], nE, nP), V)

    def rr_sg(x, s, mu, D, Vv, nk, S):
        return O.relres(1.0, z, O.sg_assemble(N, N, 1.0, z, s, mu, D, 1.0 / dt, Vv, nk, S), x)

    assert rr_poisson(ne_k, np_k) <= 1e-11
    assert rr_poisson(ne, np_) >= 1e-6
    assert rr_sg(ne, -1, ph["mu_e"], ph["D_e"], V, ne_k, Se) <= 1e-11
    assert rr_sg(np_, 1, ph["mu_p"], ph["D_p"], V, np_k, Sp) <= 1e-11
    for bad in (rr_sg(ne, -1, ph["mu_e"], ph["D_e"], V_k, ne_k, Se),
                rr_sg(ne, -1, ph["mu_p"], ph["D_p"], V, ne_k, Se),
                rr_sg(ne, 1, ph["mu_e"], ph["D_e"], V, ne_k, Se),
                rr_sg(ne, -1, ph["mu_e"], ph["D_e"], V, ne_k, Sp),
                rr_sg(np_, 1, ph["mu_p"], ph["D_p"], V_k, np_k, Sp),
                rr_sg(np_, 1, ph["mu_e"], ph["D_e"], V, np_k, Sp)):
        assert bad >= 1e-6, bad
    # species balance (Eq. 7 summed over the domain) with the fluxes of V^{k+1}
    from tests.test_oracle_pins import _electrode_outflow
    vol = O.volumes(N, N, 1.0, z)
    for n, nk, S, s, mu, D in ((ne, ne_k, Se, -1, ph["mu_e"], ph["D_e"]), (np_, np_k, Sp, 1, ph["mu_p"], ph["D_p"])):
        lhs = (vol * ((n - nk) / dt - S))[:, 1:-1].sum()
        out = _electrode_outflow(1.0, z, s, mu, D, V, n)
        assert abs(lhs + out) <= 1e-8 * np.abs(vol * S).sum(), (s, lhs, out)


# ---------------------------------------------------------------------------
# Newton stop measure and the time-step rule with rejections (Sec. 2)
# ---------------------------------------------------------------------------

def test_newton_stop_measure_counts_unknown_rows_only():
    """The Newton stop test is the relative l1 size of each field's
    correction over the unknown nodes: sum |du| / sum |u| over j = 1..nz-1
    (the electrode rows are fixed and enter neither sum)."""
    N = 8
    z = I.z_cos(N)
    ph = dict(I.PHYS, V_top=5.0)
    cp = NW.Coupled(N, N, 1.0, z, ph)
    ne = I.initial_density(N, N, 1)
    np_ = ne * 1.2
    V = I.initial_potential(N, N, z, 0.0, 5.0)
    S = I.source(N, N, z)
    u0 = [a.copy() for a in (ne, np_, V)]
    hist = []
    NW.newton_step(cp, V, ne, np_, S, S, 1e-3, max_newton=1, tol=0.0, history=hist)
    want = [np.abs((a - b)[:, 1:-1]).sum() / np.abs(a[:, 1:-1]).sum() for a, b in zip((ne, np_, V), u0)]
    assert np.allclose(hist[0], want, rtol=1e-14, atol=0)
    # the electrode row V = 5 would change the potential's measure noticeably
    whole = np.abs((V - u0[2])).sum() / np.abs(V).sum()
    assert abs(whole - want[2]) > 0.05 * want[2]


def test_time_step_rule_with_rejections():
    """Sec. 2: after an accepted step dt grows (x1.5, capped); a rejected step
    is retried with the last accepted dt, or, when it already was that dt (or
    none was accepted yet), with half of it.  Rejections leave the state
    untouched: replaying the accepted dt sequence with a generous Newton
    budget reproduces the final state bit for bit."""
    N = 8
    z = I.z_cos(N)
    ph = dict(I.PHYS)
    cp = NW.Coupled(N, N, 1.0, z, ph)
    ne0 = I.initial_density(N, N, 0)
    V0 = I.initial_potential(N, N, z)
    S = I.source(N, N, z)
    V, ne, np_ = V0.copy(), ne0.copy(), ne0.copy()
    att = []
    acc, rej, seq = NW.steady(cp, V, ne, np_, S, S, dt0=1e-2, max_newton=3, max_steps=30, attempts=att)
    assert acc == 30 and rej == len(att) - 30 and rej >= 10
    dt_acc, growth, dt_max = 0.0, 1.5, 0.1
    halvings_after_retry = 0
    for (dt, ok), (dt_next, _) in zip(att, att[1:]):
        if ok:
            assert dt_next == min(growth * dt, dt_max)
            dt_acc = dt
        else:
            if dt_acc > 0 and dt > dt_acc:
                assert dt_next == dt_acc
            else:
                assert dt_next == 0.5 * dt
                halvings_after_retry += dt_acc > 0
    assert halvings_after_retry >= 1  # the "retry failed too" branch ran
    assert seq == [dt for dt, ok in att if ok]
    V2, ne2, np2 = V0.copy(), ne0.copy(), ne0.copy()
    NW.steady(cp, V2, ne2, np2, S, S, dts=seq, max_newton=10)
    for a, b in ((V, V2), (ne, ne2), (np_, np2)):
        assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# Multilevel prolongation of a state and the chain (Sec. 2)
# ---------------------------------------------------------------------------

def test_prolong_state_is_exact_on_bilinear_fields_and_sets_electrodes():
    """The prolongation interpolates linearly in r between radial parents and
    linearly in z (distance weights) between axial parents, so a field that is
    bilinear in (r, z) on the coarse nodes is reproduced exactly on the fine
    unknown rows; the electrode rows carry the boundary values."""
    Nc = 8
    zf = I.z_cos(2 * Nc)
    zc = zf[::2]
    rc, rf = np.arange(Nc + 1) / Nc, np.arange(2 * Nc + 1) / (2 * Nc)
    f = lambda r, z, c: c[0] + c[1] * r + c[2] * z + c[3] * r * z
    cs = [(0.3, -1.0, 2.0, 0.5), (1e-3, 2e-3, -1e-3, 4e-3), (2.0, 0.0, 0.0, -3.0)]
    coarse = [np.ascontiguousarray(f(rc[:, None], zc[None, :], c)) for c in cs]
    ph = dict(I.PHYS, V_top=2.5, ne_top=0.25)
    Vf, nef, npf = NW.prolong_state(zf, *coarse, ph)
    for got, c in zip((Vf, nef, npf), cs):
        want = f(rf[:, None], zf[None, :], c)
        assert np.abs(got[:, 1:-1] - want[:, 1:-1]).max() <= 1e-14 * np.abs(want).max()
    assert np.all(Vf[:, 0] == 0.0) and np.all(Vf[:, -1] == 2.5)
    assert np.all(nef[:, 0] == 0.0) and np.all(nef[:, -1] == 0.25) and np.all(npf[:, -1] == 0.0)
    # coarse nodes are copied, not averaged
    assert np.array_equal(Vf[::2, 2:-1:2], coarse[0][:, 1:-1])


def test_chain_reaches_the_steady_state_of_the_direct_run():
    """M+L: the 9x9 steady state prolonged to 17x17 and run to steady there
    ends at the same steady state as the 17x17 run from the random start
    (both polished by steady Newton, dt = inf), and the 17x17 stage needs
    fewer steps than the run from the random start."""
    phys = dict(I.PHYS)
    (V, ne, np_), stages = NW.chain(1.0, I.z_cos, phys, 8, 16, I.initial_potential(8, 8, I.z_cos(8)),
                                    I.initial_density(8, 8, 0), I.initial_density(8, 8, 0),
                                    lambda N, z: I.source(N, N, z), tol=1e-8)
    assert [s[0] for s in stages] == [8, 16]
    N = 16
    z = I.z_cos(N)
    cp = NW.Coupled(N, N, 1.0, z, phys)
    S = I.source(N, N, z)
    V2, ne2 = I.initial_potential(N, N, z), I.initial_density(N, N, 0)
    np2 = ne2.copy()
    acc, _, _ = NW.steady(cp, V2, ne2, np2, S, S, tol=1e-8)
    assert stages[1][1] < acc
    for st in ((V, ne, np_), (V2, ne2, np2)):
        for _ in range(4):
            NW.newton_step(cp, *st, S, S, np.inf, tol=1e-14)
    for a, b in ((V, V2), (ne, ne2), (np_, np2)):
        assert np.abs(a - b).max() <= 1e-10 * np.abs(b).max()


# ---------------------------------------------------------------------------
# Adam (the optimiser of the warm-start network) beyond the first step
# ---------------------------------------------------------------------------

def test_adam_moment_recurrences_steps_two_and_three():
    """Adam: m_t = b1 m_{t-1} + (1-b1) g_t, v_t = b2 v_{t-1} + (1-b2) g_t^2,
    step lr * (m_t/(1-b1^t)) / (sqrt(v_t/(1-b2^t)) + eps).  With gradients
    g, -g, g (|g| constant) the bias-corrected second moment is g^2 at every
    t, and the first moments are worked out by hand:
      t=2: m = 0.09 g - 0.1 g = -0.01 g,  m/(1-0.81)  = -(1/19) g
      t=3: m = -0.009 g + 0.1 g = 0.091 g, m/(1-0.729) = (91/271) g
    so the parameter moves by -lr sign(g), +lr/19 sign(g), -lr 91/271 sign(g).
    A constant gradient moves it by lr sign(g) at every step."""
    lr = 1e-3
    g = np.array([0.25, -3.0, 7.5])
    p0 = np.array([1.0, -2.0, 0.5])
    p, m, v = p0.copy(), np.zeros(3), np.zeros(3)
    steps = []
    for t, sgn in ((1, 1.0), (2, -1.0), (3, 1.0)):
        before = p.copy()
        cnn.adam(p, sgn * g, m, v, t, lr=lr, eps=0.0)
        steps.append(p - before)
    sg = np.sign(g)
    # (p - before) loses about 1e-16/|step| relative to the subtraction: rtol 1e-9
    assert np.allclose(steps[0], -lr * sg, rtol=1e-9, atol=0)
    assert np.allclose(steps[1], lr / 19.0 * sg, rtol=1e-9, atol=0)
    assert np.allclose(steps[2], -lr * 91.0 / 271.0 * sg, rtol=1e-9, atol=0)
    assert np.allclose(m, 0.091 * g, rtol=1e-13) and np.allclose(v, 0.001 * (1 + 0.999 + 0.998001) * g * g, rtol=1e-13)
    p, m, v = p0.copy(), np.zeros(3), np.zeros(3)
    for t in (1, 2, 3):
        cnn.adam(p, g, m, v, t, lr=lr, eps=0.0)
    assert np.allclose(p, p0 - 3 * lr * sg, rtol=0, atol=1e-15)
