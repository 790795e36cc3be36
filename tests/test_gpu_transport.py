"""Field-dependent transport (Sec. 2: mobilities and diffusion coefficients
as functions of the field from lookup tables; in hybrid models supplied by
a Monte Carlo code after every cycle) against the oracle: node-transport
assembly on every level, the table lookup, Newton steps and the block
V-cycle with node transport, the boundary flow, and two cycles of the
hybrid loop (table lookup from the current field, then the steady fluid
solve warm-started from the previous state)."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle as O
from oracle import newton as NW
from paper_0811_4446_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def M():
    from paper_0811_4446_amd import mgfluid
    return mgfluid


def relmax(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _state_tr(N, seed):
    """Random densities; a smooth potential perturbation, so that the
    electron transport from the table varies smoothly like a field-driven
    coefficient does; smooth ion transport."""
    z = I.z_cos(N)
    r = np.arange(N + 1) / N
    rng = np.random.default_rng(seed)
    ne = I.initial_density(N, N, seed) * (1 + 50 * rng.random((N + 1, N + 1)))
    np_ = ne * (1 + 0.3 * rng.random((N + 1, N + 1)))
    ne[:, 0] = ne[:, -1] = np_[:, 0] = np_[:, -1] = 0
    c = rng.uniform(0.5, 1.5, 3)
    V = np.ascontiguousarray(I.initial_potential(N, N, z)
                             + 0.2 * c[0] * np.cos(c[1] * r[:, None]) * np.sin(np.pi * z[None, :]))
    Et, mut, Dt = I.electron_transport_table()
    mue, De = NW.transport_from_table(1.0, z, V, Et, mut, Dt)
    bump = np.cos(c[2] * r[:, None]) * (1 + 0.5 * z[None, :])
    tr = dict(mue=mue, De=De, mup=np.ascontiguousarray(1.0 + 0.2 * bump), Dp=np.ascontiguousarray(0.01 * (1 + 0.3 * bump)))
    return z, V, ne, np_, I.source(N, N, z), tr


@pytest.mark.parametrize("eq", [1, 2])
def test_node_transport_assembly_all_levels(eq):
    _say("node transport assembly", eq)
    m = M()
    N = 64
    z, V, ne, np_, S, tr = _state_tr(N, 1)
    ph = dict(I.PHYS)
    sol = m.Solver(N, N, z)
    t = [sol.upload(a) for a in (V, ne, np_, S)]
    tt = {k: sol.upload(v) for k, v in tr.items()}
    st = sol.state(t[0], t[1], t[2], t[3], t[3], tt["mue"], tt["De"], tt["mup"], tt["Dp"])
    sol.assemble(eq, m.Physics.of(ph), st, 1e-3)
    mg = O.MG(N, N, 1.0, z, coarsest=8)
    if eq == 1:
        mg.assemble_sg(-1, 0.0, 1.0, 1e3, V, ne, S, mun=tr["mue"], Dn=tr["De"])
    else:
        mg.assemble_sg(1, 0.0, 1.0, 1e3, V, np_, S, mun=tr["mup"], Dn=tr["Dp"])
    for lvl in range(mg.nlev):
        ref = mg.coef(lvl)
        for w in range(6):
            if lvl > 0 and w == 5:
                continue
            err = np.abs(sol.coef(eq, lvl, w) - ref[w])
            assert (err <= 1e-13 * np.abs(ref[w]) + 1e-15 * np.abs(ref[w]).max()).all(), (lvl, w, err.max())


def test_transport_table_matches_oracle():
    _say("transport table")
    m = M()
    N = 64
    z, V, _, _, _, _ = _state_tr(N, 2)
    sol = m.Solver(N, N, z)
    Et, mut, Dt = I.electron_transport_table()
    mu_o, D_o = sol.field(np.nan), sol.field(np.nan)
    sol.transport_table(sol.upload(V), _dev(Et), _dev(mut), _dev(Dt), mu_o, D_o)
    want_mu, want_D = NW.transport_from_table(1.0, z, V, Et, mut, Dt)
    assert relmax(sol.download(mu_o), want_mu) <= 1e-13
    assert relmax(sol.download(D_o), want_D) <= 1e-13


@pytest.mark.parametrize("N,dt", [(32, 1e-3), (64, 1e-2)])
def test_node_transport_newton_step_matches_oracle(N, dt):
    _say("node transport newton", N, dt)
    m = M()
    z, V, ne, np_, S, tr = _state_tr(N, 3)
    ph = dict(I.PHYS)
    sol = m.Solver(N, N, z, krylov_m=20, coarsest=4)
    t = [sol.upload(a) for a in (V, ne, np_, S)]
    tt = {k: sol.upload(v) for k, v in tr.items()}
    st = sol.state(t[0], t[1], t[2], t[3], t[3], tt["mue"], tt["De"], tt["mup"], tt["Dp"])
    cp = NW.Coupled(N, N, 1.0, z, ph, transport=tr)
    ok, its = NW.newton_step(cp, V, ne, np_, S, S, dt, max_newton=20, tol=1e-11)
    assert ok
    sc = m.schedule(coupling=m.NEWTON, lin_rtol=1e-13, max_cycles=400, max_newton=20, newton_tol=1e-11)
    rep = sol.step(m.Physics.of(ph), st, dt, sc)
    assert rep.newton_its == its, (rep.newton_its, its)
    errs = [relmax(sol.download(x), r) for x, r in zip(t[:3], (V, ne, np_))]
    print("node transport newton %d: max rel err %s" % (N, errs))
    assert max(errs) <= 1e-12, errs
    flows = sol.boundary_flow(m.Physics.of(ph), st)
    want = list(NW.boundary_flow(1.0, z, -1, 0.0, 1.0, V, ne, mun=tr["mue"], Dn=tr["De"])) + \
        list(NW.boundary_flow(1.0, z, 1, 0.0, 1.0, V, np_, mun=tr["mup"], Dn=tr["Dp"]))
    for g_, w_ in zip(flows, want):
        assert abs(g_ - w_) <= 1e-9 * max(abs(x) for x in want), (flows, want)


def test_node_transport_block_vcycle_matches_oracle():
    _say("node transport block vcycle")
    m = M()
    N, dt = 64, 0.1
    z, V, ne, np_, S, tr = _state_tr(N, 4)
    ph = dict(I.PHYS)
    sol = m.Solver(N, N, z, coarsest=4, krylov_m=10)
    t = [sol.upload(a) for a in (V, ne, np_, S)]
    tt = {k: sol.upload(v) for k, v in tr.items()}
    st = sol.state(t[0], t[1], t[2], t[3], t[3], tt["mue"], tt["De"], tt["mup"], tt["Dp"])
    levels = NW.block_hierarchy(N, N, 1.0, z, ph, V, ne, np_, dt, coarsest=4, transport=tr)
    rng = np.random.default_rng(6)
    planes = [rng.normal(size=(N + 1, N + 1)) for _ in range(3)]
    for p_ in planes:
        p_[:, 0] = p_[:, -1] = 0.0
    r, zt = sol.field3(), sol.field3()
    for k in range(3):
        r[k, :, : N + 1] = torch.from_numpy(planes[k]).to(r.device)
    sol.precond(m.Physics.of(ph), st, dt, r, zt)
    torch.cuda.synchronize()
    got = zt[:, :, : N + 1].cpu().numpy()
    want = levels[0]["cp"].unpack(NW.block_vcycle(levels, levels[0]["cp"].pack(*planes)))
    errs = [np.abs(got[k] - want[k]).max() / np.abs(want[k]).max() for k in range(3)]
    assert max(errs) <= 1e-12, errs


def test_hybrid_loop_two_cycles_matches_oracle():
    """Cycle 0: steady with the constant transport from the random start;
    cycles 1 and 2: electron transport from the table at the current field,
    then the steady solve warm-started from the previous steady state."""
    _say("hybrid loop")
    m = M()
    N = 16
    z = I.z_cos(N)
    ph = dict(I.PHYS)
    P = m.Physics.of(ph)
    Et, mut, Dt = I.electron_transport_table()
    kw = dict(dt0=1e-3, growth=1.5, dt_max=0.1, tol=1e-8, newton_tol=1e-10)
    sc = m.schedule(coupling=m.NEWTON, dt0=1e-3, growth=1.5, dt_max=0.1, steady_tol=1e-8, lin_rtol=1e-12,
                    max_cycles=400, newton_tol=1e-10)
    S = I.source(N, N, z)
    ne0 = I.initial_density(N, N, 0)
    V0 = I.initial_potential(N, N, z)
    # oracle
    V, ne, np_ = V0.copy(), ne0.copy(), ne0.copy()
    steps_or = []
    tr = None
    for cyc in range(3):
        cp = NW.Coupled(N, N, 1.0, z, ph, transport=tr)
        steps_or.append(NW.steady(cp, V, ne, np_, S, S, **kw)[0])
        mue, De = NW.transport_from_table(1.0, z, V, Et, mut, Dt)
        tr = dict(mue=mue, De=De, mup=np.full_like(V, ph["mu_p"]), Dp=np.full_like(V, ph["D_p"]))
    # library
    sol = m.Solver(N, N, z, krylov_m=20, coarsest=4)
    t = [sol.upload(a) for a in (V0, ne0, ne0.copy(), S)]
    mu_d, D_d = sol.field(), sol.field()
    mup, Dp = sol.field(ph["mu_p"]), sol.field(ph["D_p"])
    tab = [_dev(a) for a in (Et, mut, Dt)]
    steps = []
    for cyc in range(3):
        if cyc == 0:
            st = sol.state(t[0], t[1], t[2], t[3], t[3])
        else:
            st = sol.state(t[0], t[1], t[2], t[3], t[3], mu_d, D_d, mup, Dp)
        code, rep = sol.steady(P, st, sc)
        assert code == 0
        steps.append(rep.steps)
        sol.transport_table(t[0], *tab, mu_d, D_d)
    assert steps == steps_or, (steps, steps_or)
    errs = [relmax(sol.download(x), r) for x, r in zip(t[:3] + [mu_d], (V, ne, np_, tr["mue"]))]
    print("hybrid loop: steps per cycle %s, max rel err %s" % (steps, errs))
    assert max(errs) <= 1e-9, errs
