"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Both sides get the same seeded inputs from paper_0811_4446_amd.inputs; the
oracle shares no code with the library.  FP64 tolerance: 1e-12 relative to
the field's maximum (the GPU contracts a*b+c into FMA and sums in another
order, so results agree to rounding, not bitwise).
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_0811_4446_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def M():
    from paper_0811_4446_amd import mgfluid
    return mgfluid


def relmax(a, b):
    scale = max(np.abs(b).max(), 1e-300)
    return np.abs(a - b).max() / scale


def _problem(nr, nz, seed=0, vtop=1.0, pert=0.0):
    z = I.z_cos(nz)
    ne = I.initial_density(nr, nz, seed)
    np_ = ne.copy()
    S = np.ascontiguousarray(I.source(nr, nz, z))
    V = np.ascontiguousarray(I.initial_potential(nr, nz, z, 0.0, vtop))
    if pert:
        rng = np.random.default_rng(seed + 100)
        V[:, 1:-1] += pert * rng.normal(size=(nr + 1, nz - 1))
        ne = ne * (1 + 50 * rng.random(ne.shape))
        np_ = np_ * (1 + 50 * rng.random(ne.shape))
    phys = dict(I.PHYS)
    phys["V_top"] = vtop
    return z, V, ne, np_, S, phys


EQS = [("poisson", 0), ("electron", 1), ("ion", 2)]


def _assemble_both(m, sol, eq, z, V, ne, np_, S, phys, dt, smoother):
    nr, nz = V.shape[0] - 1, V.shape[1] - 1
    mg = O.MG(nr, nz, 1.0, z, coarsest=8, smoother=smoother)
    tV, tne, tnp, tS = sol.upload(V), sol.upload(ne), sol.upload(np_), sol.upload(S)
    st = sol.state(tV, tne, tnp, tS, tS)
    P = m.Physics.of(phys)
    sol.assemble(eq, P, st, dt)
    dt_inv = 0.0 if not math.isfinite(dt) else 1.0 / dt
    if eq == 0:
        mg.assemble_poisson(phys["k"], ne, np_)
    elif eq == 1:
        mg.assemble_sg(-1, phys["mu_e"], phys["D_e"], dt_inv, V, ne, S)
    else:
        mg.assemble_sg(+1, phys["mu_p"], phys["D_p"], dt_inv, V, np_, S)
    return mg, (tV, tne, tnp, tS), st


@pytest.mark.parametrize("nr,nz", [(64, 64), (32, 128), (128, 64), (256, 256)])
@pytest.mark.parametrize("name,eq", EQS)
def test_assembly_all_levels(nr, nz, name, eq):
    """sg_assemble vs the oracle's Eq. (12)-(13) / Eq. (7)-(11) rows on every
    level (coarse levels rediscretised with the injected potential)."""
    m = M()
    _say("assembly", name, nr, nz)
    z, V, ne, np_, S, phys = _problem(nr, nz, seed=1, vtop=2.0, pert=0.05)
    sol = m.Solver(nr, nz, z)
    mg, _, _ = _assemble_both(m, sol, eq, z, V, ne, np_, S, phys, 1e-3, O.SMOOTH_ZEBRA)
    assert sol.nlev == mg.nlev
    for lvl in range(mg.nlev):
        ref = mg.coef(lvl)
        for w in range(6):
            if lvl > 0 and w == 5:
                continue  # coarse right-hand sides are restricted residuals
            got = sol.coef(eq, lvl, w)
            err = np.abs(got - ref[w])
            bound = 1e-13 * np.abs(ref[w]) + 1e-15 * np.abs(ref[w]).max()
            assert (err <= bound).all(), (lvl, "abcdef"[w], err.max(), np.abs(ref[w]).max())


@pytest.mark.parametrize("smoother", [0, 1])
@pytest.mark.parametrize("name,eq", EQS)
@pytest.mark.parametrize("N", [64, 256])
def test_half_sweeps_and_residual(smoother, name, eq, N):
    """One red/black (point) or even/odd (z-line) half-sweep, then the residual."""
    m = M()
    _say("half-sweep", smoother, name, N)
    z, V, ne, np_, S, phys = _problem(N, N, seed=2, vtop=1.0, pert=0.02)
    sol = m.Solver(N, N, z, smoother=smoother)
    mg, (tV, tne, tnp, tS), st = _assemble_both(m, sol, eq, z, V, ne, np_, S, phys, 1e-3, smoother)
    coef = mg.coef(0)
    rng = np.random.default_rng(9)
    x = rng.random((N + 1, N + 1))
    x[:, 0] = 0.0 if eq else phys["V_bottom"]
    x[:, -1] = 0.0 if eq else phys["V_top"]
    tx = sol.upload(x)
    for colour in (0, 1):
        sol.smooth_half(eq, tx, colour)
        if smoother == 0:
            O.rbgs(coef, x, colour)
        else:
            O.zline(coef, x, colour)
        got = sol.download(tx)
        assert relmax(got, x) <= TOL, (colour, relmax(got, x))
    tr = sol.field()
    sol.residual(eq, tx, tr)
    r_ref = O.residual(coef, x)
    # f - A x cancels: measure against the size of the terms
    scale = np.abs(coef[1]).max() * np.abs(x).max() + np.abs(coef[5]).max()
    assert np.abs(sol.download(tr) - r_ref).max() <= 1e-13 * scale


@pytest.mark.parametrize("smoother", [0, 1])
@pytest.mark.parametrize("name,eq", EQS)
@pytest.mark.parametrize("nr,nz", [(64, 64), (16, 64), (128, 32)])
def test_vcycle_iterates(smoother, name, eq, nr, nz):
    """The V(2,2) iterates agree cycle by cycle, and so does the relative residual."""
    m = M()
    _say("vcycle", smoother, name, nr, nz)
    z, V, ne, np_, S, phys = _problem(nr, nz, seed=3, vtop=1.5, pert=0.05)
    sol = m.Solver(nr, nz, z, smoother=smoother)
    mg, (tV, tne, tnp, tS), st = _assemble_both(m, sol, eq, z, V, ne, np_, S, phys, 1e-2, smoother)
    x = (V if eq == 0 else (ne if eq == 1 else np_)).copy()
    tx = sol.upload(x)
    for k in range(6):
        rr = sol.vcycle(eq, tx, 1, want_relres=True)
        mg.vcycle(x)
        got = sol.download(tx)
        assert relmax(got, x) <= TOL, (k, relmax(got, x))
        rr_ref = mg.relres(x)
        assert abs(rr - rr_ref) <= 1e-6 * rr_ref + 1e-15, (k, rr, rr_ref)


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("smoother", [0, 1])
def test_implicit_step_decoupled_65(seed, smoother):
    """One backward-Euler step at 65x65 (dt = 1e-4): Poisson with n^k, then
    SG electrons and ions, each by V(2,2) cycles to relative residual 1e-10."""
    m = M()
    _say("implicit_step", seed, smoother)
    N = 64
    z = I.z_cos(N)
    ne = I.initial_density(N, N, seed)
    np_ = ne.copy()
    S = I.source(N, N, z)
    V = I.initial_potential(N, N, z, 0.0, 1.0)
    phys = dict(I.PHYS)
    # oracle
    Vo, neo, npo = V.copy(), ne.copy(), np_.copy()
    st_o, cyc_o, rr_o = O.step_decoupled(1.0, z, O.Phys(**phys), Vo, neo, npo, S, S, 1e-4,
                                         smoother=smoother, rtol=1e-10)
    assert st_o == 0
    # GPU
    sol = m.Solver(N, N, z, smoother=smoother)
    tV, tne, tnp, tS = sol.upload(V), sol.upload(ne), sol.upload(np_), sol.upload(S)
    st = sol.state(tV, tne, tnp, tS, tS)
    rep = sol.step(m.Physics.of(phys), st, 1e-4, m.schedule(lin_rtol=1e-10, max_cycles=500))
    assert rep.vcycles == sum(cyc_o), (rep.vcycles, cyc_o)
    for t, ref in ((tV, Vo), (tne, neo), (tnp, npo)):
        assert relmax(sol.download(t), ref) <= TOL
    assert (sol.download(tne) >= 0).all() and (sol.download(tnp) >= 0).all()


def test_full_size_1025_electron_solve():
    """1025x1025 nodes (the mixed-precision workload's grid): six zebra V(2,2)
    cycles of the electron SG equation agree with the oracle everywhere."""
    m = M()
    N = 1024
    _say("full size", N)
    z, V, ne, np_, S, phys = _problem(N, N, seed=4, vtop=1.0, pert=0.01)
    sol = m.Solver(N, N, z, smoother=1)
    mg, (tV, tne, tnp, tS), st = _assemble_both(m, sol, 1, z, V, ne, np_, S, phys, 1e-2, 1)
    x = ne.copy()
    tx = sol.upload(x)
    sol.vcycle(1, tx, 6)
    for _ in range(6):
        mg.vcycle(x)
    assert relmax(sol.download(tx), x) <= TOL


@pytest.mark.parametrize("N,coarsest", [(8, 8), (4, 2), (16, 2)])
def test_small_grids_direct_and_dense(N, coarsest):
    """Edge cases: the finest grid is the coarsest (pure direct solve) and
    tiny hierarchies; the solution equals numpy's dense LU."""
    m = M()
    _say("small", N, coarsest)
    z, V, ne, np_, S, phys = _problem(N, N, seed=5, vtop=1.0, pert=0.1)
    sol = m.Solver(N, N, z, coarsest=coarsest, smoother=1)
    tV, tne, tnp, tS = sol.upload(V), sol.upload(ne), sol.upload(np_), sol.upload(S)
    st = sol.state(tV, tne, tnp, tS, tS)
    sol.assemble(1, m.Physics.of(phys), st, 1e-3)
    mg = O.MG(N, N, 1.0, z, coarsest=coarsest, smoother=1)
    mg.assemble_sg(-1, phys["mu_e"], phys["D_e"], 1e3, V, ne, S)
    ref = ne.copy()
    O.direct_solve(mg.coef(0), ref)
    cyc, rr = sol.solve(1, tne, rtol=1e-14, max_cycles=60)
    assert relmax(sol.download(tne), ref) <= TOL


@pytest.mark.parametrize("name,eq", EQS)
@pytest.mark.parametrize("nr,nz,prec", [(64, 64, 0), (256, 256, 0), (128, 32, 0), (128, 128, 1)])
def test_fused_scalar_vcycle_matches_half_sweeps(name, eq, nr, nz, prec, monkeypatch):
    """Red-black V(2,2) cycles built from one-launch sweeps (zero-guess first
    sweep, prolongation on read, residual + restriction in one launch, the
    coarse levels in one workgroup staged in LDS) give bitwise the iterates
    of the per-step launches (half-sweeps, residual, restriction, fill,
    prolongation, per-level coarse end), in FP64 and in FP32 refinement."""
    m = M()
    _say("fused scalar vcycle", name, nr, nz, prec)
    z, V, ne, np_, S, phys = _problem(nr, nz, seed=4, vtop=1.0, pert=0.02)
    out = {}
    for half in (1, 0):
        if half:
            monkeypatch.setenv("MGF_HALF_SWEEPS", "1")
        else:
            monkeypatch.delenv("MGF_HALF_SWEEPS", raising=False)
        sol = m.Solver(nr, nz, z, smoother=0, prec=prec)
        tV, tne, tnp, tS = sol.upload(V), sol.upload(ne), sol.upload(np_), sol.upload(S)
        st = sol.state(tV, tne, tnp, tS, tS)
        sol.assemble(eq, m.Physics.of(phys), st, 1e-3)
        x = (tV, tne, tnp)[eq].clone()
        its = []
        for k in range(4):
            sol.vcycle(eq, x, 1)
            its.append(sol.download(x))
        out[half] = its
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)
