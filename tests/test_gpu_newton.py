"""Parity of the coupled Newton path (Sec. 2, Eq. 14) with the oracle: one
backward-Euler step, and whole steady runs with the paper's time-step rule
(the oracle solves each Newton system by sparse LU; the library by FGMRES
preconditioned with a block V-cycle, iterated to the same tolerance)."""
import sys

import numpy as np
import pytest

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


def _gpu(N, V, ne, np_, S, krylov_m=20, smoother=1, prec=None):
    m = M()
    z = I.z_cos(N)
    sol = m.Solver(N, N, z, smoother=smoother, krylov_m=krylov_m, prec=m.FP64 if prec is None else prec)
    t = [sol.upload(V), sol.upload(ne), sol.upload(np_), sol.upload(S)]
    st = sol.state(t[0], t[1], t[2], t[3], t[3])
    return sol, t, st


def _start(N, seed=0):
    z = I.z_cos(N)
    ne = I.initial_density(N, N, seed)
    return z, I.initial_potential(N, N, z), ne, ne.copy(), I.source(N, N, z)


@pytest.mark.parametrize("N,dt,pre", [(16, 1e-4, 0), (32, 1e-4, 0), (32, 1e-3, 12), (64, 0.1, 25)])
def test_newton_step_matches_oracle(N, dt, pre):
    """One BE step from the initial state (or after `pre` oracle steps of the
    steady schedule): same Newton iterates within FP64 rounding."""
    _say("newton step", N, dt, pre)
    m = M()
    z, V, ne, np_, S = _start(N)
    ph = dict(I.PHYS)
    cp = NW.Coupled(N, N, 1.0, z, ph)
    if pre:
        NW.steady(cp, V, ne, np_, S, S, max_steps=pre)
    sol, t, st = _gpu(N, V, ne, np_, S)
    hist = []
    ok, its = NW.newton_step(cp, V, ne, np_, S, S, dt, max_newton=20, tol=1e-11, history=hist)
    assert ok
    sc = m.schedule(coupling=m.NEWTON, lin_rtol=1e-13, max_cycles=400, max_newton=20, newton_tol=1e-11)
    rep = sol.step(m.Physics.of(ph), st, dt, sc)
    assert rep.newton_its == its, (rep.newton_its, its)
    errs = [relmax(sol.download(tt), ref) for tt, ref in zip(t[:3], (V, ne, np_))]
    print("newton step %s dt %g: max rel err %s" % (N, dt, errs))
    assert max(errs) <= 1e-12, errs


def test_relaxation_only_preconditioner_matches_oracle(monkeypatch):
    """The relaxation-only preconditioner (red-black sweeps on the finest
    grid, no coarse correction; the plain-relaxation curve of the Fig. 1
    measurement) changes the linear-solver path, not the Newton iterates:
    one BE step at 33x33 equals the oracle's within FP64 rounding."""
    _say("relaxation-only preconditioner", 32)
    m = M()
    N, dt = 32, 1e-3
    z, V, ne, np_, S = _start(N)
    ph = dict(I.PHYS)
    cp = NW.Coupled(N, N, 1.0, z, ph)
    monkeypatch.setenv("MGF_SMOOTHER_ONLY", "1")
    sol, t, st = _gpu(N, V, ne, np_, S, krylov_m=30)
    monkeypatch.delenv("MGF_SMOOTHER_ONLY", raising=False)
    ok, its = NW.newton_step(cp, V, ne, np_, S, S, dt, max_newton=20, tol=1e-11)
    assert ok
    sc = m.schedule(coupling=m.NEWTON, lin_rtol=1e-13, max_cycles=20000, max_newton=20, newton_tol=1e-11)
    rep = sol.step(m.Physics.of(ph), st, dt, sc)
    assert rep.newton_its == its, (rep.newton_its, its)
    for tt, ref in zip(t[:3], (V, ne, np_)):
        assert relmax(sol.download(tt), ref) <= 1e-12
    # without the coarse correction the linear solves need more iterations
    base, tb, stb = _gpu(N, *_start(N)[1:], krylov_m=30)
    rb = base.step(m.Physics.of(ph), stb, dt, sc)
    assert rep.vcycles > rb.vcycles, (rep.vcycles, rb.vcycles)


@pytest.mark.parametrize("N,dt,pre,prec_name", [(32, 1e-3, 12, "FP64"), (64, 0.1, 25, "FP64"),
                                                 (64, 0.1, 25, "FP32_IR")])
def test_newton_step_block_zebra_matches_oracle(N, dt, pre, prec_name):
    """One BE step with the block zebra z-line preconditioner (FP64 or FP32
    cycles; FGMRES and Newton in FP64): the oracle's exact Newton iterates,
    same iteration count, within 1e-12."""
    _say("newton step zebra", N, dt, pre, prec_name)
    m = M()
    z, V, ne, np_, S = _start(N)
    ph = dict(I.PHYS)
    cp = NW.Coupled(N, N, 1.0, z, ph)
    if pre:
        NW.steady(cp, V, ne, np_, S, S, max_steps=pre)
    sol, t, st = _gpu(N, V, ne, np_, S, smoother=m.SMOOTH_ZEBRA_BLOCK, prec=getattr(m, prec_name))
    ok, its = NW.newton_step(cp, V, ne, np_, S, S, dt, max_newton=20, tol=1e-11)
    assert ok
    sc = m.schedule(coupling=m.NEWTON, lin_rtol=1e-13, max_cycles=400, max_newton=20, newton_tol=1e-11)
    rep = sol.step(m.Physics.of(ph), st, dt, sc)
    assert rep.newton_its == its, (rep.newton_its, its)
    errs = [relmax(sol.download(tt), ref) for tt, ref in zip(t[:3], (V, ne, np_))]
    print("newton step zebra %s dt %g %s: max rel err %s, %d FGMRES" % (N, dt, prec_name, errs, rep.vcycles))
    assert max(errs) <= 1e-12, errs


def test_block_zebra_preconditions_with_fewer_iterations():
    """On the cos-stretched axial grid the block zebra cycle is the stronger
    preconditioner: the same Newton step (65x65 and 129x129, dt = 0.1, linear
    tolerance 1e-6) takes fewer FGMRES iterations than with point smoothing,
    and both reach the same state."""
    m = M()
    ph = dict(I.PHYS)
    for N, pre in ((64, 25), (128, 25)):
        _say("zebra iterations", N)
        z, V, ne, np_, S = _start(N)
        cp = NW.Coupled(N, N, 1.0, z, ph)
        NW.steady(cp, V, ne, np_, S, S, max_steps=pre)
        its, states = {}, {}
        for sm in (m.SMOOTH_ZEBRA, m.SMOOTH_ZEBRA_BLOCK):
            sol, t, st = _gpu(N, V, ne, np_, S, smoother=sm)
            sc = m.schedule(coupling=m.NEWTON, lin_rtol=1e-6, max_cycles=400, max_newton=20, newton_tol=1e-10)
            rep = sol.step(m.Physics.of(ph), st, 0.1, sc)
            its[sm] = (rep.newton_its, rep.vcycles)
            states[sm] = [sol.download(x) for x in t[:3]]
        print("%dx%d FGMRES iterations (Newton, FGMRES): point %s, zebra %s" % (N + 1, N + 1, its[m.SMOOTH_ZEBRA],
                                                                                 its[m.SMOOTH_ZEBRA_BLOCK]))
        assert its[m.SMOOTH_ZEBRA_BLOCK][1] < its[m.SMOOTH_ZEBRA][1]
        for a, b in zip(states[m.SMOOTH_ZEBRA_BLOCK], states[m.SMOOTH_ZEBRA]):
            assert relmax(a, b) <= 1e-8


@pytest.mark.parametrize("N,dt,pre,mode", [(32, 1e-3, 0, "default"), (64, 0.1, 12, "default"),
                                            (64, 0.1, 12, "no_fuse"), (64, 0.1, 12, "one_sweep"),
                                            (64, 0.1, 12, "half"), (128, 1e-2, 0, "default"),
                                            (64, 0.1, 12, "fp32"), ((32, 64), 1e-2, 0, "default"),
                                            ((64, 32), 1e-2, 0, "no_fuse"), (64, float("inf"), 12, "default"),
                                            (32, 1e-3, 0, "zebra"), (64, 0.1, 12, "zebra"),
                                            ((32, 64), 1e-2, 0, "zebra"), ((64, 32), float("inf"), 12, "zebra"),
                                            (64, 0.1, 12, "zebra_fp32")])
def test_block_vcycle_matches_oracle(N, dt, pre, mode, monkeypatch):
    """One block V(2,2) cycle z = M r at the Newton Jacobian of a state
    (mg_newton_precond) against the oracle's cycle written from its
    definition, element by element: rediscretised coarse Jacobians at the
    injected state, collective red-black sweeps, R = P^T, exact coarsest
    solve.  Covers the coarse sub-cycle and the per-level launches, one and
    two sweeps per launch, half-sweeps, the FP32 cycle, and the block zebra
    z-line smoother (every axial line's block-tridiagonal system solved by
    block elimination on the GPU, by sparse LU in the oracle)."""
    _say("block vcycle", N, dt, pre, mode)
    m = M()
    nr, nz = N if isinstance(N, tuple) else (N, N)
    z = I.z_cos(nz)
    ne = I.initial_density(nr, nz, 0)
    np_ = ne.copy()
    V = I.initial_potential(nr, nz, z)
    S = I.source(nr, nz, z)
    ph = dict(I.PHYS)
    if pre:
        cp = NW.Coupled(nr, nz, 1.0, z, ph)
        NW.steady(cp, V, ne, np_, S, S, max_steps=pre)
    env = {"no_fuse": "MGF_NO_FUSE", "one_sweep": "MGF_ONE_SWEEP", "half": "MGF_HALF_SWEEPS"}.get(mode)
    if env:
        monkeypatch.setenv(env, "1")
    prec = m.FP32_IR if mode in ("fp32", "zebra_fp32") else m.FP64
    lines = mode.startswith("zebra")
    sol = m.Solver(nr, nz, z, coarsest=4, krylov_m=10, prec=prec,
                   smoother=m.SMOOTH_ZEBRA_BLOCK if lines else m.SMOOTH_ZEBRA)
    if env:
        monkeypatch.delenv(env, raising=False)
    t = [sol.upload(V), sol.upload(ne), sol.upload(np_), sol.upload(S)]
    st = sol.state(t[0], t[1], t[2], t[3], t[3])
    levels = NW.block_hierarchy(nr, nz, 1.0, z, ph, V, ne, np_, dt, coarsest=4)
    assert len(levels) == sol.nlev, (len(levels), sol.nlev)
    rng = np.random.default_rng(nr + 3 * nz + pre)
    planes = [rng.normal(size=(nr + 1, nz + 1)) for _ in range(3)]
    for p_ in planes:
        p_[:, 0] = p_[:, -1] = 0.0
    import torch
    r, zt = sol.field3(), sol.field3()
    for k in range(3):
        r[k, :, : nz + 1] = torch.from_numpy(planes[k]).to(r.device)
    sol.precond(m.Physics.of(ph), st, dt, r, zt)
    torch.cuda.synchronize()
    got = zt[:, :, : nz + 1].cpu().numpy()
    want = levels[0]["cp"].unpack(NW.block_vcycle(levels, levels[0]["cp"].pack(*planes), lines=lines))
    tol = 1e-4 if mode in ("fp32", "zebra_fp32") else 1e-12
    errs = [np.abs(got[k] - want[k]).max() / np.abs(want[k]).max() for k in range(3)]
    print("block vcycle %s dt %g %s: max rel err %s" % (N, dt, mode, errs))
    for k in range(3):
        scale = np.abs(want[k]).max()
        assert np.abs(got[k] - want[k]).max() <= tol * scale, (k, np.abs(got[k] - want[k]).max() / scale)
        assert np.all(got[k][:, 0] == 0.0) and np.all(got[k][:, -1] == 0.0)


def test_steady_run_matches_oracle_33():
    """The whole steady run at 33x33 from the random start: the library's
    solve_steady takes the same accepted steps (dt x1.5 up to 0.1, stop at
    relative change 1e-8) and ends in the oracle's state."""
    _say("steady 33")
    m = M()
    N = 32
    z, V, ne, np_, S = _start(N)
    ph = dict(I.PHYS)
    sol, t, st = _gpu(N, V, ne, np_, S)
    cp = NW.Coupled(N, N, 1.0, z, ph)
    acc, rej, seq = NW.steady(cp, V, ne, np_, S, S, tol=1e-8, newton_tol=1e-10)
    sc = m.schedule(coupling=m.NEWTON, lin_rtol=1e-12, max_cycles=400, newton_tol=1e-10, steady_tol=1e-8)
    code, rep = sol.steady(m.Physics.of(ph), st, sc)
    assert code == 0, m.lib().mg_last_error()
    assert rep.steps == acc and rep.rejected == rej, (rep.steps, acc, rep.rejected, rej)
    for tt, ref in zip(t[:3], (V, ne, np_)):
        assert relmax(sol.download(tt), ref) <= 1e-9
    print("steady 33: steps %d, newton %d, fgmres %d" % (rep.steps, rep.newton_its, rep.vcycles))


@pytest.mark.parametrize("N", [64, 128])
def test_fused_subcycle_and_graphs_match_eager(N, monkeypatch):
    """The single-workgroup coarse sub-cycle and the captured Arnoldi graphs
    (replayed many times, with eager work in between) give bitwise the same
    Newton steps as per-level eager launches."""
    _say("fused/graph", N)
    m = M()
    z, V, ne, np_, S = _start(N)
    ph = dict(I.PHYS)
    cp = NW.Coupled(N, N, 1.0, z, ph)
    NW.steady(cp, V, ne, np_, S, S, max_steps=15)
    results = {}
    for fuse in (1, 0):
        for graphs in (1, 0):
            if fuse:
                monkeypatch.delenv("MGF_NO_FUSE", raising=False)
            else:
                monkeypatch.setenv("MGF_NO_FUSE", "1")
            if graphs:
                monkeypatch.delenv("MGF_NO_GRAPHS", raising=False)
            else:
                monkeypatch.setenv("MGF_NO_GRAPHS", "1")
            sol, t, st = _gpu(N, V, ne, np_, S, krylov_m=20)
            sc = m.schedule(coupling=m.NEWTON, lin_rtol=1e-10, max_cycles=400, newton_tol=1e-10)
            for dt in (1e-3, 1e-2, 0.1):
                sol.step(m.Physics.of(ph), st, dt, sc)
            results[(fuse, graphs)] = [sol.download(x) for x in t[:3]]
    base = results[(0, 0)]
    for key, res in results.items():
        for a, b in zip(res, base):
            assert np.array_equal(a, b), key


@pytest.mark.parametrize("N", [64, 128])
def test_fused_rb_sweep_matches_half_sweeps(N, monkeypatch):
    """One-launch red-black sweeps (tile + recomputed ring in LDS, ping-pong
    buffers), one or two full sweeps per launch, give bitwise the Newton
    steps of half-sweep launches, for every tile height of the other kernels
    (the reductions' order depends on it, so each height is compared with
    itself) and in the FP32 preconditioner."""
    _say("fused rb sweep", N)
    m = M()
    z, V, ne, np_, S = _start(N)
    ph = dict(I.PHYS)
    cp = NW.Coupled(N, N, 1.0, z, ph)
    NW.steady(cp, V, ne, np_, S, S, max_steps=15)
    # two: pairs of sweeps per launch on every launched level (the last
    # pre-smoothing launch also restricting the residual); two_sep: the same
    # with the restriction in its own launch; two_r4: 4-row two-sweep tiles;
    # mixed: pairs only on levels of at most 5000 nodes (65^2 and 33^2),
    # single sweeps above
    big = str(10 ** 9)
    modes = {"half": {"MGF_HALF_SWEEPS": "1"}, "one": {"MGF_ONE_SWEEP": "1"},
             "two": {"MGF_TWO_SWEEP_NODES": big},
             "two_sep": {"MGF_TWO_SWEEP_NODES": big, "MGF_NO_SWEEP_RESTRICT": "1"},
             "two_r4": {"MGF_TWO_SWEEP_NODES": big, "MGF_SWEEP2_ROWS": "4"},
             "mixed": {"MGF_TWO_SWEEP_NODES": "5000"}}
    envs = ("MGF_HALF_SWEEPS", "MGF_ONE_SWEEP", "MGF_TWO_SWEEP_NODES", "MGF_NO_SWEEP_RESTRICT", "MGF_SWEEP2_ROWS")
    for prec in (m.FP64, m.FP32_IR):
        for rows in (1, 2, 4, 16):
            results = {}
            for mode, env in modes.items():
                for k in envs:
                    if k in env:
                        monkeypatch.setenv(k, env[k])
                    else:
                        monkeypatch.delenv(k, raising=False)
                sol, t, st = _gpu(N, V, ne, np_, S, krylov_m=20, prec=prec)
                sol.tune(rows, 32)
                sc = m.schedule(coupling=m.NEWTON, lin_rtol=1e-10, max_cycles=400, newton_tol=1e-10)
                for dt in (1e-3, 1e-2, 0.1):
                    sol.step(m.Physics.of(ph), st, dt, sc)
                results[mode] = [sol.download(x) for x in t[:3]]
            for mode in modes:
                for a, b in zip(results[mode], results["half"]):
                    assert np.array_equal(a, b), (prec, rows, mode)
        # the 16-row one-sweep tile gives the same bits as the default 8-row one
        for k in envs:
            monkeypatch.delenv(k, raising=False)
        monkeypatch.setenv("MGF_ONE_SWEEP", "1")
        monkeypatch.setenv("MGF_SWEEP_ROWS", "16")
        sol, t, st = _gpu(N, V, ne, np_, S, krylov_m=20, prec=prec)
        sol.tune(16, 32)
        for dt in (1e-3, 1e-2, 0.1):
            sol.step(m.Physics.of(ph), st, dt, sc)
        monkeypatch.delenv("MGF_SWEEP_ROWS", raising=False)
        monkeypatch.delenv("MGF_ONE_SWEEP", raising=False)
        for a, b in zip([sol.download(x) for x in t[:3]], results["half"]):
            assert np.array_equal(a, b), (prec, "sweep rows 16")


@pytest.mark.parametrize("nr,nz,prec_name", [(32, 64, "FP64"), (64, 32, "FP64"), (32, 64, "FP32_IR")])
def test_newton_step_rectangular_grid(nr, nz, prec_name):
    """N_r != N_z (ragged sweep tiles and a rectangular coarsest grid): one
    BE step after 10 oracle steps of the steady schedule matches the oracle's
    Newton iterates (FP64 preconditioner: 1e-12; FP32 preconditioner inside
    FP64 FGMRES, converged to the same tolerance: 1e-9)."""
    _say("newton step rectangular", nr, nz, prec_name)
    m = M()
    z = I.z_cos(nz)
    ne = I.initial_density(nr, nz, 3)
    np_, V, S = ne.copy(), I.initial_potential(nr, nz, z), I.source(nr, nz, z)
    ph = dict(I.PHYS)
    cp = NW.Coupled(nr, nz, 1.0, z, ph)
    NW.steady(cp, V, ne, np_, S, S, max_steps=10)
    sol = m.Solver(nr, nz, z, krylov_m=20, coarsest=4, prec=getattr(m, prec_name))
    t = [sol.upload(V), sol.upload(ne), sol.upload(np_), sol.upload(S)]
    st = sol.state(t[0], t[1], t[2], t[3], t[3])
    dt = 1e-2
    ok, its = NW.newton_step(cp, V, ne, np_, S, S, dt, max_newton=20, tol=1e-11)
    assert ok
    sc = m.schedule(coupling=m.NEWTON, lin_rtol=1e-13, max_cycles=400, max_newton=20, newton_tol=1e-11)
    rep = sol.step(m.Physics.of(ph), st, dt, sc)
    assert rep.newton_its == its, (rep.newton_its, its)
    tol = 1e-12 if prec_name == "FP64" else 1e-9
    errs = [relmax(sol.download(tt), ref) for tt, ref in zip(t[:3], (V, ne, np_))]
    print("rectangular %dx%d %s: max rel err %s" % (nr, nz, prec_name, errs))
    assert max(errs) <= tol, errs
