"""Batched steady solves: problems of one grid shape solved together (one
launch per step of the whole batch, problem = blockIdx.z).  Every problem
must end exactly where its own single-problem solve ends (same kernels,
same per-problem decisions), and agree with the oracle."""
import os
import sys

import numpy as np
import pytest

from oracle import newton as NW
from paper_0811_4446_amd import inputs as I

pytestmark = pytest.mark.gpu
os.environ.setdefault("MGF_PROGRESS", "1")


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def M():
    from paper_0811_4446_amd import mgfluid
    return mgfluid


def _draw(N, nprob, seed):
    draws = I.sweep_draws(nprob, seed, sizes=(N,))
    probs = []
    for q, d in enumerate(draws):
        phys = dict(I.PHYS)
        phys.update(V_top=d["V_top"], mu_e=d["mu_e"], D_e=d["D_e"], mu_p=d["mu_p"], D_p=d["D_p"])
        z = I.z_cos(N)
        ne = I.initial_density(N, N, 1000 + q)
        probs.append((phys, I.initial_potential(N, N, z, 0.0, phys["V_top"]), ne, ne.copy(), I.source(N, N, z)))
    return probs


@pytest.mark.parametrize("N,nprob,prec,smoother", [(16, 5, 1, 1), (16, 1, 1, 1), (32, 4, 1, 1), (32, 3, 0, 1),
                                                   (32, 3, 0, 2)])
def test_batch_equals_single_problem_solves(N, nprob, prec, smoother):
    _say("batch vs single", N, nprob, prec, smoother)
    m = M()
    z = I.z_cos(N)
    probs = _draw(N, nprob, 12345)
    sc = m.schedule(coupling=m.NEWTON, lin_rtol=1e-3, max_cycles=200, newton_tol=1e-6, steady_tol=1e-8,
                    max_steps=3000)
    B = m.Batch(N, N, z, nprob, prec=prec, krylov_m=20, smoother=smoother)
    for p, (phys, V, ne, np_, S) in enumerate(probs):
        B.set_problem(p, V, ne, np_, S)
    code, reps = B.steady([m.Physics.of(pr[0]) for pr in probs], sc)
    assert code == 0, m.lib().mg_last_error()
    for p, (phys, V, ne, np_, S) in enumerate(probs):
        sol = m.Solver(N, N, z, krylov_m=20, coarsest=4, prec=prec, smoother=smoother)
        t = [sol.upload(V), sol.upload(ne), sol.upload(np_), sol.upload(S)]
        c1, rep = sol.steady(m.Physics.of(phys), sol.state(t[0], t[1], t[2], t[3], t[3]), sc)
        assert c1 == 0
        assert reps[p]["steps"] == rep.steps and reps[p]["newton_its"] == rep.newton_its, (p, reps[p], rep.as_dict())
        assert reps[p]["vcycles"] == rep.vcycles
        for name, tt in (("V", t[0]), ("ne", t[1]), ("np", t[2])):
            assert np.array_equal(B.get(p, name), sol.download(tt)), (p, name)


def test_batch_matches_oracle_17():
    _say("batch vs oracle")
    m = M()
    N = 16
    z = I.z_cos(N)
    probs = _draw(N, 3, 777)
    sc = m.schedule(coupling=m.NEWTON, lin_rtol=1e-12, max_cycles=400, newton_tol=1e-10, steady_tol=1e-8,
                    max_steps=3000)
    B = m.Batch(N, N, z, len(probs), prec=m.FP32_IR, krylov_m=20)
    for p, (phys, V, ne, np_, S) in enumerate(probs):
        B.set_problem(p, V, ne, np_, S)
    code, reps = B.steady([m.Physics.of(pr[0]) for pr in probs], sc)
    assert code == 0
    for p, (phys, V, ne, np_, S) in enumerate(probs):
        cp = NW.Coupled(N, N, 1.0, z, phys)
        Vo, neo, npo = V.copy(), ne.copy(), np_.copy()
        acc, rej, seq = NW.steady(cp, Vo, neo, npo, S, S, tol=1e-8, newton_tol=1e-10)
        assert reps[p]["steps"] == acc
        for name, ref in (("V", Vo), ("ne", neo), ("np", npo)):
            got = B.get(p, name)
            assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max(), (p, name)


def test_every_launch_shape_gives_the_same_step():
    """All autotuner candidates (rows per workgroup 1..16, fused coarse
    sub-cycle off/16/32/64) give the same Newton step up to summation order."""
    _say("launch shapes")
    m = M()
    N = 64
    z = I.z_cos(N)
    ne = I.initial_density(N, N, 0)
    np_, V, S = ne.copy(), I.initial_potential(N, N, z), I.source(N, N, z)
    ph = dict(I.PHYS)
    sc = m.schedule(coupling=m.NEWTON, lin_rtol=1e-12, max_cycles=400, newton_tol=1e-10)
    ref = None
    for ty in (4, 1, 2, 8, 16):
        for fm in (32, 0, 16, 64):
            sol = m.Solver(N, N, z, krylov_m=20, coarsest=4, prec=m.FP32_IR)
            sol.tune(ty, fm)
            t = [sol.upload(V), sol.upload(ne), sol.upload(np_), sol.upload(S)]
            st = sol.state(t[0], t[1], t[2], t[3], t[3])
            for dt in (1e-4, 1e-3):
                sol.step(m.Physics.of(ph), st, dt, sc)
            res = [sol.download(x) for x in t[:3]]
            if ref is None:
                ref = res
            for a, b in zip(res, ref):
                assert np.abs(a - b).max() <= 1e-11 * np.abs(b).max(), (ty, fm)


def test_concurrent_batches_of_uneven_sizes_equal_separate_solves():
    """Batches of different grid sizes (17x17 x 3 and 33x33 x 2), each on a
    stream of its own, solved together by solve_steady_batches (one host
    thread per batch): every problem ends bit for bit where its batch ends
    when solved alone."""
    _say("concurrent batches 17x3 + 33x2")
    import torch
    m = M()
    sc = m.schedule(coupling=m.NEWTON, lin_rtol=1e-3, max_cycles=200, newton_tol=1e-6, steady_tol=1e-8,
                    max_steps=3000)
    specs = [(16, 3, 777), (32, 2, 778)]

    def make(streams):
        out = []
        for (N, nprob, seed), stream in zip(specs, streams):
            B = m.Batch(N, N, I.z_cos(N), nprob, prec=1, krylov_m=20, stream=stream)
            probs = _draw(N, nprob, seed)
            for p, (phys, V, ne, np_, S) in enumerate(probs):
                B.set_problem(p, V, ne, np_, S)
            out.append((B, [m.Physics.of(pr[0]) for pr in probs]))
        return out

    alone = []
    for B, phys in make([None, None]):
        code, reps = B.steady(phys, sc)
        assert code == 0, m.lib().mg_last_error()
        alone.append((reps, {(p, k): B.get(p, k) for p in range(B.n) for k in ("V", "ne", "np")}))
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    both = make(streams)
    code, reps_all = m.solve_batches([b for b, _ in both], [ph for _, ph in both], sc)
    assert code == 0, m.lib().mg_last_error()
    for (B, _), reps, (reps1, fields1) in zip(both, reps_all, alone):
        for p in range(B.n):
            assert reps[p]["steps"] == reps1[p]["steps"] and reps[p]["vcycles"] == reps1[p]["vcycles"], (reps[p],
                                                                                                  reps1[p])
            for k in ("V", "ne", "np"):
                assert np.array_equal(B.get(p, k), fields1[(p, k)]), (B.nr, p, k)
