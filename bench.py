#!/usr/bin/env python
"""Benchmark of the steady axisymmetric drift-diffusion solver on one MI355X.

Workload: the multilevel-prolongation chain of Sec. 2 on the synthetic
discharge (dimensionless physics, cos-stretched z grid, Gaussian source):
65x65 from a seeded random start -> steady -> bilinear prolongation ->
129x129 -> steady -> prolongation -> 257x257 -> steady.  Each time step is
a coupled backward-Euler step solved by Newton (Eq. 14) with FGMRES
preconditioned by a block V(2,2) cycle; dt starts at 1e-4 and grows x1.5
per accepted step up to 0.1; the run is steady when the relative density
change per step drops below 1e-8.  Applied voltage V_top in {0.5, 1, 2}.

A bench "step" is the timed 257x257 stage for all three voltages, from
initial states already resident in HBM.  `value` is the mean
time-to-steady per voltage (seconds, lower is better).  After the timed
steps, once per voltage: the chain continued to 513x513 and prolonged to
1025x1025, whose steady solve is timed with the FP64 and with the FP32
block preconditioner (config.t1025).  The roofline entry is the kernel with
the largest share of GPU time in the 257x257 solve; the finest-level sweep
at 257x257 (cache-resident) and at 1025x1025 (HBM) is reported beside it.

Prints one JSON line.  --gpus N with N > 1 exits: the solver runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("time-to-steady at 257² & 1025² (s), V-cycle HBM GB/s; "
          "plain FP64 vs chosen forms")
HBM_PEAK_GBS = 8000.0
# Relative tolerance of every linear (FGMRES) solve inside Newton, the
# inexact-Newton forcing term: the final steady states differ from those of
# solves to 1e-10 by at most 4.7e-10 relative at 257x257 and 1025x1025 (all
# voltages, both preconditioner precisions), with the same accepted steps.
LIN_RTOL = 1e-2
# HBM bytes per launch of the finest-level sweep (k_block_rb_sweep) and per
# V-cycle of the two-sweep launches (k_block_rb_sweep2 on 129x129, 65x65,
# 33x33, pre- and post-smoothing), from FETCH_SIZE and WRITE_SIZE counter
# runs (x2.0 and x1.0 by a 512 MiB copy's counters; the runs and tables are
# kept under profiles/).  Valid only for the kernel source they were taken
# with (the text between the two markers, which holds both sweep kernels
# and their device helpers): any change to it reports null.
MEASURED_TRAFFIC = {"source": "paper_0811_4446_amd/csrc/mg_newton.hip",
                    "begin": "// x plus the bilinear prolongation (z-distance weights) of one coarse field",
                    "end": "__global__ void k_block_residual(Geom g, BOpT<T> J",
                    "sha1": "c8749accfbbad713a3c3fc615e9c67c093a485eb",
                    "bytes": {256: 20511539, 1024: 313476403},
                    "sweep2_vcycle_bytes": {256: 20192357}}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def schedule(M, lin_rtol):
    return M.schedule(dt0=1e-4, growth=1.5, dt_max=0.1, steady_tol=1e-8, lin_rtol=lin_rtol,
                      max_steps=20000, max_cycles=400, coupling=M.NEWTON, max_newton=10,
                      newton_tol=1e-6)


def chain_to(M, I, N_final, vtop, lin_rtol, seed=0, N0=64, prec=None):
    """Steady runs N0 -> ... -> N_final/2, then prolong to N_final.  Returns
    the fine solver and its initial (V, ne, np, S) device fields."""
    prec = M.FP64 if prec is None else prec
    phys = dict(I.PHYS)
    phys["V_top"] = vtop
    P = M.Physics.of(phys)
    N = N0
    z = I.z_cos(N)
    sol = M.Solver(N, N, z, krylov_m=30, coarsest=4, prec=prec)
    ne = I.initial_density(N, N, seed)
    t = [sol.upload(I.initial_potential(N, N, z, 0.0, vtop)), sol.upload(ne), sol.upload(ne),
         sol.upload(I.source(N, N, z))]
    info = []
    while True:
        st = sol.state(t[0], t[1], t[2], t[3], t[3])
        t0 = time.time()
        code, rep = sol.steady(P, st, schedule(M, lin_rtol))
        if code != 0:
            raise RuntimeError("steady %d failed: %s" % (N, M.lib().mg_last_error()))
        info.append(dict(N=N, steps=rep.steps, seconds=time.time() - t0))
        if 2 * N == N_final:
            break
        N2 = 2 * N
        z2 = I.z_cos(N2)
        fine = M.Solver(N2, N2, z2, krylov_m=30, coarsest=4, prec=prec)
        t2 = [fine.field(), fine.field(), fine.field(), fine.upload(I.source(N2, N2, z2))]
        M.prolong_state(sol, st, fine, fine.state(t2[0], t2[1], t2[2], t2[3], t2[3]), P)
        sol, t, N = fine, t2, N2
    z2 = I.z_cos(N_final)
    fine = M.Solver(N_final, N_final, z2, krylov_m=30, coarsest=4, prec=prec)
    t2 = [fine.field(), fine.field(), fine.field(), fine.upload(I.source(N_final, N_final, z2))]
    M.prolong_state(sol, sol.state(t[0], t[1], t[2], t[3], t[3]), fine,
                    fine.state(t2[0], t2[1], t2[2], t2[3], t2[3]), P)
    return fine, t2, P, info


def cpu_baseline(I, newton_its_gpu, vtop=1.0, N=256):
    """The oracle (plain FP64; SciPy sparse LU for each Newton system) on the
    host: one Newton iteration at 257x257 (residual, Jacobian, LU solve),
    timed single-threaded and scaled by the GPU run's Newton iteration
    count."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import scipy.sparse.linalg as spla
    from oracle import newton as NW
    z = I.z_cos(N)
    phys = dict(I.PHYS)
    phys["V_top"] = vtop
    cp = NW.Coupled(N, N, 1.0, z, phys)
    ne = I.initial_density(N, N, 0)
    np_ = ne.copy()
    V = I.initial_potential(N, N, z, 0.0, vtop)
    S = I.source(N, N, z)
    t0 = time.time()
    (Fe, Fp, FV), (Ae, Ap) = cp.residual(V, ne, np_, ne, np_, S, S, 1e4)
    J = cp.jacobian(V, ne, np_, Ae, Ap)
    du = spla.splu(J).solve(-cp.pack(Fe, Fp, FV))
    per_it = time.time() - t0
    assert du.shape[0] == J.shape[0]
    return dict(value=round(per_it * newton_its_gpu, 1), unit="s", cores=1, kind="oracle", host=_host(),
                sample="1 oracle Newton iteration at %dx%d (residual, Jacobian, sparse LU; single thread) = %.2f s "
                       "from the seeded start (the sparse LU's cost depends on the grid, not on the state), x %d "
                       "Newton iterations of the GPU run (extrapolated)" % (N + 1, N + 1, per_it, newton_its_gpu))


def _host():
    """Host CPU model and logical core count (for the oracle baseline)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(cpu=model, nproc=os.cpu_count())


def _traffic(N, key="bytes"):
    import hashlib
    with open(os.path.join(ROOT, MEASURED_TRAFFIC["source"])) as fh:
        src = fh.read()
    a, e = src.find(MEASURED_TRAFFIC["begin"]), src.find(MEASURED_TRAFFIC["end"])
    same = 0 <= a < e and hashlib.sha1(src[a:e].encode()).hexdigest() == MEASURED_TRAFFIC["sha1"]
    return MEASURED_TRAFFIC[key].get(N) if same else None


def roofline(sol, N, reps=200, resident=None):
    """Roofline entry of the one-launch collective red-black block sweep
    (k_block_rb_sweep) on the finest level: its average launch duration from
    HIP events recorded on the library's stream around `reps` consecutive
    sweeps (the Jacobian of the last solve), against the algorithmic bytes
    of one sweep: per unknown node 27 Jacobian entries, 3 right-hand-side
    values and 3 old unknowns read, 3 new unknowns written (FP64)."""
    avg_ms = sol.time_kernel(4, 0, reps=reps)
    nodes = (N + 1) * (N - 1)
    bytes_launch = 8.0 * nodes * 36
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    out = dict(bound="hbm", kernel="k_block_rb_sweep", level="%dx%d" % (N + 1, N + 1), achieved=round(achieved, 1),
               peak=HBM_PEAK_GBS, unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4), traffic=_traffic(N),
               avg_launch_us=round(avg_ms * 1e3, 3), algorithmic_bytes_per_launch=int(bytes_launch),
               timed_launches=reps)
    if resident:
        out["resident"] = resident
    return out


def roofline_dominant(sol, N, reps=200):
    """Roofline entry of the kernel with the largest share of GPU time in the
    257x257 steady solve: the two-sweep collective red-black launch
    (k_block_rb_sweep2) on the levels 129x129, 65x65 and 33x33, twice per
    V-cycle each: pre-smoothing (from a zero guess, with the residual
    restricted to the next level in the same launch) and post-smoothing.
    Per level and launch form, the mean duration of `reps` back-to-back
    launches between HIP events on the library's stream (the Jacobian of
    the last solve); algorithmic bytes of one launch: per unknown node 27
    Jacobian entries, 3 right-hand-side and 3 old values read once, 3 new
    values written (FP64, 288 B), plus 3 values per unknown coarse node
    written by the restricting launch.  The entry's achieved rate is the sum
    of those bytes over one V-cycle's launches divided by their summed
    durations.  The working set of these levels (under 5 MB) sits in the
    256 MB Infinity Cache and each launch lasts a few microseconds: the
    launches are bound by latency, not by HBM."""
    levels = []
    tot_b = tot_t = 0.0
    n = N
    for l in range(1, sol.nlev):
        n //= 2
        if n > 128 or n <= 16:  # two-sweep launches: 129^2 down to 33^2; below, the coarse sub-cycle
            continue
        pre_ms = sol.time_kernel(6, l, reps=reps)
        post_ms = sol.time_kernel(5, l, reps=reps)
        b = 8.0 * 36 * (n + 1) * (n - 1)
        bc = 8.0 * 3 * (n // 2 + 1) * (n // 2 - 1)
        levels.append(dict(level="%dx%d" % (n + 1, n + 1), pre_restrict_launch_us=round(pre_ms * 1e3, 3),
                           post_launch_us=round(post_ms * 1e3, 3), algorithmic_bytes_post=int(b),
                           algorithmic_bytes_pre=int(b + bc)))
        tot_b += 2 * b + bc
        tot_t += (pre_ms + post_ms) * 1e-3
    achieved = tot_b / tot_t / 1e9
    return dict(bound="hbm", kernel="k_block_rb_sweep2", achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4), traffic=_traffic(N, "sweep2_vcycle_bytes"),
                algorithmic_bytes_per_unit=int(tot_b),
                resident="Infinity Cache (levels 129x129..33x33 of the 257x257 solve, < 5 MB)",
                limited_by="launch and memory latency (microsecond launches)",
                unit_of_work="one V-cycle's two-sweep launches (pre with restriction, and post, on each level)",
                levels=levels, timed_launches_per_level=reps)


def roofline_only(args, M, I):
    """The roofline measurement alone (for counter runs): a 257x257 context,
    one Newton step from the seeded start to assemble a Jacobian, the timed
    half-sweeps, then a plain 512 MiB device copy whose bytes calibrate the
    FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    N = args.grid
    z = I.z_cos(N)
    phys = dict(I.PHYS)
    P = M.Physics.of(phys)
    sol = M.Solver(N, N, z, krylov_m=30, coarsest=4, prec=M.FP64)
    ne = I.initial_density(N, N, 0)
    t = [sol.upload(I.initial_potential(N, N, z, 0.0, phys["V_top"])), sol.upload(ne), sol.upload(ne),
         sol.upload(I.source(N, N, z))]
    st = sol.state(t[0], t[1], t[2], t[3], t[3])
    sol.step(P, st, 1e-3, schedule(M, args.lin_rtol))
    roof = roofline(sol, N, reps=args.reps)
    a = torch.ones(1 << 26, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    roof["calibration_copy_bytes"] = a.numel() * 8
    # practical ceiling of this GPU's HBM for a streaming kernel: a plain
    # 512 MiB device copy (read + write bytes), 20 back to back
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    roof["plain_copy_GBps"] = round(2 * a.numel() * 8 * 20 / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    print(json.dumps({"roofline": roof}), flush=True)


def trace_summary(path, top=25, tail_kernel="k_block_rb_sweep", tail=200):
    """Summary of a rocprofv3 CSV: a kernel trace (per kernel and grid
    shape: calls, total and average duration) or a counter collection (per
    kernel, grid shape and counter: dispatches and mean value).  For a
    trace, also the mean duration of the last `tail` dispatches of every
    kernel whose name contains `tail_kernel`, per grid shape: the roofline
    loops' launches, which come last for each of their grids in the
    benchmark."""
    import csv
    import collections
    agg = collections.OrderedDict()
    tails = collections.defaultdict(list)
    kind = None
    with open(path) as f:
        rd = csv.DictReader(f)
        cols = rd.fieldnames
        kind = "counters" if "Counter_Name" in cols else "trace"
        for row in rd:
            name = row["Kernel_Name"].replace("(anonymous namespace)::", "").split("(")[0]
            if "Grid_Size" in row:
                grid = row["Grid_Size"]
            else:
                grid = "%sx%sx%s" % (row.get("Grid_Size_X"), row.get("Grid_Size_Y"), row.get("Grid_Size_Z"))
            if kind == "trace":
                key = (name[:70], grid)
                d = int(row["End_Timestamp"]) - int(row["Start_Timestamp"])
                e = agg.setdefault(key, [0, 0])
                e[0] += 1
                e[1] += d
                if tail_kernel in name:
                    tails[key].append((int(row["Start_Timestamp"]), d))
            else:
                key = (name[:70], grid, row["Counter_Name"])
                e = agg.setdefault(key, [0, 0.0])
                e[0] += 1
                e[1] += float(row["Counter_Value"])
    if kind == "trace":
        tot = sum(v[1] for v in agg.values())
        print("%-70s %-16s %9s %12s %10s %7s" % ("kernel", "grid", "calls", "total_ms", "avg_us", "share"))
        for (name, grid), (c, t) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:top]:
            print("%-70s %-16s %9d %12.3f %10.3f %6.2f%%" % (name, grid, c, t / 1e6, t / c / 1e3, 100.0 * t / tot))
        for (name, grid), v in sorted(tails.items()):
            if len(v) < tail:
                continue
            last = [d for _, d in sorted(v)[-tail:]]
            print("last %d dispatches of %s on grid %s: mean %.3f us" % (tail, name, grid, sum(last) / tail / 1e3))
    else:
        print("%-70s %-16s %-14s %9s %16s" % ("kernel", "grid", "counter", "dispatches", "mean_per_dispatch"))
        for (name, grid, cn), (c, v) in agg.items():
            print("%-70s %-16s %-14s %9d %16.1f" % (name, grid, cn, c, v / c))


def vcycle_bench(args, M, I):
    """The scalar path: (1) one decoupled backward-Euler step at 65x65 (dt
    1e-4): Poisson with n^k, then the SG electron and ion equations, each by
    V(2,2) red-black cycles to relative residual 1e-10, timed beside the
    oracle's same step on one host core; (2) V-cycle throughput: back-to-back
    V(2,2) cycles on the assembled Poisson and electron operators at 257x257
    and 1025x1025, for both smoothers, on one context and (1025x1025) on four
    contexts in turn, whose working set exceeds the 256 MB Infinity Cache.
    Algorithmic bytes of one FP64 V(2,2) cycle per fine node: 4 sweeps x 8
    values + residual 8 + restriction 1.25 + prolongation 2.25 = 43.5 values
    on the fine level, x 4/3 for the coarser levels = 58 values = 464 B."""
    import numpy as np
    import torch
    import oracle as O
    out_rows = {}
    N = 64
    z = I.z_cos(N)
    ne0 = I.initial_density(N, N, 0)
    S = I.source(N, N, z)
    V0 = I.initial_potential(N, N, z, 0.0, 1.0)
    phys = dict(I.PHYS)
    sol = M.Solver(N, N, z, smoother=M.SMOOTH_RB)
    sched = M.schedule(lin_rtol=1e-10, max_cycles=500)
    tS = sol.upload(S)
    times, cycles = [], None
    for k in range(6):
        t = [sol.upload(V0), sol.upload(ne0), sol.upload(ne0.copy())]
        st = sol.state(t[0], t[1], t[2], tS, tS)
        torch.cuda.synchronize()
        t0 = time.time()
        rep = sol.step(M.Physics.of(phys), st, 1e-4, sched)
        torch.cuda.synchronize()
        if k:
            times.append(time.time() - t0)
        cycles = rep.vcycles
    Vo, neo, npo = V0.copy(), ne0.copy(), ne0.copy()
    t0 = time.time()
    code, cyc, rr = O.step_decoupled(1.0, z, O.Phys(**phys), Vo, neo, npo, S, S, 1e-4, smoother=O.SMOOTH_RB,
                                     rtol=1e-10)
    t_or = time.time() - t0
    out_rows["step_65"] = dict(gpu_ms_median=round(1e3 * float(np.median(times)), 3), vcycles=cycles,
                               oracle_ms=round(1e3 * t_or, 1), oracle_cycles=list(cyc), oracle_cores=1)
    log(out_rows["step_65"])
    # V-cycle throughput
    vrows = []
    for N, nctx in ((256, 1), (1024, 1), (1024, 4)):
        for smoother, sname in ((M.SMOOTH_RB, "red-black"), (M.SMOOTH_ZEBRA, "zebra")):
            z = I.z_cos(N)
            ctxs = []
            for c in range(nctx):
                s = M.Solver(N, N, z, smoother=smoother)
                ne = I.initial_density(N, N, c)
                t = [s.upload(I.initial_potential(N, N, z, 0.0, 1.0)), s.upload(ne), s.upload(ne.copy()),
                     s.upload(I.source(N, N, z))]
                st = s.state(t[0], t[1], t[2], t[3], t[3])
                for eq in (0, 1):
                    s.assemble(eq, M.Physics.of(phys), st, 1e-4)
                ctxs.append((s, [s.field(), s.field()], t))
            for eq, ename in ((0, "poisson"), (1, "electron")):
                for s, xs, _ in ctxs:
                    s.vcycle(eq, xs[eq], 2)
                torch.cuda.synchronize()
                reps = 20
                t0 = time.time()
                for r in range(reps):
                    for s, xs, _ in ctxs:
                        s.vcycle(eq, xs[eq], 1)
                torch.cuda.synchronize()
                per = (time.time() - t0) / (reps * nctx)
                nodes = (N + 1) * (N + 1)
                gbs = 464.0 * nodes / per / 1e9
                vrows.append(dict(grid="%dx%d" % (N + 1, N + 1), contexts=nctx, smoother=sname, eq=ename,
                                  ms_per_cycle=round(per * 1e3, 4), algorithmic_GBps=round(gbs, 1),
                                  frac_of_8TBps=round(gbs / HBM_PEAK_GBS, 3)))
                log(vrows[-1])
            del ctxs
            torch.cuda.empty_cache()
    out = {"metric": METRIC, "value": out_rows["step_65"]["gpu_ms_median"] / 1e3, "unit": "s", "n_gpus": 1,
           "steps": 5, "warmup": 1, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "decoupled BE step at 65x65 (dt 1e-4, V(2,2) red-black to 1e-10 per equation) "
                                  "and scalar V-cycle throughput at 257x257 and 1025x1025",
                      "step_65": out_rows["step_65"], "vcycle": vrows}}
    print(json.dumps(out), flush=True)


def compare_precisions(args, M, I, N, vtops):
    """Time-to-steady of the finest stage with the FP64 and the FP32 block
    preconditioner (Newton residuals, FGMRES and the stop rules in FP64), from
    the same prolonged state; reports both and their difference."""
    import numpy as np
    import torch
    forms = ["fp64", "fp32"] if args.prec == "both" else [args.prec]
    rows = []
    for vt in vtops:
        fine, t, P, info = chain_to(M, I, N, vt, args.lin_rtol)
        log("prep V_top=%g: %s" % (vt, info))
        init = [x.clone() for x in t[:3]]
        finals = {}
        for form in forms:
            prec = M.FP64 if form == "fp64" else M.FP32_IR
            sol = M.Solver(N, N, I.z_cos(N), krylov_m=30, coarsest=4, prec=prec)
            tt = [x.clone() for x in init] + [t[3]]
            torch.cuda.synchronize()
            t0 = time.time()
            code, rep = sol.steady(P, sol.state(tt[0], tt[1], tt[2], tt[3], tt[3]), schedule(M, args.lin_rtol))
            torch.cuda.synchronize()
            el = time.time() - t0
            if code != 0:
                raise RuntimeError("steady failed: %s" % M.lib().mg_last_error())
            finals[form] = [sol.download(x) for x in tt[:3]]
            rows.append(dict(V_top=vt, form=form, seconds=round(el, 3), steps=rep.steps, newton=rep.newton_its,
                             fgmres=rep.vcycles))
            log(rows[-1])
            del sol
        if len(forms) == 2:
            d = [float(np.abs(a - b).max() / np.abs(b).max()) for a, b in zip(finals["fp32"], finals["fp64"])]
            rows.append(dict(V_top=vt, fp32_vs_fp64_maxrel=d))
            log(rows[-1])
    secs = {f: [r["seconds"] for r in rows if r.get("form") == f] for f in forms}
    out = {"metric": METRIC, "value": round(float(np.mean(secs[forms[-1]])), 4), "unit": "s", "n_gpus": 1,
           "steps": 1, "warmup": 0, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64+f32" if "fp32" in forms else "f64", "data": "synthetic",
           "config": {"workload": "steady %dx%d from the prolonged %dx%d steady state, coupled Newton BE, "
                                  "block preconditioner precision comparison" % (N + 1, N + 1, N // 2 + 1, N // 2 + 1),
                      "forms": forms, "lin_rtol": args.lin_rtol,
                      "mean_seconds": {f: round(float(np.mean(v)), 4) for f, v in secs.items()},
                      "runs": rows}}
    print(json.dumps(out), flush=True)


def sweep_reference(args, M, I):
    """The first `--sweep-ref` problems of every size class of the sweep,
    solved one at a time (single-problem contexts, same FP32 preconditioner
    and schedule): the per problem-step cost the batch is compared with."""
    import numpy as np
    import torch
    draws = I.sweep_draws(args.nprob, 12345)
    classes = {}
    for q, d in enumerate(draws):
        classes.setdefault(d["N"], []).append((q, d))
    sched = schedule(M, args.lin_rtol)
    rows = []
    for N in sorted(classes):
        z = I.z_cos(N)
        sol = M.Solver(N, N, z, krylov_m=20, coarsest=4, prec=M.FP32_IR)
        for q, d in classes[N][:args.sweep_ref]:
            ph = dict(I.PHYS)
            ph.update(V_top=d["V_top"], mu_e=d["mu_e"], D_e=d["D_e"], mu_p=d["mu_p"], D_p=d["D_p"])
            ne = I.initial_density(N, N, 1000 + q)
            t = [sol.upload(I.initial_potential(N, N, z, 0.0, ph["V_top"])), sol.upload(ne), sol.upload(ne),
                 sol.upload(I.source(N, N, z))]
            torch.cuda.synchronize()
            t0 = time.time()
            code, rep = sol.steady(M.Physics.of(ph), sol.state(t[0], t[1], t[2], t[3], t[3]), sched)
            torch.cuda.synchronize()
            el = time.time() - t0
            rows.append(dict(grid="%dx%d" % (N + 1, N + 1), problem=q, code=code, seconds=round(el, 3),
                             steps=rep.steps, ms_per_step=round(1e3 * el / max(rep.steps, 1), 3)))
            log(rows[-1])
        del sol
    out = {"metric": METRIC, "value": None, "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32",
           "data": "synthetic",
           "config": {"workload": "reference for the parameter sweep: its first problems of each size solved "
                                  "one at a time", "runs": rows}}
    print(json.dumps(out), flush=True)


def sweep(args, M, I):
    """Parameter sweep: independent steady solves from their own seeded
    random starts, grid sizes drawn from {65, 129, 257, 513}^2, V_top ~
    U(0.2, 5), mu_e/mu_p ~ logU(10, 1000).  Problems of one size form one
    batch (every kernel launch advances the whole batch); the FP32 block
    preconditioner sits inside FP64 FGMRES/Newton; launch shapes come from
    the autotuner.  The batches run one after another, or with --concurrent
    all at once (solve_steady_batches: each batch on a stream and a host
    thread of its own)."""
    import numpy as np
    import torch
    from paper_0811_4446_amd import autotune
    os.environ.setdefault("MGF_PROGRESS", "1")
    draws = I.sweep_draws(args.nprob, 12345)
    classes = {}
    for q, d in enumerate(draws):
        classes.setdefault(d["N"], []).append((q, d))
    sched = schedule(M, args.lin_rtol)
    rows, total_t, total_cycles_bytes = [], 0.0, 0.0
    t_all = time.time()
    # algorithmic bytes of one FP32 block V(2,2) preconditioner cycle per fine
    # node: 4 collective half-sweep pairs x 36 values, residual 36,
    # restriction ~3.75, prolongation ~6.75, all levels x 4/3, 4 B each
    vbytes = (4 * 36 + 36 + 3.75 + 6.75) * 4.0 / 3.0 * 4.0

    def build(N, items, stream):
        z = I.z_cos(N)
        B = M.Batch(N, N, z, len(items), prec=M.FP32_IR, krylov_m=20, stream=stream)
        phys, init = [], []
        for q, d in items:
            ph = dict(I.PHYS)
            ph.update(V_top=d["V_top"], mu_e=d["mu_e"], D_e=d["D_e"], mu_p=d["mu_p"], D_p=d["D_p"])
            phys.append(M.Physics.of(ph))
            ne = I.initial_density(N, N, 1000 + q)
            init.append((I.initial_potential(N, N, z, 0.0, ph["V_top"]), ne, ne.copy(), I.source(N, N, z)))

        def reset():
            for p, (V, ne, np_, S) in enumerate(init):
                B.set_problem(p, V, ne, np_, S)

        choice, tim = autotune.tune(B, phys, reset, 1, log=log)
        reset()
        return B, phys, choice

    def row(N, items, B, reps, el, choice):
        ok = sum(1 for r in reps if r["steps"] > 0 and r["last_change"] < 1e-8)
        cyc = sum(r["vcycles"] for r in reps)
        return dict(grid="%dx%d" % (N + 1, N + 1), problems=len(items), converged=ok,
                    seconds=None if el is None else round(el, 3),
                    tuning=dict(rows_per_block=choice[0], fuse_max=choice[1]),
                    steps_mean=float(np.mean([r["steps"] for r in reps])),
                    ms_per_problem_step=None if el is None else round(1e3 * el / max(1, sum(r["steps"] for r in reps)), 4),
                    fgmres_total=int(cyc), newton_total=int(sum(r["newton_its"] for r in reps))), cyc

    if args.concurrent:
        built = []
        for N in sorted(classes):
            B, phys, choice = build(N, classes[N], torch.cuda.Stream())
            built.append((N, B, phys, choice))
        torch.cuda.synchronize()
        t0 = time.time()
        code, reps_all = M.solve_batches([b[1] for b in built], [b[2] for b in built], sched)
        torch.cuda.synchronize()
        total_t = time.time() - t0
        for (N, B, phys, choice), reps in zip(built, reps_all):
            r, cyc = row(N, classes[N], B, reps, None, choice)
            r["code"] = code
            total_cycles_bytes += cyc * (N + 1) * (N + 1) * vbytes
            rows.append(r)
            log(r)
    else:
        for N in sorted(classes):
            B, phys, choice = build(N, classes[N], None)
            torch.cuda.synchronize()
            t0 = time.time()
            code, reps = B.steady(phys, sched)
            torch.cuda.synchronize()
            el = time.time() - t0
            r, cyc = row(N, classes[N], B, reps, el, choice)
            r["code"] = code
            total_cycles_bytes += cyc * (N + 1) * (N + 1) * vbytes
            total_t += el
            rows.append(r)
            log(r)
            del B
            torch.cuda.empty_cache()
    wall = time.time() - t_all
    out = {"metric": METRIC, "value": round(total_t, 3), "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32",
           "data": "synthetic",
           "config": {"workload": "parameter sweep of %d independent steady solves, grids 65..513, batched per "
                                  "grid size (%s), FP32 block preconditioner in FP64 Newton-FGMRES"
                                  % (args.nprob, "all batches at once" if args.concurrent else "one batch after another"),
                      "solves_per_s": round(args.nprob / total_t, 3), "wall_incl_setup_and_tuning_s": round(wall, 1),
                      "preconditioner_GBps_lower_bound": round(total_cycles_bytes / total_t / 1e9, 1),
                      "classes": rows}}
    print(json.dumps(out), flush=True)


def learned(args, M, I):
    """Learned warm start on 257x257: train the network on solver-generated
    steady solutions, then compare time-to-steady from its prediction with
    the plain prolongation start on held-out draws."""
    import numpy as np
    import torch
    from paper_0811_4446_amd import warmstart as WS
    os.environ.setdefault("MGF_PROGRESS", "1")
    t0 = time.time()
    tr = WS.generate(WS.draws(args.n_train, 2024), log=log)
    va = WS.generate(WS.draws(args.n_val, 7), log=log)
    te = WS.generate(WS.draws(args.n_test, 8), log=log)
    tgen = time.time() - t0
    t1 = time.time()
    net, hist = WS.train(tr, va, epochs=args.epochs, log=log)
    torch.cuda.synchronize()
    ttrain = time.time() - t1
    if args.save_weights:
        np.save(args.save_weights, net.params.cpu().numpy())
    summary = WS.compare(net, te, timed=args.n_timed, criterion=args.criterion, log=log)
    summary = {k: v for k, v in summary.items() if not k.startswith("_")}
    thr = WS.network_throughput(net)
    log("network throughput: %s" % thr)
    vals = summary["single_seconds_learned"]
    out = {"metric": METRIC, "value": round(float(np.mean(vals)), 4) if vals else None, "unit": "s", "n_gpus": 1,
           "steps": 1, "warmup": 0, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64+bf16", "data": "synthetic",
           "config": {"workload": "steady 257x257 from the learned warm start vs the plain prolongation of the "
                                  "129x129 steady state (held-out draws)",
                      "n_train": args.n_train, "n_val": args.n_val, "n_test": args.n_test, "epochs": args.epochs,
                      "data_generation_s": round(tgen, 1), "training_s": round(ttrain, 1),
                      "final_train_loss": hist[-1][1], "final_val_loss": hist[-1][2],
                      "initial_val_loss": hist[0][2], "summary": summary, "network_throughput": thr}}
    print(json.dumps(out), flush=True)


def argon(args, M, I):
    """Sec. 3 of the paper: the obstructed argon glow discharge (SI units,
    Dirichlet wall, sources S_e, S_p with the radial parameters (a, b) of the
    two cases shown), solved by the multilevel prolongation chain 17x17 -> ...
    -> N with the paper's time-step rule (dt from 1 ns, x5 per accepted step,
    capped at 1 ms; steady when the relative density change per step is below
    1e-6), FP64 Newton with the block multigrid preconditioner.  Reports the
    ion current to the cathode, 2 pi e times the ion flow through the cathode
    face, per stage, and the time of each stage.  The ion mobility is a stated
    substitute, so the comparison with the paper's currents (0.59 mA and
    0.035 mA) is context.  The oracle runs the same chain up to 65x65 on one
    host core beside it."""
    import numpy as np
    import torch
    R, d = I.ARGON_R, I.ARGON_D
    ph = dict(I.ARGON)
    P = M.Physics.of(ph)
    sc = M.schedule(coupling=M.NEWTON, dt0=1e-9, growth=5.0, dt_max=1e-3, steady_tol=1e-6, lin_rtol=args.lin_rtol,
                    max_cycles=400, newton_tol=1e-6, max_steps=2000)
    paper = {(30.0, 24.0): 0.59e-3, (10.0, 1.0): 0.035e-3}
    rows = []
    for (a, b) in I.ARGON_CASES:
        N = 16
        z = I.z_cos(N, d)
        V, ne, np_ = I.argon_initial(N, N, z)
        Se, Sp = I.argon_sources(N, N, z, a, b)
        sol = M.Solver(N, N, z, R=R, d=d, krylov_m=30, coarsest=4, r_outer_bc=M.WALL_DIRICHLET)
        t = [sol.upload(V), sol.upload(ne), sol.upload(np_), sol.upload(Se), sol.upload(Sp)]
        stages = []
        t_chain = 0.0
        while True:
            st = sol.state(*t)
            torch.cuda.synchronize()
            t0 = time.time()
            code, rep = sol.steady(P, st, sc)
            torch.cuda.synchronize()
            el = time.time() - t0
            t_chain += el
            if code != 0:
                raise RuntimeError("argon %dx%d: %s" % (N + 1, N + 1, M.lib().mg_last_error()))
            fl = sol.boundary_flow(P, st)
            cur = 2 * np.pi * I.ELEMENTARY_CHARGE * fl[3]
            stages.append(dict(grid="%dx%d" % (N + 1, N + 1), seconds=round(el, 4), steps=rep.steps,
                               rejected=rep.rejected, newton=rep.newton_its, fgmres=rep.vcycles,
                               ion_current_cathode_A=cur, ion_flow_per_rad=dict(cathode=fl[3], anode=fl[4], wall=fl[5])))
            log("argon a=%g b=%g: %s" % (a, b, stages[-1]))
            if N == args.argon_grid:
                break
            N2 = 2 * N
            z2 = I.z_cos(N2, d)
            fine = M.Solver(N2, N2, z2, R=R, d=d, krylov_m=30, coarsest=4, r_outer_bc=M.WALL_DIRICHLET)
            Se2, Sp2 = I.argon_sources(N2, N2, z2, a, b)
            t2 = [fine.field(), fine.field(), fine.field(), fine.upload(Se2), fine.upload(Sp2)]
            M.prolong_state(sol, st, fine, fine.state(*t2), P)
            sol, t, N = fine, t2, N2
        rows.append(dict(a=a, b=b, stages=stages, chain_seconds=round(t_chain, 3),
                         ion_current_cathode_mA=round(stages[-1]["ion_current_cathode_A"] * 1e3, 5),
                         paper_mA=paper[(a, b)] * 1e3))
    out = {"metric": METRIC, "value": rows[0]["chain_seconds"], "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "argon obstructed glow (Sec. 3), SI units, Dirichlet wall; multilevel prolongation "
                                  "chain 17x17 -> %dx%d; value: whole chain of the first case (s)"
                                  % (args.argon_grid + 1, args.argon_grid + 1),
                      "ion_mobility_substitute_m2_per_Vs": I.ARGON_MU_P, "cases": rows}}
    if not args.no_cpu:
        out["cpu_baseline"] = argon_oracle(I, I.ARGON_CASES[0])
    print(json.dumps(out), flush=True)


def argon_oracle(I, case, N1=64):
    """The oracle's argon chain 17x17 -> 65x65 (first case) on one host core:
    its time and its ion current to the cathode."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import numpy as np
    from oracle import newton as NW
    a, b = case
    R, d = I.ARGON_R, I.ARGON_D
    ph = dict(I.ARGON)
    N = 16
    V, ne, np_ = I.argon_initial(N, N, I.z_cos(N, d))
    t0 = time.time()
    while True:
        z = I.z_cos(N, d)
        cp = NW.Coupled(N, N, R, z, ph, wall=1)
        Se, Sp = I.argon_sources(N, N, z, a, b)
        NW.steady(cp, V, ne, np_, Se, Sp, dt0=1e-9, growth=5.0, dt_max=1e-3, tol=1e-6)
        if N == N1:
            break
        V, ne, np_ = NW.prolong_state(I.z_cos(2 * N, d), V, ne, np_, ph, wall=1)
        N *= 2
    el = time.time() - t0
    cur = 2 * np.pi * I.ELEMENTARY_CHARGE * NW.boundary_flow(R, I.z_cos(N1, d), 1, ph["mu_p"], ph["D_p"], V, np_, 1)[0]
    return dict(value=round(el, 2), unit="s", cores=1, kind="oracle", host=_host(),
                sample="the oracle's argon chain 17x17 -> %dx%d, case a=%g b=%g, single thread (sparse LU per "
                       "Newton system); its ion current to the cathode %.5f mA" % (N1 + 1, N1 + 1, a, b, cur * 1e3))


def hybrid(args, M, I):
    """The fluid solver inside a hybrid loop (Sec. 2: transport coefficients
    supplied by lookup tables / a Monte Carlo code, the fluid equations
    solved again after every cycle): 257x257 synthetic workload, cycle 0 the
    steady state of the default chain (constant transport), then per cycle
    the electron mobility and diffusion coefficient from a table of the field
    strength at the current potential (mg_transport_table) and the steady
    solve warm-started from the previous cycle's state (dt from 1e-3, x1.5,
    capped at 0.1; stop at relative change 1e-8).  Reports each cycle's
    solve time, steps, the change of the mobility field and the particle
    flow through the electrodes."""
    import numpy as np
    import torch
    N = args.grid
    phys = dict(I.PHYS)
    fine, t, P, info = chain_to(M, I, N, phys["V_top"], args.lin_rtol)
    st = fine.state(t[0], t[1], t[2], t[3], t[3])
    code, rep = fine.steady(P, st, schedule(M, args.lin_rtol))
    if code != 0:
        raise RuntimeError("cycle 0: %s" % M.lib().mg_last_error())
    Et, mut, Dt = I.electron_transport_table()
    tab = [torch.tensor(a, dtype=torch.float64, device="cuda") for a in (Et, mut, Dt)]
    mu, D, mu_prev = fine.field(), fine.field(), fine.field()
    mup, Dp = fine.field(phys["mu_p"]), fine.field(phys["D_p"])
    sc = M.schedule(coupling=M.NEWTON, dt0=1e-3, growth=1.5, dt_max=0.1, steady_tol=1e-8, lin_rtol=args.lin_rtol,
                    max_cycles=400, newton_tol=1e-6, max_steps=20000)
    rows = [dict(cycle=0, steps=rep.steps, seconds=round(rep.seconds, 4), transport="constant",
                 flow=fine.boundary_flow(P, st))]
    log("hybrid cycle 0: %s" % rows[-1])
    for cyc in range(1, args.hybrid_cycles + 1):
        torch.cuda.synchronize()
        t0 = time.time()
        fine.transport_table(t[0], *tab, mu, D)
        torch.cuda.synchronize()
        t_tab = time.time() - t0
        dmu = float((mu[:, : N + 1] - mu_prev[:, : N + 1]).abs().max() / mu[:, : N + 1].abs().max()) if cyc > 1 else None
        mu_prev.copy_(mu)
        stc = fine.state(t[0], t[1], t[2], t[3], t[3], mu, D, mup, Dp)
        torch.cuda.synchronize()
        t0 = time.time()
        code, rep = fine.steady(P, stc, sc)
        torch.cuda.synchronize()
        el = time.time() - t0
        if code != 0:
            raise RuntimeError("hybrid cycle %d: %s" % (cyc, M.lib().mg_last_error()))
        rows.append(dict(cycle=cyc, steps=rep.steps, newton=rep.newton_its, fgmres=rep.vcycles, seconds=round(el, 4),
                         table_ms=round(t_tab * 1e3, 3), mobility_change=dmu, flow=fine.boundary_flow(P, stc)))
        log("hybrid cycle %d: %s" % (cyc, rows[-1]))
    out = {"metric": METRIC, "value": round(float(np.mean([r["seconds"] for r in rows[1:]])), 4), "unit": "s",
           "n_gpus": 1, "steps": args.hybrid_cycles, "warmup": 0, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "hybrid loop at %dx%d: field-dependent electron transport from a table, steady "
                                  "solve warm-started per cycle (value: mean seconds per cycle)" % (N + 1, N + 1),
                      "cycles": rows, "table": dict(points=len(Et), E_max=float(Et[-1]))}}
    print(json.dumps(out), flush=True)


def fig1(args, M, I):
    """Sec. 3, Fig. 1 re-measured on this GPU: time to the steady state against N for plain relaxation
    (R: the coupled Newton path with its preconditioner reduced to V(2,2)'s four red-black sweeps on the
    finest grid, no coarse correction), multigrid from the random start (M), and multigrid with
    multilevel prolongation (M+L: steady runs 17x17 -> 33x33 -> ... -> N, each prolonged to the next).
    Same physics, schedule and stop rule as the default benchmark (V_top = 1); slopes are d log t /
    d log N between consecutive grids."""
    import math
    import numpy as np
    import torch
    Ns = [int(v) for v in args.fig1_grids.split(",")]
    Rs = [int(v) for v in args.fig1_rgrids.split(",")] if args.fig1_rgrids else []
    if min(Ns) <= 16 or any(n & (n - 1) for n in Ns + Rs):
        raise SystemExit("--fig1-grids: powers of two above 16 (the chain starts at 17x17)")
    phys = dict(I.PHYS)
    P = M.Physics.of(phys)

    def from_random(N, relax):
        log("fig1: %s from the random start at %dx%d" % ("R" if relax else "M", N + 1, N + 1))
        if relax:
            os.environ["MGF_SMOOTHER_ONLY"] = "1"
        try:
            z = I.z_cos(N)
            sol = M.Solver(N, N, z, krylov_m=30, coarsest=4, prec=M.FP64)
        finally:
            os.environ.pop("MGF_SMOOTHER_ONLY", None)
        ne = I.initial_density(N, N, 0)
        t = [sol.upload(I.initial_potential(N, N, z, 0.0, phys["V_top"])), sol.upload(ne), sol.upload(ne),
             sol.upload(I.source(N, N, z))]
        sc = schedule(M, args.lin_rtol)
        if relax:
            sc = M.schedule(dt0=1e-4, growth=1.5, dt_max=0.1, steady_tol=1e-8, lin_rtol=args.lin_rtol,
                            max_steps=2000, max_cycles=args.fig1_rmax_cycles, coupling=M.NEWTON, max_newton=10,
                            newton_tol=1e-6)
        torch.cuda.synchronize()
        t0 = time.time()
        code, rep = sol.steady(P, sol.state(t[0], t[1], t[2], t[3], t[3]), sc)
        torch.cuda.synchronize()
        dt = time.time() - t0
        fields = [sol.download(x) for x in t[:3]]
        return dict(seconds=round(dt, 4), ok=code == 0, steps=rep.steps, newton=rep.newton_its,
                    fgmres=rep.vcycles), fields

    def chained(N):
        log("fig1: M+L chain 17x17 -> %dx%d" % (N + 1, N + 1))
        torch.cuda.synchronize()
        t0 = time.time()
        fine, t, P2, info = chain_to(M, I, N, phys["V_top"], args.lin_rtol, N0=16)
        code, rep = fine.steady(P2, fine.state(t[0], t[1], t[2], t[3], t[3]), schedule(M, args.lin_rtol))
        torch.cuda.synchronize()
        dt = time.time() - t0
        fields = [fine.download(x) for x in t[:3]]
        return dict(seconds=round(dt, 4), ok=code == 0, steps_final=rep.steps,
                    stages=[s_["N"] for s_ in info] + [N]), fields

    def rel(a, b):
        return max(float(np.abs(x - y).max() / max(np.abs(y).max(), 1e-300)) for x, y in zip(a, b))

    from_random(16, False)  # first-use costs (library load, graph capture) outside the timings
    rows = []
    for N in sorted(set(Ns) | set(n for n in Rs)):
        m, fm = from_random(N, False)
        row = dict(N=N + 1, M=m)
        if N in Ns:
            ml, fml = chained(N)
            row["ML"] = ml
            row["ML_vs_M"] = rel(fml, fm)
        if N in Rs:
            r, fr = from_random(N, True)
            row["R"] = r
            row["R_vs_M"] = rel(fr, fm)
        rows.append(row)
        log("fig1 %dx%d: %s" % (N + 1, N + 1, row))
    slopes = {}
    for key in ("R", "M", "ML"):
        pts = [(r["N"], r[key]["seconds"]) for r in rows if key in r and r[key]["ok"]]
        slopes[key] = [round(math.log(t2 / t1) / math.log(n2 / n1), 2)
                       for (n1, t1), (n2, t2) in zip(pts, pts[1:])]
    print(json.dumps({"fig1": rows, "slopes": slopes, "V_top": phys["V_top"], "lin_rtol": args.lin_rtol}),
          flush=True)


def network(args, M):
    """Throughput of the warm-start network's kernels with random weights at
    257x257 (the timings do not depend on the weights)."""
    import numpy as np
    from paper_0811_4446_amd import warmstart as WS
    rng = np.random.default_rng(0)
    p = []
    for ci, co in [(7, 32), (32, 32), (32, 32), (32, 3)]:
        p.append(rng.normal(size=co * ci * 9) * np.sqrt(2.0 / (9 * ci)))
        p.append(rng.normal(size=co) * 0.1)
    net = M.Net(np.concatenate(p))
    rows = [WS.network_throughput(net, B=b, H=257, W=257) for b in (1, 8)]
    for r in rows:
        log("network throughput: %s" % r)
    f8 = rows[1]
    print(json.dumps({"metric": "warm-start network forward throughput", "value": f8["forward_tflops"],
                      "unit": "TFLOP/s", "n_gpus": 1, "higher_is_better": True, "dtype": "bf16",
                      "data": "synthetic", "config": {"workload": "4-layer 3x3 CNN 7-32-32-32-3 at 257x257",
                                                      "rows": rows}}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--lin-rtol", type=float, default=LIN_RTOL)
    ap.add_argument("--vtops", type=str, default="0.5,1,2")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-1025", action="store_true", help="skip the 1025x1025 FP64 / FP32 time-to-steady")
    ap.add_argument("--grid", type=int, default=256, help="finest N (256: 257x257 workload; 1024 for 1025x1025)")
    ap.add_argument("--sweep", action="store_true", help="batched parameter sweep instead of the chain")
    ap.add_argument("--nprob", type=int, default=512)
    ap.add_argument("--concurrent", action="store_true", help="sweep: all size classes at once (own streams)")
    ap.add_argument("--sweep-ref", type=int, default=0, help="solve this many problems per size class of the "
                                                              "sweep one at a time (reference for the batch)")
    ap.add_argument("--learned", action="store_true", help="learned warm start: train and compare on 257x257")
    ap.add_argument("--n-train", type=int, default=128)
    ap.add_argument("--n-val", type=int, default=16)
    ap.add_argument("--n-test", type=int, default=16)
    ap.add_argument("--n-timed", type=int, default=6)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--save-weights", type=str, default="")
    ap.add_argument("--criterion", choices=["run", "newton", "residual"], default="run",
                    help="fallback test of the learned warm start")
    ap.add_argument("--roofline-only", action="store_true", help="only the roofline timing (+ copy calibration)")
    ap.add_argument("--vcycle", action="store_true", help="scalar path: 65x65 decoupled step and V-cycle GB/s")
    ap.add_argument("--reps", type=int, default=200, help="timed half-sweeps of the roofline measurement")
    ap.add_argument("--trace-summary", type=str, default="", help="summarise a rocprofv3 CSV and exit")
    ap.add_argument("--fig1", action="store_true", help="Sec. 3 Fig. 1 re-measured: R / M / M+L time vs N")
    ap.add_argument("--argon", action="store_true", help="Sec. 3 argon discharge: ion current to the cathode")
    ap.add_argument("--hybrid", action="store_true", help="hybrid loop: table transport, warm-started solves")
    ap.add_argument("--zebra", action="store_true", help="time-to-steady: point vs block zebra z-line smoother")
    ap.add_argument("--hybrid-cycles", type=int, default=5)
    ap.add_argument("--argon-grid", type=int, default=256, help="finest N of the argon chain (power of two >= 16)")
    ap.add_argument("--fig1-grids", type=str, default="32,64,128,256", help="N values, each > 16")
    ap.add_argument("--fig1-rgrids", type=str, default="16,32",
                    help="N values of the relaxation-only runs (65x65 and above take minutes)")
    ap.add_argument("--fig1-rmax-cycles", type=int, default=20000, help="FGMRES iterations per Newton, R runs")
    ap.add_argument("--network", action="store_true",
                    help="warm-start network alone: forward (batch 1 and 8) and gradient (batch 8) at 257x257")
    ap.add_argument("--prec", choices=["fp64", "fp32", "both"], default="fp64",
                    help="block preconditioner precision (FGMRES and Newton stay FP64)")
    args = ap.parse_args()
    if args.trace_summary:
        return trace_summary(args.trace_summary)
    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU only (asked for %d); a batch of independent "
              "solves would shard across GPUs by problem" % args.gpus)
        sys.exit(2)

    import torch
    from paper_0811_4446_amd import inputs as I
    from paper_0811_4446_amd import mgfluid as M

    if args.roofline_only:
        return roofline_only(args, M, I)
    if args.vcycle:
        return vcycle_bench(args, M, I)
    if args.sweep_ref:
        return sweep_reference(args, M, I)
    if args.sweep:
        return sweep(args, M, I)
    if args.learned:
        return learned(args, M, I)
    if args.network:
        return network(args, M)
    if args.fig1:
        return fig1(args, M, I)
    if args.argon:
        return argon(args, M, I)
    if args.hybrid:
        return hybrid(args, M, I)
    vtops = [float(v) for v in args.vtops.split(",")]
    N = args.grid
    if args.zebra:
        return compare_smoothers(args, M, I, N, vtops)
    if args.prec != "fp64":
        return compare_precisions(args, M, I, N, vtops)
    cases = []
    for vt in vtops:
        fine, t, P, info = chain_to(M, I, N, vt, args.lin_rtol)
        log("prep V_top=%g: %s" % (vt, info))
        cases.append((vt, fine, t, P, info))
    # initial 257x257 states for every timed run, resident in HBM
    runs = []
    for k in range(args.warmup + args.steps):
        for vt, fine, t, P, info in cases:
            runs.append((vt, fine, [x.clone() for x in t[:3]] + [t[3]], P))
    torch.cuda.synchronize()
    for r in range(args.warmup * len(cases)):
        vt, fine, t, P = runs[r]
        code, rep = fine.steady(P, fine.state(t[0], t[1], t[2], t[3], t[3]), schedule(M, args.lin_rtol))
    torch.cuda.synchronize()
    reps = []
    t0 = time.time()
    for r in range(args.warmup * len(cases), len(runs)):
        vt, fine, t, P = runs[r]
        code, rep = fine.steady(P, fine.state(t[0], t[1], t[2], t[3], t[3]), schedule(M, args.lin_rtol))
        if code != 0:
            raise RuntimeError("257x257 steady failed: %s" % M.lib().mg_last_error())
        reps.append((vt, rep.as_dict()))
    torch.cuda.synchronize()
    elapsed = time.time() - t0
    nrun = args.steps * len(cases)
    value = elapsed / nrun
    for vt, rd in reps:
        log("V_top=%g steps=%d newton=%d fgmres=%d t=%.3f s" % (vt, rd["steps"], rd["newton_its"],
                                                              rd["vcycles"], rd["seconds"]))
    roof_dom = roofline_dominant(cases[-1][1], N)
    roof_fine = roofline(cases[-1][1], N, resident="Infinity Cache (257x257 working set about 19 MB)")
    log("roofline (dominant kernel): %s" % roof_dom)
    steps_mean = sum(rd["steps"] for _, rd in reps) / len(reps)
    newton_mean = sum(rd["newton_its"] for _, rd in reps) / len(reps)
    per_v = []
    for vt in vtops:
        rs = [rd for v, rd in reps if v == vt]
        secs = sorted(rd["seconds"] for rd in rs)
        per_v.append(dict(V_top=vt, steps=rs[0]["steps"], newton=rs[0]["newton_its"], fgmres=rs[0]["vcycles"],
                          seconds_median=round(secs[len(secs) // 2], 4), seconds_min=round(secs[0], 4),
                          seconds_max=round(secs[-1], 4), runs=len(rs)))
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(elapsed / args.steps * 1e3, 2),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "steady 257x257 from the prolonged 129x129 steady state, coupled Newton BE, "
                               "dt x1.5 to 0.1, stop at relative change 1e-8 (value: mean time-to-steady per "
                               "voltage, FP64)",
                   "grid": "257x257, r uniform, z cos-stretched", "V_top": vtops,
                   "lin_rtol": args.lin_rtol, "mean_steps": steps_mean, "per_voltage": per_v,
                   "chain": [dict(V_top=c[0], stages=c[4]) for c in cases],
                   "roofline_finest_257": roof_fine},
        "roofline": roof_dom,
    }
    if not args.no_1025:
        out["config"]["t1025"] = time_to_steady_1025(args, M, I, vtops)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(I, int(round(newton_mean)))
    print(json.dumps(out), flush=True)


def compare_smoothers(args, M, I, N, vtops):
    """Time-to-steady on N x N from the prolonged N/2 steady state with the
    collective red-black point smoother and with the block zebra z-line
    smoother (MG_SMOOTH_ZEBRA_BLOCK), same state, schedule and FP64 path;
    one run per smoother and voltage after one untimed run."""
    import numpy as np
    import torch
    rows = []
    for vt in vtops:
        fine, t, P, info = chain_to(M, I, N, vt, args.lin_rtol)
        init = [x.clone() for x in t[:3]]
        finals = {}
        for name, sm in (("point", M.SMOOTH_ZEBRA), ("zebra_block", M.SMOOTH_ZEBRA_BLOCK)):
            sol = M.Solver(N, N, I.z_cos(N), krylov_m=30, coarsest=4, smoother=sm)
            for k in range(2):
                tt = [x.clone() for x in init] + [t[3]]
                torch.cuda.synchronize()
                t0 = time.time()
                code, rep = sol.steady(P, sol.state(tt[0], tt[1], tt[2], tt[3], tt[3]), schedule(M, args.lin_rtol))
                torch.cuda.synchronize()
                el = time.time() - t0
                if code != 0:
                    raise RuntimeError("steady (%s) failed: %s" % (name, M.lib().mg_last_error()))
            finals[name] = [sol.download(x) for x in tt[:3]]
            rows.append(dict(V_top=vt, smoother=name, seconds=round(el, 4), steps=rep.steps,
                             newton=rep.newton_its, fgmres=rep.vcycles))
            log("%dx%d V_top=%g %s: %.3f s, %d steps, %d Newton, %d FGMRES" % (N + 1, N + 1, vt, name, el, rep.steps,
                                                                              rep.newton_its, rep.vcycles))
        rows.append(dict(V_top=vt, zebra_vs_point_maxrel=[
            float(np.abs(a - b).max() / np.abs(b).max()) for a, b in zip(finals["zebra_block"], finals["point"])]))
    mean = {k: round(sum(r["seconds"] for r in rows if r.get("smoother") == k) / len(vtops), 4)
            for k in ("point", "zebra_block")}
    out = {"metric": METRIC, "value": mean["zebra_block"], "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 1,
           "higher_is_better": False, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "steady %dx%d from the prolonged %dx%d state, point vs block zebra smoother "
                                  "(value: zebra mean)" % (N + 1, N + 1, N // 2 + 1, N // 2 + 1),
                      "mean_seconds": mean, "runs": rows}}
    print(json.dumps(out), flush=True)


def time_to_steady_1025(args, M, I, vtops, N=1024):
    """1025x1025: for each voltage the chain 65 -> 129 -> 257 -> 513 (FP64,
    steady at each stage) prolonged to 1025x1025, then the 1025x1025 steady
    solve from that state with the FP64 block preconditioner and with the
    FP32 one (Newton, FGMRES and the stop rules in FP64 for both); one run
    per form and voltage.  Also the roofline of the finest-level sweep on the
    1025x1025 Jacobian (working set beyond the Infinity Cache)."""
    import numpy as np
    import torch
    rows, roof, dmax = [], None, []
    for vt in vtops:
        fine, t, P, info = chain_to(M, I, N, vt, args.lin_rtol)
        init = [x.clone() for x in t[:3]]
        finals = {}
        for form, prec in (("fp64", M.FP64), ("fp32", M.FP32_IR)):
            sol = M.Solver(N, N, I.z_cos(N), krylov_m=30, coarsest=4, prec=prec)
            tt = [x.clone() for x in init] + [t[3]]
            torch.cuda.synchronize()
            t0 = time.time()
            code, rep = sol.steady(P, sol.state(tt[0], tt[1], tt[2], tt[3], tt[3]), schedule(M, args.lin_rtol))
            torch.cuda.synchronize()
            el = time.time() - t0
            if code != 0:
                raise RuntimeError("1025x1025 steady failed: %s" % M.lib().mg_last_error())
            finals[form] = [sol.download(x) for x in tt[:3]]
            rows.append(dict(V_top=vt, form=form, seconds=round(el, 3), steps=rep.steps, newton=rep.newton_its,
                             fgmres=rep.vcycles))
            log("1025: %s" % rows[-1])
            if form == "fp64" and roof is None:
                roof = roofline(sol, N, resident="HBM (1025x1025 working set about 300 MB, beyond the "
                                                 "256 MB Infinity Cache)")
            del sol
            torch.cuda.empty_cache()
        dmax.append(max(float(np.abs(a - b).max() / np.abs(b).max()) for a, b in zip(finals["fp32"], finals["fp64"])))
        del fine, t, init
        torch.cuda.empty_cache()
    mean = {f: round(float(np.mean([r["seconds"] for r in rows if r["form"] == f])), 4) for f in ("fp64", "fp32")}
    return dict(workload="steady 1025x1025 from the prolonged 513x513 steady state (chain from 65x65), mean of "
                         "the voltages", fp64_mean_s=mean["fp64"], fp32_preconditioner_mean_s=mean["fp32"],
                fp32_vs_fp64_final_state_maxrel=max(dmax), runs=rows, roofline_finest_1025=roof)


if __name__ == "__main__":
    main()
