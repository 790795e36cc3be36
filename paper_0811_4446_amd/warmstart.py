"""Learned warm start for the multilevel prolongation (Sec. 2).

The paper starts the fine-grid time integration from the steady coarse
solution extrapolated to the fine grid.  Here a small convolutional network
(the library's wn_* kernels) predicts the correction from that prolonged
state to the fine steady state; the steady solver is unchanged and decides
convergence.  If the time integration from the network's start fails, it
is repeated from the plain prolongation (fallback).  A static test before
the run (steady residual or Newton correction of the two starts) is
available too, but the residual is dominated by the prediction's
grid-scale noise and does not predict the step count.

Pipeline (all numerical work in the library's kernels; torch holds memory):
  1. data: for parameter draws (V_top, mobility ratio) steady solves on
     65x65 from seeded random starts, prolongation to 129x129, steady,
     prolongation to 257x257 ("up"), and the plain 257x257 steady solve from
     "up" (the target, and the baseline step count) -- each stage one batch;
  2. training: Adam on the mean squared error of the scaled correction;
  3. evaluation on held-out draws: steps and time to steady from the
     network's start versus from "up", fallback count, and the agreement of
     the two final states once both are polished by steady Newton.
"""
import time

import numpy as np
import torch

from . import inputs as I
from . import mgfluid as M


def _phys(d):
    ph = dict(I.PHYS)
    ph.update(V_top=d["V_top"], mu_e=d["mu_e"], D_e=d["D_e"], mu_p=d["mu_p"], D_p=d["D_p"])
    return ph


def _sched(lin_rtol=1e-3, max_steps=20000):
    return M.schedule(coupling=M.NEWTON, lin_rtol=lin_rtol, max_cycles=200, newton_tol=1e-6, steady_tol=1e-8,
                      max_steps=max_steps)


def _state_of(batch, p):
    v = batch.views[p]
    return M.State(v["V"].data_ptr(), v["ne"].data_ptr(), v["np"].data_ptr(), v["Se"].data_ptr(),
                   v["Sp"].data_ptr())


def draws(n, seed):
    return I.sweep_draws(n, seed, sizes=(256,))


def generate(ds, log=print, prec=M.FP32_IR, chunk=64, N=256):
    """Solver-generated samples for the draws `ds` (list of dicts), in
    batches of at most `chunk` problems, on the chain N/4 -> N/2 -> N."""
    if len(ds) > chunk:
        parts = [generate(ds[i:i + chunk], log, prec, chunk, N) for i in range(0, len(ds), chunk)]
        out = dict(parts[0])
        for k in ("draws", "phys", "up", "steady", "NS", "plain_steps"):
            out[k] = sum((q[k] for q in parts), [])
        out["X"] = torch.cat([q["X"] for q in parts])
        out["T"] = torch.cat([q["T"] for q in parts])
        out["gen_info"] = [q["gen_info"] for q in parts]
        return out
    n = len(ds)
    phys = [_phys(d) for d in ds]
    P = [M.Physics.of(ph) for ph in phys]
    t0 = time.time()
    prev = None
    info = {}
    Nf = N
    for N in (Nf // 4, Nf // 2, Nf):
        z = I.z_cos(N)
        B = M.Batch(N, N, z, n, prec=prec, krylov_m=20)
        S = I.source(N, N, z)
        for p in range(n):
            if prev is None:
                ne = I.initial_density(N, N, 5000 + p)
                B.set_problem(p, I.initial_potential(N, N, z, 0.0, phys[p]["V_top"]), ne, ne.copy(), S)
            else:
                for name in ("Se", "Sp"):
                    B.views[p][name][:, : N + 1] = torch.from_numpy(S).to(B.device)
                M.prolong_state(prev, _state_of(prev, p), B, _state_of(B, p), P[p])
        torch.cuda.synchronize()
        if N == Nf:
            up = [{k: B.views[p][k].clone() for k in ("V", "ne", "np", "Se")} for p in range(n)]
        ts = time.time()
        code, reps = B.steady(P, _sched())
        torch.cuda.synchronize()
        info[N] = dict(seconds=time.time() - ts, code=code, steps=[r["steps"] for r in reps])
        log("data %dx%d: %d problems, %.1f s, steps %.0f mean" % (N + 1, N + 1, n, info[N]["seconds"],
                                                                  np.mean(info[N]["steps"])))
        if prev is not None:
            prev.close()
        prev = B
    steady = [{k: prev.views[p][k].clone() for k in ("V", "ne", "np")} for p in range(n)]
    prev.close()
    # features and targets on the finest context
    z = I.z_cos(Nf)
    sol = M.Solver(Nf, Nf, z, krylov_m=20, coarsest=4, prec=prec)
    X = torch.empty((n, 7, Nf + 1, Nf + 1), dtype=torch.float32, device=sol.device)
    T = torch.empty((n, 3, Nf + 1, Nf + 1), dtype=torch.float32, device=sol.device)
    NS = []
    for p in range(n):
        su = sol.state(up[p]["V"], up[p]["ne"], up[p]["np"], up[p]["Se"], up[p]["Se"])
        ss = sol.state(steady[p]["V"], steady[p]["ne"], steady[p]["np"], up[p]["Se"], up[p]["Se"])
        f, ns = M.features(sol, su, phys[p]["V_top"], ds[p]["ratio"])
        X[p] = f
        T[p] = M.targets(sol, su, ss, phys[p]["V_top"], ns)
        NS.append(ns)
    torch.cuda.synchronize()
    log("data total %.1f s" % (time.time() - t0))
    return dict(draws=ds, phys=phys, up=up, steady=steady, X=X, T=T, NS=NS, plain_steps=info[Nf]["steps"],
                sol=sol, gen_info=info, N=Nf)


def init_params(seed):
    rng = np.random.default_rng(seed)
    out = []
    layers = [(7, 32), (32, 32), (32, 32), (32, 3)]
    for l, (ci, co) in enumerate(layers):
        scale = np.sqrt(2.0 / (9 * ci)) * (0.1 if l == 3 else 1.0)  # start near the plain prolongation
        out.append(rng.normal(size=co * ci * 9) * scale)
        out.append(np.zeros(co))
    return np.concatenate(out).astype(np.float32)


def train(data, val, epochs=60, batch=8, lr=1e-3, seed=0, log=print):
    net = M.Net(init_params(seed))
    X, T = data["X"], data["T"]
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    hist = []
    t0 = time.time()
    for ep in range(epochs):
        perm = rng.permutation(n)
        losses = []
        for s in range(0, n - batch + 1, batch):
            idx = torch.as_tensor(perm[s:s + batch], device=X.device)
            losses.append(net.train_step(X[idx].contiguous(), T[idx].contiguous(), lr=lr))
        vl = evaluate_loss(net, val)
        hist.append((ep, float(np.mean(losses)), vl))
        if ep % 10 == 0 or ep == epochs - 1:
            log("epoch %d train %.5f val %.5f (%.1f s)" % (ep, hist[-1][1], vl, time.time() - t0))
    return net, hist


def evaluate_loss(net, data, batch=8):
    X, T = data["X"], data["T"]
    tot, cnt = 0.0, 0
    for s in range(0, X.shape[0], batch):
        x, t = X[s:s + batch].contiguous(), T[s:s + batch].contiguous()
        loss, _ = net.grad(x, t)
        tot += loss * x.shape[0]
        cnt += x.shape[0]
    return tot / max(cnt, 1)


def newton_distance(sol, phys, fields, S):
    """Size of one Newton correction towards the steady state (dt -> inf)
    from `fields` (diagnostic of the distance to the steady state)."""
    t = [fields["V"].clone(), fields["ne"].clone(), fields["np"].clone()]
    st = sol.state(t[0], t[1], t[2], S, S)
    sc = M.schedule(coupling=M.NEWTON, lin_rtol=1e-3, max_cycles=200, max_newton=1, newton_tol=1e-300)
    rep = sol.step(phys, st, 1e30, sc, raise_on_noconv=False)
    return rep.last_change


def polish(sol, phys, fields, S, iters=8):
    """Newton on the steady equations (dt -> inf) from a near-steady state,
    to a relative correction of 1e-13: the discrete steady solution that
    every converged start approaches.  Returns the polished fields."""
    t = [fields["V"].clone(), fields["ne"].clone(), fields["np"].clone()]
    st = sol.state(t[0], t[1], t[2], S, S)
    sc = M.schedule(coupling=M.NEWTON, lin_rtol=1e-10, max_cycles=400, max_newton=iters, newton_tol=1e-13)
    rep = sol.step(phys, st, 1e30, sc, raise_on_noconv=False)
    return dict(V=t[0], ne=t[1], np=t[2]), rep


def maxrel(a, b):
    return max(float((a[k] - b[k]).abs().max() / b[k].abs().max()) for k in ("V", "ne", "np"))


def converged(rep, sched_tol=1e-8):
    return rep["steps"] > 0 and rep["last_change"] < sched_tol


def warm_start_states(net, data, criterion="run", log=print):
    """Initial 257x257 states from the network.

    The fallback to the plain prolongation is decided by `criterion`:
    "run" (default): the network's start is used, and the plain start only
    if the steady run from it fails (no convergence within the schedule);
    "residual": before the run, if the steady residual of the network's
    start is not below the plain start's; "newton": likewise with the size
    of one steady Newton correction.  Both static measures are computed for
    every draw (with the error against the known steady state, a diagnostic
    only) so that their predictive value can be reported."""
    sol = data["sol"]
    out = []
    for p in range(len(data["draws"])):
        up = data["up"][p]
        ph = data["phys"][p]
        P = M.Physics.of(ph)
        pred = net.forward(data["X"][p:p + 1].contiguous())[0].contiguous()
        g = {k: sol.field() for k in ("V", "ne", "np")}
        su = sol.state(up["V"], up["ne"], up["np"], up["Se"], up["Se"])
        sg = sol.state(g["V"], g["ne"], g["np"], up["Se"], up["Se"])
        M.apply_prediction(sol, su, pred, ph["V_top"], data["NS"][p], P, sg)
        o = dict(raw=g, r_up=sol.steady_residual(P, su), r_nn=sol.steady_residual(P, sg),
                 d_up=newton_distance(sol, P, up, up["Se"]), d_nn=newton_distance(sol, P, g, up["Se"]))
        st = data["steady"][p]
        o["e_up"], o["e_nn"] = maxrel(up, st), maxrel(g, st)
        if criterion == "run":
            o["fallback"] = False
        else:
            key = "r" if criterion == "residual" else "d"
            o["fallback"] = not (o[key + "_nn"] < o[key + "_up"])
        out.append(o)
    for nm, what in (("e", "error vs steady"), ("r", "steady residual"), ("d", "Newton distance")):
        log("  %s ratio network/plain per draw: %s" % (what, ["%.2f" % (o[nm + "_nn"] / o[nm + "_up"]) for o in out]))
    return out


def compare(net, data, timed=8, criterion="run", log=print, prec=M.FP32_IR, attempt_steps=None):
    """Steps to steady for every test draw from the plain prolongation and
    from the network's start (one batch each; batched solves are bitwise
    those of single solves), the start the fallback rule chooses, the
    agreement of the final states after a steady Newton polish, and
    single-problem time-to-steady (first `timed` draws).  `attempt_steps`
    caps the steps of the run from the network's start (a cap that is too
    small forces the fallback)."""
    n = len(data["draws"])
    Nf = data["N"]
    P = [M.Physics.of(ph) for ph in data["phys"]]
    starts = warm_start_states(net, data, criterion=criterion, log=log)
    z = I.z_cos(Nf)
    res = {}
    for name in ("plain", "raw"):
        B = M.Batch(Nf, Nf, z, n, prec=prec, krylov_m=20)
        for p in range(n):
            src = data["up"][p] if name == "plain" else starts[p]["raw"]
            for k in ("V", "ne", "np"):
                B.views[p][k].copy_(src[k])
            for k in ("Se", "Sp"):
                B.views[p][k].copy_(data["up"][p]["Se"])
        torch.cuda.synchronize()
        t0 = time.time()
        cap = attempt_steps if (name == "raw" and attempt_steps) else 20000
        code, reps = B.steady(P, _sched(max_steps=cap))
        torch.cuda.synchronize()
        res[name] = dict(batch_seconds=time.time() - t0, reps=reps,
                         finals=[{k: B.views[p][k].clone() for k in ("V", "ne", "np")} for p in range(n)])
        B.close()
    sp = np.array([r["steps"] for r in res["plain"]["reps"]])
    sr = np.array([r["steps"] for r in res["raw"]["reps"]])
    if criterion == "run":
        for p in range(n):
            starts[p]["fallback"] = not converged(res["raw"]["reps"][p])
    fb = np.array([s["fallback"] for s in starts])
    # chosen start: the network's, or the plain one (after the failed run for "run")
    sl = np.where(fb, sp + (sr if criterion == "run" else 0), sr)
    ratio, rraw = sl / sp, sr / sp
    log("steps plain   %s" % sp.tolist())
    log("steps network %s" % sr.tolist())
    agree = {nm: float(np.mean([(s[nm + "_nn"] < s[nm + "_up"]) == (r < q) for s, r, q in zip(starts, sr, sp)]))
             for nm in ("e", "r", "d")}
    chosen = []
    for p in range(n):
        chosen.append(res["plain"]["finals"][p] if fb[p] else res["raw"]["finals"][p])
    # the check of the answer: both final states, polished by steady Newton, are the same discrete solution
    sol = data["sol"]
    d_final, d_pol, d_to_pol = [], [], []
    for p in range(n):
        S = data["up"][p]["Se"]
        a, b = res["raw"]["finals"][p], res["plain"]["finals"][p]
        d_final.append(maxrel(a, b))
        pa, ra = polish(sol, P[p], a, S)
        pb, rb = polish(sol, P[p], b, S)
        d_pol.append(maxrel(pa, pb))
        d_to_pol.append(max(maxrel(a, pa), maxrel(b, pb)))
    # single-problem wall clock, FP64 preconditioner; the learned start's time
    # includes computing its input planes, the network and applying its output
    sol64 = M.Solver(Nf, Nf, z, krylov_m=30, coarsest=4, prec=M.FP64)
    single = {"plain": [], "learned": []}
    for p in range(min(timed, n)):
        for name in ("plain", "learned"):
            use_plain = name == "plain" or (fb[p] and criterion != "run")
            src = data["up"][p] if use_plain else starts[p]["raw"]
            t_inf = 0.0
            if not use_plain:
                up, ph = data["up"][p], data["phys"][p]
                su = sol64.state(up["V"], up["ne"], up["np"], up["Se"], up["Se"])
                g = {k: sol64.field() for k in ("V", "ne", "np")}
                torch.cuda.synchronize()
                ti = time.time()
                feat, ns = M.features(sol64, su, ph["V_top"], data["draws"][p]["ratio"])
                pred = net.forward(feat.unsqueeze(0).contiguous())[0].contiguous()
                M.apply_prediction(sol64, su, pred, ph["V_top"], ns, P[p], sol64.state(g["V"], g["ne"], g["np"],
                                                                                     up["Se"], up["Se"]))
                torch.cuda.synchronize()
                t_inf = time.time() - ti
                src = g
            t = [src["V"].clone(), src["ne"].clone(), src["np"].clone(), data["up"][p]["Se"]]
            st = sol64.state(t[0], t[1], t[2], t[3], t[3])
            torch.cuda.synchronize()
            t0 = time.time() - t_inf
            cap = attempt_steps if (name == "learned" and attempt_steps) else 20000
            code, rep = sol64.steady(P[p], st, _sched(max_steps=cap))
            if name == "learned" and criterion == "run" and (code != 0 or rep.last_change >= 1e-8):
                src = data["up"][p]
                t = [src["V"].clone(), src["ne"].clone(), src["np"].clone(), data["up"][p]["Se"]]
                st = sol64.state(t[0], t[1], t[2], t[3], t[3])
                code, rep = sol64.steady(P[p], st, _sched())
            torch.cuda.synchronize()
            single[name].append(dict(seconds=time.time() - t0, steps=rep.steps, code=code, inference=t_inf))
    summary = dict(test_draws=n, criterion=criterion, fallbacks=int(fb.sum()),
                   steps_plain_mean=float(sp.mean()), steps_learned_mean=float(sl.mean()),
                   steps_network_start_mean=float(sr.mean()),
                   steps_ratio_median=float(np.median(ratio)), steps_ratio_p90=float(np.percentile(ratio, 90)),
                   steps_ratio_worst=float(ratio.max()),
                   network_start_steps_ratio_median=float(np.median(rraw)),
                   network_start_steps_ratio_worst=float(rraw.max()),
                   fewer_steps_predicted_by=agree,
                   residual_ratio_median=float(np.median([s["r_nn"] / s["r_up"] for s in starts])),
                   newton_distance_ratio_median=float(np.median([s["d_nn"] / s["d_up"] for s in starts])),
                   error_ratio_median=float(np.median([s["e_nn"] / s["e_up"] for s in starts])),
                   final_states_maxrel_diff_max=float(max(d_final)),
                   polished_states_maxrel_diff_max=float(max(d_pol)),
                   final_to_polished_maxrel_max=float(max(d_to_pol)),
                   single_seconds_plain=[round(s["seconds"], 3) for s in single["plain"]],
                   single_seconds_learned=[round(s["seconds"], 3) for s in single["learned"]],
                   single_inference_seconds=[round(s["inference"], 4) for s in single["learned"]],
                   single_steps_plain=[s["steps"] for s in single["plain"]],
                   single_steps_learned=[s["steps"] for s in single["learned"]],
                   time_ratio_median=(float(np.median([l["seconds"] / p_["seconds"]
                                                       for l, p_ in zip(single["learned"], single["plain"])]))
                                      if single["plain"] else None),
                   batch_seconds=dict(plain=res["plain"]["batch_seconds"], network=res["raw"]["batch_seconds"]))
    log(summary)
    summary["_chosen_finals"] = chosen
    summary["_plain_finals"] = res["plain"]["finals"]
    return summary


def network_throughput(net, B=8, H=257, W=257, reps=20, peak_tflops=2500.0):
    """Timed forward passes and gradient evaluations of the network on a
    B x 7 x H x W batch: milliseconds, achieved TFLOP/s and the fraction of
    the dense bf16 MFMA peak.  Flops per pixel: forward 2*9*(7*32 + 32*32 +
    32*32 + 32*3) = 42,624; gradient = forward + input gradients of layers
    2-4 (38,592) + weight gradients (42,624)."""
    x = torch.randn((B, 7, H, W), dtype=torch.float32, device=net.device)
    t = torch.randn((B, 3, H, W), dtype=torch.float32, device=net.device)
    px = B * H * W
    f_fwd, f_grad = 42624.0 * px, (42624.0 + 38592.0 + 42624.0) * px
    net.forward(x)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(net.stream)
    for _ in range(reps):
        net.forward(x)
    b.record(net.stream)
    b.synchronize()
    fwd_ms = a.elapsed_time(b) / reps
    net.grad(x, t)
    torch.cuda.synchronize()
    t0 = time.time()
    for _ in range(reps):
        net.grad(x, t)
    torch.cuda.synchronize()
    grad_ms = (time.time() - t0) * 1e3 / reps
    return dict(batch=B, H=H, W=W, forward_ms=round(fwd_ms, 3), forward_tflops=round(f_fwd / fwd_ms / 1e9, 2),
                forward_mfma_frac=round(f_fwd / fwd_ms / 1e9 / peak_tflops, 5), grad_ms=round(grad_ms, 3),
                grad_tflops=round(f_grad / grad_ms / 1e9, 2), grad_mfma_frac=round(f_grad / grad_ms / 1e9 / peak_tflops, 5))
