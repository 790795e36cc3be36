"""Autotuner of the launch shapes of a batched solve.

For a batch (one grid size, a given number of problems and precision) it
times every candidate (radial rows per workgroup of the 2D kernels x the
largest level run by the single-workgroup coarse sub-cycle) on two real
time steps of the batch from its initial state, keeps the fastest, and
caches the choice in JSON keyed by GPU architecture, grid, batch size and
precision.  The states are restored before and after probing.
"""
import json
import os
import time

import torch

from . import mgfluid as M

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")
ROWS = (1, 2, 4, 8)
FUSE = (16, 32, 64)


def arch():
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def key_of(batch, prec):
    return "%s:%dx%d:B%d:%s" % (arch(), batch.nr + 1, batch.nz + 1, batch.n, "fp32" if prec else "fp64")


def load_cache(path=CACHE):
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def tune(batch, phys_list, reset, prec, path=CACHE, log=None):
    """Pick (rows_per_block, fuse_max) for `batch`; `reset()` rewrites the
    problems' initial states.  Returns (choice, timings)."""
    cache = load_cache(path)
    key = key_of(batch, prec)
    if key in cache:
        ty, fm = cache[key]["rows_per_block"], cache[key]["fuse_max"]
        batch.tune(ty, fm)
        return (ty, fm), cache[key].get("timings", {})
    probe = M.schedule(coupling=M.NEWTON, lin_rtol=1e-3, max_cycles=200, newton_tol=1e-6, steady_tol=1e-8,
                       max_steps=2)
    timings = {}
    for ty in ROWS:
        for fm in FUSE:
            try:
                batch.tune(ty, fm)
            except M.MGError:
                continue
            reset()
            torch.cuda.synchronize()
            t0 = time.time()
            batch.steady(phys_list, probe)
            torch.cuda.synchronize()
            timings["%d,%d" % (ty, fm)] = time.time() - t0
            if log:
                log("tune %s rows=%d fuse=%d: %.4f s" % (key, ty, fm, timings["%d,%d" % (ty, fm)]))
    best = min(timings, key=timings.get)
    ty, fm = (int(v) for v in best.split(","))
    batch.tune(ty, fm)
    reset()
    cache[key] = dict(rows_per_block=ty, fuse_max=fm, timings=timings)
    try:
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    except OSError:
        pass
    return (ty, fm), timings
