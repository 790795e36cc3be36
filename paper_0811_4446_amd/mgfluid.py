"""Thin Python binding of libmgfluid.so (include/mgfluid.h).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels.  PyTorch provides device memory (tensors) and the stream.
Device fields are float64 tensors of shape (nr+1, pitch) -- z contiguous,
columns beyond nz are padding; ``Solver.field`` / ``Solver.upload`` create
them and ``Solver.download`` returns the (nr+1, nz+1) numpy view.

The library must be built (``python -m paper_0811_4446_amd.build``); there
is no fallback: a missing library or GPU raises.
"""
import ctypes
import math
import os

import numpy as np
import torch  # loaded first so that the library binds to torch's HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgfluid.so")

ABI_VERSION = 2
FP64, FP32_IR = 0, 1
POISSON, ELECTRON, ION = 0, 1, 2
SMOOTH_RB, SMOOTH_ZEBRA, SMOOTH_ZEBRA_BLOCK = 0, 1, 2
DECOUPLED, NEWTON = 0, 2
WALL_ZERO_FLUX, WALL_DIRICHLET = 0, 1

ERRORS = {-1: "MG_EINVAL", -2: "MG_EHIP", -3: "MG_ENOCONV", -4: "MG_ENONFINITE",
          -5: "MG_EREJECT", -6: "MG_ENOMEM"}

_D, _I32, _I64, _VP = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
_PD = ctypes.POINTER(ctypes.c_double)


class GridDesc(ctypes.Structure):
    _fields_ = [("abi_version", _I32), ("nr", _I32), ("nz", _I32), ("R", _D), ("d", _D),
                ("z_host", _PD), ("coarsest_n", _I32), ("nu1", _I32), ("nu2", _I32),
                ("smoother", _I32), ("prec", _I32), ("krylov_m", _I32), ("r_outer_bc", _I32)]


class Physics(ctypes.Structure):
    _fields_ = [(n, _D) for n in ("mu_e", "mu_p", "D_e", "D_p", "k", "V_bottom", "V_top",
                                  "ne_bottom", "ne_top", "np_bottom", "np_top")]

    @classmethod
    def of(cls, d):
        return cls(**{k: float(d[k]) for k, _ in cls._fields_})


class State(ctypes.Structure):
    _fields_ = [("V", _VP), ("ne", _VP), ("np", _VP), ("Se", _VP), ("Sp", _VP),
                ("mue", _VP), ("De", _VP), ("mup", _VP), ("Dp", _VP)]


class Schedule(ctypes.Structure):
    _fields_ = [("dt0", _D), ("growth", _D), ("dt_max", _D), ("steady_tol", _D), ("lin_rtol", _D),
                ("max_steps", _I32), ("max_cycles", _I32), ("coupling", _I32), ("max_newton", _I32),
                ("newton_tol", _D), ("reject_limit", _D)]


class Report(ctypes.Structure):
    _fields_ = [("steps", _I32), ("rejected", _I32), ("vcycles", _I32), ("newton_its", _I32),
                ("last_change", _D), ("final_relres", _D), ("seconds", _D), ("t_end", _D)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# every symbol the header declares, with its ctypes signature
SIGNATURES = {
    "mg_query": (ctypes.c_int, [ctypes.POINTER(GridDesc), ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    "mg_setup": (ctypes.c_int, [ctypes.POINTER(GridDesc), _VP, _I64, _VP, ctypes.POINTER(_VP)]),
    "mg_destroy": (None, [_VP]),
    "sg_assemble": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.POINTER(Physics), ctypes.POINTER(State), _D]),
    "vcycle": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _I32, _PD]),
    "mg_solve": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _D, _I32, ctypes.POINTER(_I32), _PD]),
    "mg_relres": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _PD]),
    "implicit_step": (ctypes.c_int, [_VP, ctypes.POINTER(Physics), ctypes.POINTER(State), _D,
                                     ctypes.POINTER(Schedule), ctypes.POINTER(Report)]),
    "solve_steady": (ctypes.c_int, [_VP, ctypes.POINTER(Physics), ctypes.POINTER(State),
                                    ctypes.POINTER(Schedule), ctypes.POINTER(Report)]),
    "prolong_state": (ctypes.c_int, [_VP, ctypes.POINTER(State), _VP, ctypes.POINTER(State),
                                     ctypes.POINTER(Physics)]),
    "mg_levels": (ctypes.c_int, [_VP]),
    "mg_level_shape": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                                      ctypes.POINTER(_I64)]),
    "mg_copy_coef": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP]),
    "mg_smooth_half": (ctypes.c_int, [_VP, ctypes.c_int, _VP, ctypes.c_int]),
    "mg_residual": (ctypes.c_int, [_VP, ctypes.c_int, _VP, _VP]),
    "mg_time_kernel": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, _I32, _PD]),
    "mg_batch_query": (ctypes.c_int, [ctypes.POINTER(GridDesc), _I32, ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    "mg_batch_setup": (ctypes.c_int, [ctypes.POINTER(GridDesc), _I32, _VP, _I64, _VP, ctypes.POINTER(_VP)]),
    "mg_batch_state": (ctypes.c_int, [_VP, _I32, ctypes.POINTER(State)]),
    "solve_steady_batch": (ctypes.c_int, [_VP, ctypes.POINTER(Physics), ctypes.POINTER(Schedule),
                                          ctypes.POINTER(Report)]),
    "solve_steady_batches": (ctypes.c_int, [ctypes.POINTER(_VP), _I32, ctypes.POINTER(_VP), ctypes.POINTER(Schedule),
                                            ctypes.POINTER(_VP)]),
    "mg_set_tuning": (ctypes.c_int, [_VP, _I32, _I32]),
    "mg_steady_residual": (ctypes.c_int, [_VP, ctypes.POINTER(Physics), ctypes.POINTER(State), _PD]),
    "mg_boundary_flow": (ctypes.c_int, [_VP, ctypes.POINTER(Physics), ctypes.POINTER(State), _PD]),
    "mg_transport_table": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _I32, _VP, _VP]),
    "mg_newton_precond": (ctypes.c_int, [_VP, ctypes.POINTER(Physics), ctypes.POINTER(State), ctypes.c_double,
                                         _VP, _VP]),
    "wn_param_count": (ctypes.c_int, []),
    "wn_scratch_bytes": (ctypes.c_int, [_I32, _I32, _I32, ctypes.POINTER(_I64)]),
    "wn_forward": (ctypes.c_int, [_VP, _VP, _VP, _I32, _I32, _I32, _VP, _I64, _VP]),
    "wn_forward_noalloc": (ctypes.c_int, [_VP, _VP, _VP, _I32, _I32, _I32, _VP]),
    "wn_grad": (ctypes.c_int, [_VP, _VP, _VP, _I32, _I32, _I32, _VP, _PD, _VP, _I64, _VP]),
    "wn_train_step": (ctypes.c_int, [_VP, _VP, _VP, _I32, ctypes.c_float, _VP, _VP, _I32, _I32, _I32, _PD, _VP,
                                     _I64, _VP]),
    "wn_features": (ctypes.c_int, [_VP, ctypes.POINTER(State), _D, _D, _VP, _VP]),
    "wn_targets": (ctypes.c_int, [_VP, ctypes.POINTER(State), ctypes.POINTER(State), _D, _VP, _VP]),
    "wn_apply": (ctypes.c_int, [_VP, ctypes.POINTER(State), _VP, _D, _VP, ctypes.POINTER(Physics),
                                ctypes.POINTER(State)]),
    "mg_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libmgfluid.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmgfluid.so is not built: run python -m paper_0811_4446_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class MGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


def _check(code):
    if code != 0:
        raise MGError(code, lib().mg_last_error().decode())
    return code


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def make_desc(nr, nz, z, R=1.0, d=1.0, coarsest=8, nu1=2, nu2=2, smoother=SMOOTH_ZEBRA, prec=FP64,
              krylov_m=0, r_outer_bc=WALL_ZERO_FLUX):
    z = np.ascontiguousarray(z, dtype=np.float64)
    desc = GridDesc(ABI_VERSION, nr, nz, R, d, z.ctypes.data_as(_PD), coarsest, nu1, nu2, smoother, prec,
                    krylov_m, r_outer_bc)
    desc._z_keep = z
    return desc


def query(desc):
    pitch, ws = _I64(0), _I64(0)
    _check(lib().mg_query(ctypes.byref(desc), ctypes.byref(pitch), ctypes.byref(ws)))
    return pitch.value, ws.value


class Solver:
    """One grid (and its multigrid hierarchy) on one device and stream."""

    def __init__(self, nr, nz, z, R=1.0, d=1.0, coarsest=8, nu1=2, nu2=2,
                 smoother=SMOOTH_ZEBRA, prec=FP64, krylov_m=0, device="cuda:0", stream=None,
                 r_outer_bc=WALL_ZERO_FLUX):
        if not torch.cuda.is_available():
            raise RuntimeError("mgfluid needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.nr, self.nz, self.R, self.d = nr, nz, R, d
        self.z = np.ascontiguousarray(z, dtype=np.float64)
        self.device = torch.device(device)
        self.desc = make_desc(nr, nz, self.z, R, d, coarsest, nu1, nu2, smoother, prec, krylov_m, r_outer_bc)
        self.pitch, self.ws_bytes = query(self.desc)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.workspace = torch.empty(self.ws_bytes // 8 + 64, dtype=torch.float64, device=self.device)
        assert self.workspace.data_ptr() % 256 == 0
        h = _VP()
        _check(lib().mg_setup(ctypes.byref(self.desc), _ptr(self.workspace), self.ws_bytes,
                              ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.ctx = h
        self.nlev = lib().mg_levels(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            lib().mg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- fields ----
    def field(self, fill=0.0):
        return torch.full((self.nr + 1, self.pitch), fill, dtype=torch.float64, device=self.device)

    def upload(self, arr):
        arr = np.asarray(arr, dtype=np.float64)
        assert arr.shape == (self.nr + 1, self.nz + 1), arr.shape
        t = self.field()
        t[:, : self.nz + 1] = torch.from_numpy(np.ascontiguousarray(arr)).to(self.device)
        return t

    def download(self, t):
        torch.cuda.synchronize(self.device)
        return t[:, : self.nz + 1].cpu().numpy().copy()

    def state(self, V, ne, np_, Se=None, Sp=None, mue=None, De=None, mup=None, Dp=None):
        """mg_state over device fields; mue, De, mup, Dp: optional node
        transport fields (None: the physics constants)."""
        opt = lambda t: _ptr(t).value if t is not None else None
        st = State(_ptr(V).value, _ptr(ne).value, _ptr(np_).value, opt(Se), opt(Sp), opt(mue), opt(De), opt(mup),
                   opt(Dp))
        st._keep = (V, ne, np_, Se, Sp, mue, De, mup, Dp)
        return st

    def transport_table(self, V, E_tab, mu_tab, D_tab, mu_out, D_out):
        """mg_transport_table: node mobility and diffusion from tables of
        |E| (device tensors; mu_out and D_out are fields)."""
        n = E_tab.numel()
        assert mu_tab.numel() == n and D_tab.numel() == n
        _check(lib().mg_transport_table(self.ctx, _ptr(V), _ptr(E_tab), _ptr(mu_tab), _ptr(D_tab), n, _ptr(mu_out),
                                        _ptr(D_out)))

    # ---- calls ----
    def assemble(self, eq, phys, state, dt=math.inf):
        _check(lib().sg_assemble(self.ctx, eq, ctypes.byref(phys), ctypes.byref(state), float(dt)))

    def vcycle(self, eq, x, ncycles=1, want_relres=False):
        rr = _D(0.0)
        _check(lib().vcycle(self.ctx, eq, _ptr(x), ncycles, ctypes.byref(rr) if want_relres else None))
        return rr.value if want_relres else None

    def solve(self, eq, x, rtol=1e-10, max_cycles=200, raise_on_noconv=True):
        cyc, rr = _I32(0), _D(0.0)
        code = lib().mg_solve(self.ctx, eq, _ptr(x), rtol, max_cycles, ctypes.byref(cyc), ctypes.byref(rr))
        if code != 0 and (raise_on_noconv or code != -3):
            _check(code)
        return cyc.value, rr.value

    def relres(self, eq, x):
        rr = _D(0.0)
        _check(lib().mg_relres(self.ctx, eq, _ptr(x), ctypes.byref(rr)))
        return rr.value

    def coef(self, eq, level, which):
        nr, nz, pitch = _I32(0), _I32(0), _I64(0)
        _check(lib().mg_level_shape(self.ctx, level, ctypes.byref(nr), ctypes.byref(nz), ctypes.byref(pitch)))
        t = torch.zeros((nr.value + 1, pitch.value), dtype=torch.float64, device=self.device)
        _check(lib().mg_copy_coef(self.ctx, eq, level, which, _ptr(t)))
        torch.cuda.synchronize(self.device)
        return t[:, : nz.value + 1].cpu().numpy().copy()

    def smooth_half(self, eq, x, colour):
        _check(lib().mg_smooth_half(self.ctx, eq, _ptr(x), colour))

    def residual(self, eq, x, r):
        _check(lib().mg_residual(self.ctx, eq, _ptr(x), _ptr(r)))

    def step(self, phys, state, dt, sched, raise_on_noconv=True):
        rep = Report()
        code = lib().implicit_step(self.ctx, ctypes.byref(phys), ctypes.byref(state), float(dt),
                                   ctypes.byref(sched), ctypes.byref(rep))
        if code != 0 and (raise_on_noconv or code != -3):
            _check(code)
        rep.code = code
        return rep

    def tune(self, rows_per_block, fuse_max):
        _check(lib().mg_set_tuning(self.ctx, rows_per_block, fuse_max))

    def steady_residual(self, phys, state):
        r = _D(0.0)
        _check(lib().mg_steady_residual(self.ctx, ctypes.byref(phys), ctypes.byref(state), ctypes.byref(r)))
        return r.value

    def boundary_flow(self, phys, state):
        """mg_boundary_flow: particle flow per radian out through cathode,
        anode and wall, electrons then ions (6 floats)."""
        out = (_D * 6)()
        _check(lib().mg_boundary_flow(self.ctx, ctypes.byref(phys), ctypes.byref(state), out))
        return [out[k] for k in range(6)]

    def field3(self):
        """Three consecutive planes (n_e, n_p, V rows), the layout of
        mg_newton_precond's vectors."""
        return torch.zeros((3, self.nr + 1, self.pitch), dtype=torch.float64, device=self.device)

    def precond(self, phys, state, dt, r, z):
        """z = M r: one block V-cycle at the Newton Jacobian of `state`
        (mg_newton_precond); r and z from field3()."""
        assert r.shape == z.shape == (3, self.nr + 1, self.pitch)
        _check(lib().mg_newton_precond(self.ctx, ctypes.byref(phys), ctypes.byref(state), float(dt), _ptr(r),
                                       _ptr(z)))

    def time_kernel(self, which, eq=0, reps=50):
        ms = _D(0.0)
        _check(lib().mg_time_kernel(self.ctx, which, eq, reps, ctypes.byref(ms)))
        return ms.value

    def steady(self, phys, state, sched):
        rep = Report()
        code = lib().solve_steady(self.ctx, ctypes.byref(phys), ctypes.byref(state), ctypes.byref(sched),
                                  ctypes.byref(rep))
        return code, rep


class Batch:
    """nprob same-shape problems solved together (one size class)."""

    def __init__(self, nr, nz, z, nprob, R=1.0, d=1.0, coarsest=4, nu1=2, nu2=2, prec=FP32_IR, krylov_m=20,
                 device="cuda:0", stream=None, r_outer_bc=WALL_ZERO_FLUX, smoother=SMOOTH_ZEBRA):
        if not torch.cuda.is_available():
            raise RuntimeError("mgfluid needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.nr, self.nz, self.n = nr, nz, nprob
        self.z = np.ascontiguousarray(z, dtype=np.float64)
        self.device = torch.device(device)
        self.desc = make_desc(nr, nz, self.z, R, d, coarsest, nu1, nu2, smoother, prec, krylov_m, r_outer_bc)
        self.pitch, _ = query(self.desc)
        stride, total = _I64(0), _I64(0)
        _check(lib().mg_batch_query(ctypes.byref(self.desc), nprob, ctypes.byref(stride), ctypes.byref(total)))
        self.stride, self.bytes = stride.value, total.value
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.workspace = torch.empty(self.bytes // 8 + 64, dtype=torch.float64, device=self.device)
        h = _VP()
        _check(lib().mg_batch_setup(ctypes.byref(self.desc), nprob, _ptr(self.workspace), self.bytes,
                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.ctx = h
        base = self.workspace.data_ptr()
        self.views = []
        for p in range(nprob):
            st = State()
            _check(lib().mg_batch_state(self.ctx, p, ctypes.byref(st)))
            v = {}
            for name in ("V", "ne", "np", "Se", "Sp"):
                off = (getattr(st, name) - base) // 8
                v[name] = self.workspace[off: off + (nr + 1) * self.pitch].view(nr + 1, self.pitch)
            self.views.append(v)

    def set_problem(self, p, V, ne, np_, S):
        # on the batch's stream, so that its solve sees the values whatever
        # stream is current
        with torch.cuda.stream(self.stream):
            for name, arr in (("V", V), ("ne", ne), ("np", np_), ("Se", S), ("Sp", S)):
                t = self.views[p][name]
                t[:, : self.nz + 1] = torch.from_numpy(np.ascontiguousarray(arr, dtype=np.float64)).to(self.device)

    def get(self, p, name):
        torch.cuda.synchronize(self.device)
        return self.views[p][name][:, : self.nz + 1].cpu().numpy().copy()

    def tune(self, rows_per_block, fuse_max):
        _check(lib().mg_set_tuning(self.ctx, rows_per_block, fuse_max))

    def steady(self, phys_list, sched):
        P = (Physics * self.n)(*phys_list)
        R = (Report * self.n)()
        code = lib().solve_steady_batch(self.ctx, P, ctypes.byref(sched), R)
        return code, [R[i].as_dict() for i in range(self.n)]

    def close(self):
        if getattr(self, "ctx", None):
            lib().mg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batches(batches, phys_lists, sched):
    """Steady solves of several batches at once (solve_steady_batches): the
    library drives each batch from a host thread of its own, so batches set
    up on different streams overlap on the GPU.  Returns (code, per-batch
    report lists)."""
    n = len(batches)
    ctxs = (_VP * n)(*[b.ctx.value for b in batches])
    Ps = [(Physics * b.n)(*pl) for b, pl in zip(batches, phys_lists)]
    Rs = [(Report * b.n)() for b in batches]
    parr = (_VP * n)(*[ctypes.cast(P, _VP).value for P in Ps])
    rarr = (_VP * n)(*[ctypes.cast(R, _VP).value for R in Rs])
    code = lib().solve_steady_batches(ctxs, n, parr, ctypes.byref(sched), rarr)
    return code, [[R[i].as_dict() for i in range(b.n)] for b, R in zip(batches, Rs)]


class Net:
    """The warm-start network's parameters, Adam moments and scratch on one
    device; every call runs the library's kernels."""

    def __init__(self, params, device="cuda:0", stream=None):
        self.device = torch.device(device)
        self.P = lib().wn_param_count()
        p = torch.as_tensor(np.asarray(params, dtype=np.float32))
        assert p.numel() == self.P, (p.numel(), self.P)
        self.params = p.to(self.device).contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._scratch = {}

    def scratch(self, B, H, W):
        key = (B, H, W)
        if key not in self._scratch:
            n = _I64(0)
            _check(lib().wn_scratch_bytes(B, H, W, ctypes.byref(n)))
            self._scratch[key] = (torch.empty(n.value // 8 + 64, dtype=torch.float64, device=self.device), n.value)
        return self._scratch[key]

    def forward(self, x):
        B, C, H, W = x.shape
        out = torch.empty((B, 3, H, W), dtype=torch.float32, device=self.device)
        s, n = self.scratch(B, H, W)
        _check(lib().wn_forward(_ptr(self.params), _ptr(x), _ptr(out), B, H, W, _ptr(s), n,
                                ctypes.c_void_p(self.stream.cuda_stream)))
        return out

    def forward_noalloc(self, x, out):
        """wn_forward_noalloc: the forward pass with the library's static
        scratch array (no scratch tensor; out is caller-allocated)."""
        B, C, H, W = x.shape
        assert out.shape == (B, 3, H, W) and out.dtype == torch.float32
        _check(lib().wn_forward_noalloc(_ptr(self.params), _ptr(x), _ptr(out), B, H, W,
                                        ctypes.c_void_p(self.stream.cuda_stream)))
        return out

    def grad(self, x, target):
        B, C, H, W = x.shape
        g = torch.empty(self.P, dtype=torch.float32, device=self.device)
        loss = _D(0.0)
        s, n = self.scratch(B, H, W)
        _check(lib().wn_grad(_ptr(self.params), _ptr(x), _ptr(target), B, H, W, _ptr(g), ctypes.byref(loss),
                             _ptr(s), n, ctypes.c_void_p(self.stream.cuda_stream)))
        return loss.value, g

    def train_step(self, x, target, lr=1e-3):
        B, C, H, W = x.shape
        self.t += 1
        loss = _D(0.0)
        s, n = self.scratch(B, H, W)
        _check(lib().wn_train_step(_ptr(self.params), _ptr(self.m), _ptr(self.v), self.t, lr, _ptr(x),
                                   _ptr(target), B, H, W, ctypes.byref(loss), _ptr(s), n,
                                   ctypes.c_void_p(self.stream.cuda_stream)))
        return loss.value


def features(sol, up_state, vtop, ratio):
    """Input planes [7, H, W] of the prolonged coarse state on `sol`'s grid,
    and the density scale (device double)."""
    H, W = sol.nr + 1, sol.nz + 1
    out = torch.empty((7, H, W), dtype=torch.float32, device=sol.device)
    ns = torch.zeros(1, dtype=torch.float64, device=sol.device)
    _check(lib().wn_features(sol.ctx, ctypes.byref(up_state), float(vtop), float(ratio), _ptr(out), _ptr(ns)))
    return out, ns


def targets(sol, up_state, steady_state, vtop, ns):
    out = torch.empty((3, sol.nr + 1, sol.nz + 1), dtype=torch.float32, device=sol.device)
    _check(lib().wn_targets(sol.ctx, ctypes.byref(up_state), ctypes.byref(steady_state), float(vtop), _ptr(ns),
                            _ptr(out)))
    return out


def apply_prediction(sol, up_state, pred, vtop, ns, phys, dst_state):
    _check(lib().wn_apply(sol.ctx, ctypes.byref(up_state), _ptr(pred), float(vtop), _ptr(ns),
                          ctypes.byref(phys), ctypes.byref(dst_state)))


def schedule(dt0=1e-4, growth=1.5, dt_max=0.1, steady_tol=1e-8, lin_rtol=1e-10, max_steps=100000,
             max_cycles=200, coupling=DECOUPLED, max_newton=10, newton_tol=1e-6, reject_limit=1e30):
    return Schedule(dt0, growth, dt_max, steady_tol, lin_rtol, max_steps, max_cycles, coupling,
                    max_newton, newton_tol, reject_limit)


def prolong_state(coarse, src, fine, dst, phys):
    _check(lib().prolong_state(coarse.ctx, ctypes.byref(src), fine.ctx, ctypes.byref(dst), ctypes.byref(phys)))
