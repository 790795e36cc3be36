"""Plain FP64 CPU oracle (test infrastructure only).

This package checks the HIP library; it is never part of the product path.
Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` import it.  It shares no code with ``paper_0811_4446_amd``.

Arrays are dense numpy float64 arrays of shape (nr+1, nz+1), C order,
index [i, j] with i the radial node (r_i = i*R/nr) and j the axial node.
Rows j = 0 and j = nz are the electrodes (Dirichlet).

The arithmetic lives in ``mg_oracle.c`` (plain C, FP64, no blocking or
fusion); this module only marshals numpy arrays through ctypes, and adds the
coupled Newton step (``newton.py``), which uses SciPy's sparse LU as its
linear solver.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mg_oracle.c")
_LIB = os.path.join(_HERE, "libmgoracle.so")

SMOOTH_RB = 0
SMOOTH_ZEBRA = 1


def build(force=False):
    """Compile mg_oracle.c into libmgoracle.so with gcc -O2 (FP64, no FMA)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                           "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None
_D = ctypes.c_double
_I = ctypes.c_int
_P = ctypes.POINTER(ctypes.c_double)


class Phys(ctypes.Structure):
    """Physical parameters (mirrors the fields of the paper's model, Eqs. 1-6)."""
    _fields_ = [(n, ctypes.c_double) for n in (
        "mu_e", "mu_p", "D_e", "D_p", "k", "V_bottom", "V_top",
        "ne_bottom", "ne_top", "np_bottom", "np_top")]


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.or_bernoulli_F.restype = _D
        L.or_bernoulli_F.argtypes = [_D]
        L.or_bernoulli_G.restype = _D
        L.or_bernoulli_G.argtypes = [_D]
        L.or_volume.restype = _D
        L.or_volume.argtypes = [_I, _I, _D, _P, _I, _I]
        L.or_poisson_assemble.argtypes = [_I, _I, _D, _P, _D, _P, _P] + [_P] * 6
        L.or_poisson_assemble_w.argtypes = [_I, _I, _D, _P, _D, _P, _P, _I, _P] + [_P] * 6
        L.or_sg_assemble.argtypes = [_I, _I, _D, _P, _I, _D, _D, _D, _P, _P, _P] + [_P] * 6
        L.or_sg_assemble_w.argtypes = [_I, _I, _D, _P, _I, _D, _D, _D, _I, _P, _P, _P] + [_P] * 6
        L.or_sg_assemble_t.argtypes = [_I, _I, _D, _P, _I, _D, _D, _D, _I, _P, _P, _P, _P, _P] + [_P] * 6
        L.or_apply.argtypes = [_I, _I] + [_P] * 7
        L.or_residual.argtypes = [_I, _I] + [_P] * 8
        L.or_relres.restype = _D
        L.or_relres.argtypes = [_I, _I, _D, _P] + [_P] * 7
        L.or_rbgs.argtypes = [_I, _I] + [_P] * 7 + [_I]
        L.or_zline.argtypes = [_I, _I] + [_P] * 7 + [_I, _P]
        L.or_prolong_add.argtypes = [_I, _I, _P, _P, _P]
        L.or_restrict.argtypes = [_I, _I, _P, _P, _P]
        L.or_direct_solve.restype = _I
        L.or_direct_solve.argtypes = [_I, _I] + [_P] * 7
        L.or_levels.restype = _I
        L.or_levels.argtypes = [_I, _I, _I]
        L.or_mg_create.restype = ctypes.c_void_p
        L.or_mg_create.argtypes = [_I, _I, _D, _P, _I, _I, _I, _I]
        L.or_mg_create_w.restype = ctypes.c_void_p
        L.or_mg_create_w.argtypes = [_I, _I, _D, _P, _I, _I, _I, _I, _I]
        L.or_mg_assemble_poisson_w.argtypes = [ctypes.c_void_p, _D, _P, _P, _P]
        L.or_mg_destroy.argtypes = [ctypes.c_void_p]
        L.or_mg_nlev.restype = _I
        L.or_mg_nlev.argtypes = [ctypes.c_void_p]
        L.or_mg_get.argtypes = [ctypes.c_void_p, _I, _I, _P]
        L.or_mg_assemble_poisson.argtypes = [ctypes.c_void_p, _D, _P, _P]
        L.or_mg_assemble_sg.argtypes = [ctypes.c_void_p, _I, _D, _D, _D, _P, _P, _P]
        L.or_mg_assemble_sg_t.argtypes = [ctypes.c_void_p, _I, _D, _D, _D, _P, _P, _P, _P, _P]
        L.or_mg_vcycle.restype = _I
        L.or_mg_vcycle.argtypes = [ctypes.c_void_p, _P]
        L.or_mg_relres.restype = _D
        L.or_mg_relres.argtypes = [ctypes.c_void_p, _P]
        L.or_mg_solve.restype = _I
        L.or_mg_solve.argtypes = [ctypes.c_void_p, _P, _D, _I,
                                  ctypes.POINTER(_I), ctypes.POINTER(_D)]
        L.or_step_decoupled_w.restype = _I
        L.or_step_decoupled_w.argtypes = [_I, _I, _D, _P, ctypes.POINTER(Phys),
                                          _P, _P, _P, _P, _P, _D,
                                          _I, _I, _I, _I, _D, _I, _I,
                                          ctypes.POINTER(_I), ctypes.POINTER(_D)]
        L.or_step_decoupled.restype = _I
        L.or_step_decoupled.argtypes = [_I, _I, _D, _P, ctypes.POINTER(Phys),
                                        _P, _P, _P, _P, _P, _D,
                                        _I, _I, _I, _I, _D, _I,
                                        ctypes.POINTER(_I), ctypes.POINTER(_D)]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous, "float64 C-contiguous array expected"
    return a.ctypes.data_as(_P)


def _field(nr, nz):
    return np.zeros((nr + 1, nz + 1))


def bernoulli_F(x):
    return lib().or_bernoulli_F(float(x))


def bernoulli_G(x):
    return lib().or_bernoulli_G(float(x))


def volumes(nr, nz, R, z):
    """Control volumes vol[i, j] (j = 1..nz-1; electrode rows 0)."""
    z = np.ascontiguousarray(z, dtype=np.float64)
    v = _field(nr, nz)
    for i in range(nr + 1):
        for j in range(1, nz):
            v[i, j] = lib().or_volume(nr, nz, R, _p(z), i, j)
    return v


def poisson_assemble(nr, nz, R, z, k, ne=None, np_=None, wall=0, Vwall=None):
    """Coefficients (a, b, c, d, e, f) of Eqs. (12)-(13) in FV form.  wall=1:
    Dirichlet wall at r = R (identity rows i = nr, right-hand side Vwall)."""
    z = np.ascontiguousarray(z, dtype=np.float64)
    out = [_field(nr, nz) for _ in range(6)]
    if Vwall is not None:
        Vwall = np.ascontiguousarray(Vwall, dtype=np.float64)
    lib().or_poisson_assemble_w(nr, nz, R, _p(z), k, _p(ne), _p(np_), int(wall), _p(Vwall),
                                *[_p(o) for o in out])
    return out


def sg_assemble(nr, nz, R, z, s, mu, D, dt_inv, V, nk=None, S=None, wall=0, mun=None, Dn=None):
    """Coefficients (a, b, c, d, e, f) of Eqs. (7)-(11) in FV form.  wall=1:
    Dirichlet wall at r = R with density 0 (identity rows i = nr).  mun, Dn:
    node values of the mobility and diffusion coefficient (faces: mean of
    the two nodes) instead of the constants mu, D."""
    z = np.ascontiguousarray(z, dtype=np.float64)
    out = [_field(nr, nz) for _ in range(6)]
    lib().or_sg_assemble_t(nr, nz, R, _p(z), int(s), mu, D, dt_inv, int(wall), _p(mun), _p(Dn), _p(V), _p(nk),
                           _p(S), *[_p(o) for o in out])
    return out


def wall_values(z, V_bottom, V_top):
    """Wall potential of the paper's experiment (Sec. 3): linear in z between
    the electrode values."""
    z = np.asarray(z, dtype=np.float64)
    return V_bottom + (V_top - V_bottom) * ((z - z[0]) / (z[-1] - z[0]))


def apply(coef, x):
    nr, nz = x.shape[0] - 1, x.shape[1] - 1
    y = np.zeros_like(x)
    lib().or_apply(nr, nz, *[_p(c) for c in coef[:5]], _p(x), _p(y))
    return y


def residual(coef, x):
    nr, nz = x.shape[0] - 1, x.shape[1] - 1
    r = np.zeros_like(x)
    lib().or_residual(nr, nz, *[_p(c) for c in coef[:6]], _p(x), _p(r))
    return r


def relres(R, z, coef, x):
    nr, nz = x.shape[0] - 1, x.shape[1] - 1
    z = np.ascontiguousarray(z, dtype=np.float64)
    return lib().or_relres(nr, nz, R, _p(z), *[_p(c) for c in coef[:6]], _p(x))


def rbgs(coef, x, colour):
    nr, nz = x.shape[0] - 1, x.shape[1] - 1
    lib().or_rbgs(nr, nz, *[_p(c) for c in coef[:6]], _p(x), int(colour))


def zline(coef, x, parity):
    nr, nz = x.shape[0] - 1, x.shape[1] - 1
    w = np.zeros(2 * (nz + 1))
    lib().or_zline(nr, nz, *[_p(c) for c in coef[:6]], _p(x), int(parity), _p(w))


def prolong_add(zf, ec, xf):
    nrf, nzf = xf.shape[0] - 1, xf.shape[1] - 1
    zf = np.ascontiguousarray(zf, dtype=np.float64)
    lib().or_prolong_add(nrf, nzf, _p(zf), _p(ec), _p(xf))


def restrict(zf, rf):
    nrf, nzf = rf.shape[0] - 1, rf.shape[1] - 1
    zf = np.ascontiguousarray(zf, dtype=np.float64)
    fc = _field(nrf // 2, nzf // 2)
    lib().or_restrict(nrf, nzf, _p(zf), _p(rf), _p(fc))
    return fc


def direct_solve(coef, x):
    """Dense Gaussian elimination of the whole system; x's electrode rows are inputs."""
    nr, nz = x.shape[0] - 1, x.shape[1] - 1
    st = lib().or_direct_solve(nr, nz, *[_p(c) for c in coef[:6]], _p(x))
    if st != 0:
        raise ArithmeticError("singular system")


def levels(nr, nz, coarsest=8):
    return lib().or_levels(nr, nz, coarsest)


class MG:
    """Multigrid hierarchy (V(nu1, nu2) cycle) of the oracle."""

    def __init__(self, nr, nz, R, z, coarsest=8, smoother=SMOOTH_ZEBRA, nu1=2, nu2=2, wall=0):
        self.nr, self.nz, self.R = nr, nz, R
        self.z = np.ascontiguousarray(z, dtype=np.float64)
        self.h = lib().or_mg_create_w(nr, nz, R, _p(self.z), coarsest, smoother, nu1, nu2, int(wall))
        if not self.h:
            raise ValueError("grid not coarsenable to %d" % coarsest)
        self.nlev = lib().or_mg_nlev(self.h)

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.or_mg_destroy(h)
            self.h = None

    def assemble_poisson(self, k, ne, np_, Vwall=None):
        if Vwall is not None:
            Vwall = np.ascontiguousarray(Vwall, dtype=np.float64)
        lib().or_mg_assemble_poisson_w(self.h, k, _p(ne), _p(np_), _p(Vwall))

    def assemble_sg(self, s, mu, D, dt_inv, V, nk, S, mun=None, Dn=None):
        lib().or_mg_assemble_sg_t(self.h, int(s), mu, D, dt_inv, _p(V), _p(nk), _p(S), _p(mun), _p(Dn))

    def coef(self, level=0):
        nr, nz = self.nr >> level, self.nz >> level
        out = []
        for w in range(6):
            a = _field(nr, nz)
            lib().or_mg_get(self.h, level, w, _p(a))
            out.append(a)
        return out

    def vcycle(self, x):
        st = lib().or_mg_vcycle(self.h, _p(x))
        if st != 0:
            raise ArithmeticError("coarse solve failed")

    def relres(self, x):
        return lib().or_mg_relres(self.h, _p(x))

    def solve(self, x, rtol=1e-10, max_cycles=200):
        cyc = _I(0)
        rr = _D(0.0)
        st = lib().or_mg_solve(self.h, _p(x), rtol, max_cycles, ctypes.byref(cyc), ctypes.byref(rr))
        return st, cyc.value, rr.value


def step_decoupled(R, z, phys, V, ne, np_, Se, Sp, dt, coarsest=8, smoother=SMOOTH_RB,
                   nu1=2, nu2=2, rtol=1e-10, max_cycles=500, wall=0):
    """One backward-Euler step (Eq. 7): Poisson with n^k, then SG electrons and
    ions with the new potential.  Updates V, ne, np_ in place.  wall=1:
    Dirichlet wall at r = R (potential linear in z, densities 0)."""
    nr, nz = V.shape[0] - 1, V.shape[1] - 1
    z = np.ascontiguousarray(z, dtype=np.float64)
    cyc = (_I * 3)()
    rr = (_D * 3)()
    st = lib().or_step_decoupled_w(nr, nz, R, _p(z), ctypes.byref(phys), _p(V), _p(ne), _p(np_),
                                   _p(Se), _p(Sp), dt, coarsest, smoother, nu1, nu2, rtol,
                                   max_cycles, int(wall), cyc, rr)
    return st, list(cyc), list(rr)
