"""Coupled backward-Euler step by Newton-Raphson (Sec. 2, Eq. 14) and the
steady driver (Sec. 2, time-step rule and multilevel prolongation).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Unknowns per node u = (n_e, n_p, V) on i = 0..nr, j = 1..nz-1.  The
nonlinear residual in finite-volume form is
    F_e = A_e(V) n_e - vol (S_e + n_e^k / dt)          (Eqs. 7-11, s = -1)
    F_p = A_p(V) n_p - vol (S_p + n_p^k / dt)          (s = +1)
    F_V = A_P V - vol k (n_p - n_e)                    (Eqs. 12-13)
where A_e, A_p are the SG operators assembled with the current V and A_P
is the Poisson operator (all from mg_oracle.c).  The Jacobian is the
3x3-block five-point matrix of Eq. (14); each linear system J du = -F is
solved exactly with SciPy's sparse LU.
"""
import ctypes

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import _p, lib, poisson_assemble, sg_assemble, apply, volumes, wall_values


def _sg_dV(nr, nz, R, z, s, mu, D, V, n, wall=0, mun=None, Dn=None):
    L = lib()
    if not hasattr(L, "_dv_ready"):
        P = ctypes.POINTER(ctypes.c_double)
        L.or_sg_dV_t.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, P, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_int, P, P, P, P] + [P] * 5
        L.or_bernoulli_dF.restype = ctypes.c_double
        L.or_bernoulli_dF.argtypes = [ctypes.c_double]
        L._dv_ready = True
    out = [np.zeros((nr + 1, nz + 1)) for _ in range(5)]
    L.or_sg_dV_t(nr, nz, R, _p(z), int(s), mu, D, int(wall), _p(mun), _p(Dn), _p(V), _p(n),
                 *[_p(o) for o in out])
    return out


def bernoulli_dF(x):
    _sg_dV(2, 2, 1.0, np.array([0.0, 0.5, 1.0]), 1, 1.0, 1.0, np.zeros((3, 3)), np.zeros((3, 3)))
    return lib().or_bernoulli_dF(float(x))


class Coupled:
    """Residual and Jacobian of the coupled BE system on one grid.  wall=1:
    the paper's Dirichlet wall at r = R (Sec. 3): potential linear in z
    between the electrode values, densities 0; the wall nodes' equations are
    u = u_wall (identity rows)."""

    def __init__(self, nr, nz, R, z, phys, wall=0, transport=None):
        self.nr, self.nz, self.R = nr, nz, R
        self.z = np.ascontiguousarray(z, dtype=np.float64)
        self.ph = dict(phys)
        self.wall = int(wall)
        # node values of mu_e, D_e, mu_p, D_p (Sec. 2: field-dependent transport
        # supplied by tables); None: the constants of phys
        self.tr = None
        if transport is not None:
            self.tr = {k: np.ascontiguousarray(transport[k], dtype=np.float64) for k in ("mue", "De", "mup", "Dp")}
        self.vol = volumes(nr, nz, R, self.z)
        self.P = poisson_assemble(nr, nz, R, self.z, 0.0, wall=self.wall)
        self.interior = np.ones((nr + 1, nz + 1))  # 0 on the wall rows
        if self.wall:
            self.interior[nr, :] = 0.0
            self.Vwall = wall_values(self.z, self.ph["V_bottom"], self.ph["V_top"])
        m = nz - 1
        self.m = m
        self.nun = (nr + 1) * m
        ii, jj = np.meshgrid(np.arange(nr + 1), np.arange(1, nz), indexing="ij")
        self.ii, self.jj = ii.ravel(), jj.ravel()
        self.node = (ii * m + (jj - 1)).ravel()

    def electrodes(self, V, ne, np_):
        ph = self.ph
        V[:, 0], V[:, -1] = ph["V_bottom"], ph["V_top"]
        ne[:, 0], ne[:, -1] = ph["ne_bottom"], ph["ne_top"]
        np_[:, 0], np_[:, -1] = ph["np_bottom"], ph["np_top"]
        if self.wall:
            V[-1, :], ne[-1, :], np_[-1, :] = self.Vwall, 0.0, 0.0

    def residual(self, V, ne, np_, nek, npk, Se, Sp, dt_inv):
        ph, nr, nz, R, z = self.ph, self.nr, self.nz, self.R, self.z
        tr = self.tr or {}
        Ae = sg_assemble(nr, nz, R, z, -1, ph["mu_e"], ph["D_e"], dt_inv, V, nek, Se, wall=self.wall,
                         mun=tr.get("mue"), Dn=tr.get("De"))
        Ap = sg_assemble(nr, nz, R, z, +1, ph["mu_p"], ph["D_p"], dt_inv, V, npk, Sp, wall=self.wall,
                         mun=tr.get("mup"), Dn=tr.get("Dp"))
        Fe = apply(Ae, ne) - Ae[5]
        Fp = apply(Ap, np_) - Ap[5]
        rhsV = self.interior * self.vol * ph["k"] * (np_ - ne)
        if self.wall:
            rhsV[-1, 1:-1] = self.Vwall[1:-1]
        FV = apply(self.P, V) - rhsV
        return (Fe, Fp, FV), (Ae, Ap)

    def pack(self, Fe, Fp, FV):
        out = np.empty(3 * self.nun)
        out[0::3] = Fe[:, 1:-1].ravel()
        out[1::3] = Fp[:, 1:-1].ravel()
        out[2::3] = FV[:, 1:-1].ravel()
        return out

    def unpack(self, vec):
        nr, nz = self.nr, self.nz
        f = [np.zeros((nr + 1, nz + 1)) for _ in range(3)]
        for k in range(3):
            f[k][:, 1:-1] = vec[k::3].reshape(nr + 1, nz - 1)
        return f

    def jacobian(self, V, ne, np_, Ae, Ap):
        """Sparse 3x3-block five-point Jacobian (Eq. 14)."""
        ph, nr, nz, R, z = self.ph, self.nr, self.nz, self.R, self.z
        tr = self.tr or {}
        eV = _sg_dV(nr, nz, R, z, -1, ph["mu_e"], ph["D_e"], V, ne, self.wall, tr.get("mue"), tr.get("De"))
        pV = _sg_dV(nr, nz, R, z, +1, ph["mu_p"], ph["D_p"], V, np_, self.wall, tr.get("mup"), tr.get("Dp"))
        rows, cols, vals = [], [], []
        i, j, node, m = self.ii, self.jj, self.node, self.m
        offs = {0: (-1, 0), 1: (0, 0), 2: (1, 0), 3: (0, -1), 4: (0, 1)}  # a, b, c, d, e
        for w, (di, dj) in offs.items():
            ni, nj = i + di, j + dj
            ok = (ni >= 0) & (ni <= nr) & (nj >= 1) & (nj <= nz - 1)
            src = node[ok]
            dst = (ni * m + (nj - 1))[ok]
            sel = (i[ok], j[ok])
            for (rf, cf, arr) in ((0, 0, Ae[w]), (0, 2, eV[w]), (1, 1, Ap[w]), (1, 2, pV[w]),
                                  (2, 2, self.P[w])):
                rows.append(3 * src + rf)
                cols.append(3 * dst + cf)
                vals.append(arr[sel])
        kv = self.interior[i, j] * self.vol[i, j] * ph["k"]
        rows += [3 * node + 2, 3 * node + 2]
        cols += [3 * node + 0, 3 * node + 1]
        vals += [kv, -kv]
        n = 3 * self.nun
        return sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(n, n))


def newton_step(cp, V, ne, np_, Se, Sp, dt, max_newton=10, tol=1e-6, history=None):
    """One BE step by Newton (Sec. 2): iterate J du = -F from u^k until the
    relative l1 norm of the correction of every field is < tol.  Updates
    V, ne, np_ in place and returns (converged, iterations)."""
    dt_inv = 0.0 if not np.isfinite(dt) else 1.0 / dt
    cp.electrodes(V, ne, np_)
    nek, npk = ne.copy(), np_.copy()
    for it in range(1, max_newton + 1):
        (Fe, Fp, FV), (Ae, Ap) = cp.residual(V, ne, np_, nek, npk, Se, Sp, dt_inv)
        J = cp.jacobian(V, ne, np_, Ae, Ap)
        du = spla.splu(J).solve(-cp.pack(Fe, Fp, FV))
        dne, dnp, dV = cp.unpack(du)
        ne += dne
        np_ += dnp
        V += dV
        un = (slice(None), slice(1, -1))  # unknown nodes only (electrode rows are fixed)
        rel = [np.abs(dne[un]).sum() / max(np.abs(ne[un]).sum(), 1e-300),
               np.abs(dnp[un]).sum() / max(np.abs(np_[un]).sum(), 1e-300),
               np.abs(dV[un]).sum() / max(np.abs(V[un]).sum(), 1e-300)]
        if history is not None:
            history.append(rel)
        if not np.all(np.isfinite(du)):
            return False, it
        if max(rel) < tol:
            return True, it
    return False, max_newton


def steady(cp, V, ne, np_, Se, Sp, dt0=1e-4, growth=1.5, dt_max=0.1, tol=1e-8,
           max_steps=100000, newton_tol=1e-6, max_newton=10, dts=None, log=None, attempts=None):
    """Steps with dt <- min(growth*dt, dt_max) until max over species of
    ||n^{k+1}-n^k||_2/||n^{k+1}||_2 < tol.  A step whose Newton iteration
    does not converge, or that ends with a density below -1e-10 times its
    mean magnitude, is rejected: it is retried with the last accepted step
    (Sec. 2), or with half the step if it already was that long.  If `dts`
    is given, that sequence of accepted steps is replayed instead.  If
    `attempts` is a list, every tried step is appended as (dt, accepted).
    Returns (steps, rejected, dt_list)."""
    dt = dt0
    dt_acc = 0.0
    acc, rej, seq = 0, 0, []
    while acc < max_steps:
        if dts is not None:
            if acc >= len(dts):
                break
            dt = dts[acc]
        s0 = (V.copy(), ne.copy(), np_.copy())
        ok, its = newton_step(cp, V, ne, np_, Se, Sp, dt, max_newton, newton_tol)
        if ok:
            un = (slice(None), slice(1, -1))
            ok = (ne[un].min() >= -1e-10 * np.abs(ne[un]).mean()
                  and np_[un].min() >= -1e-10 * np.abs(np_[un]).mean())
        if attempts is not None:
            attempts.append((dt, bool(ok)))
        if not ok:
            V[:], ne[:], np_[:] = s0
            rej += 1
            dt = dt_acc if (dt_acc > 0 and dt > dt_acc) else 0.5 * dt
            if rej > 200:
                raise RuntimeError("too many rejected steps")
            continue
        acc += 1
        seq.append(dt)
        ch = max(np.linalg.norm((ne - s0[1])[:, 1:-1]) / np.linalg.norm(ne[:, 1:-1]),
                 np.linalg.norm((np_ - s0[2])[:, 1:-1]) / np.linalg.norm(np_[:, 1:-1]))
        if log is not None:
            log.append((acc, dt, its, ch))
        dt_acc = dt
        if dts is None and ch < tol:
            break
        dt = min(growth * dt, dt_max)
    return acc, rej, seq


def boundary_flow(R, z, s, mu, D, V, n, wall=0, mun=None, Dn=None):
    """Particle flow per radian out of the domain (Sec. 3's observable is the
    ion current to the cathode): the SG face fluxes of Eqs. (8)-(9) through
    the cathode face z_{1/2}, the anode face z_{nz-1/2} and, with the
    Dirichlet wall, the wall face r_{nr-1/2}, times the faces' areas, summed
    over the unknown cells.  Returns (cathode, anode, wall)."""
    from . import bernoulli_F
    nr, nz = V.shape[0] - 1, V.shape[1] - 1
    dr = R / nr

    def face(a, b):  # (D, q) of the face between nodes a and b
        if mun is None:
            return D, -s * mu / D
        Df = 0.5 * (Dn[a] + Dn[b])
        return Df, -s * 0.5 * (mun[a] + mun[b]) / Df

    imax = nr - 1 if wall else nr
    cath = anode = wflow = 0.0
    for i in range(imax + 1):
        w = dr * dr / 8 if i == 0 else (0.5 * dr * (R - 0.25 * dr) if i == nr else i * dr * dr)
        Df, q = face((i, 0), (i, 1))
        al = q * (V[i, 1] - V[i, 0])
        cath -= w * Df / (z[1] - z[0]) * (n[i, 0] * bernoulli_F(-al) - n[i, 1] * bernoulli_F(al))
        Df, q = face((i, nz - 1), (i, nz))
        al = q * (V[i, nz] - V[i, nz - 1])
        anode += w * Df / (z[nz] - z[nz - 1]) * (n[i, nz - 1] * bernoulli_F(-al) - n[i, nz] * bernoulli_F(al))
    if wall:
        for j in range(1, nz):
            area = (nr - 0.5) * dr * 0.5 * (z[j + 1] - z[j - 1])
            Df, q = face((nr - 1, j), (nr, j))
            al = q * (V[nr, j] - V[nr - 1, j])
            wflow += area * Df / dr * (n[nr - 1, j] * bernoulli_F(-al) - n[nr, j] * bernoulli_F(al))
    return cath, anode, wflow


def field_strength(R, z, V):
    """|E| = |grad V| at every node (Eq. 6): central differences, one-sided at
    the electrodes (z) and at r = R, radial component 0 on the axis."""
    nr, nz = V.shape[0] - 1, V.shape[1] - 1
    dr = R / nr
    E = np.zeros_like(V)
    for i in range(nr + 1):
        for j in range(nz + 1):
            if i == 0:
                er = 0.0
            elif i == nr:
                er = (V[i, j] - V[i - 1, j]) / dr
            else:
                er = (V[i + 1, j] - V[i - 1, j]) / (2.0 * dr)
            if j == 0:
                ez = (V[i, 1] - V[i, 0]) / (z[1] - z[0])
            elif j == nz:
                ez = (V[i, nz] - V[i, nz - 1]) / (z[nz] - z[nz - 1])
            else:
                ez = (V[i, j + 1] - V[i, j - 1]) / (z[j + 1] - z[j - 1])
            E[i, j] = np.sqrt(er * er + ez * ez)
    return E


def transport_from_table(R, z, V, Et, mut, Dt):
    """Node mobility and diffusion coefficient from tables of the field
    strength (Sec. 2: mu(E), D(E) from lookup tables): linear interpolation
    between the bracketing entries, the end values outside the table."""
    E = field_strength(R, z, V)
    return np.interp(E, Et, mut), np.interp(E, Et, Dt)


def prolong_state(zf, Vc, nec, npc, phys, wall=0):
    """Multilevel prolongation (Sec. 2, last paragraphs): the state of the
    grid one level coarser, interpolated onto the twice finer grid with the
    multigrid prolongation (bilinear, z-distance weights) on the unknown
    rows, and the electrode rows (with wall=1 also the wall) set to their
    boundary values."""
    from . import prolong_add
    nrc, nzc = Vc.shape[0] - 1, Vc.shape[1] - 1
    out = []
    for c, lo, hi in ((Vc, "V_bottom", "V_top"), (nec, "ne_bottom", "ne_top"), (npc, "np_bottom", "np_top")):
        f = np.zeros((2 * nrc + 1, 2 * nzc + 1))
        prolong_add(zf, np.ascontiguousarray(c, dtype=np.float64), f)
        f[:, 0], f[:, -1] = phys[lo], phys[hi]
        out.append(f)
    if wall:
        out[0][-1, :] = wall_values(zf, phys["V_bottom"], phys["V_top"])
        out[1][-1, :] = out[2][-1, :] = 0.0
    return out


def chain(R, z_of, phys, N0, N1, V, ne, np_, S_of, wall=0, **steady_kw):
    """Multilevel prolongation chain (Sec. 2): steady run on the N0 grid from
    (V, ne, np_), then for each finer grid up to N1 the steady run from the
    prolonged steady state of the grid before.  z_of(N) gives the axial
    nodes, S_of(N, z) the source.  Returns the finest steady state and the
    accepted step count of every stage."""
    N = N0
    stages = []
    while True:
        z = z_of(N)
        cp = Coupled(N, N, R, z, phys, wall=wall)
        S = S_of(N, z)
        acc, rej, _ = steady(cp, V, ne, np_, S, S, **steady_kw)
        stages.append((N, acc, rej))
        if N == N1:
            return (V, ne, np_), stages
        V, ne, np_ = prolong_state(z_of(2 * N), V, ne, np_, phys, wall=wall)
        N *= 2


# ---------------------------------------------------------------------------
# Block multigrid for the Newton system (Sec. 2: Eq. (14) solved by the
# multigrid method).  Hierarchy: the grid halved in r and z until the
# oracle's level rule stops (coarse z nodes are every second fine node),
# the Jacobian rediscretised on every level at the state injected there;
# smoother: collective red-black Gauss-Seidel (the three unknowns of a node
# solved together; nodes with (i + j) even first), or block zebra z-line
# Gauss-Seidel (all unknowns of an axial line i solved together, the 3x3-
# block tridiagonal system of Eq. (14) along z; even lines first); the
# restriction: the transpose of the bilinear prolongation, field by field;
# coarsest level solved exactly.
# ---------------------------------------------------------------------------
def block_hierarchy(nr, nz, R, z, phys, V, ne, np_, dt, coarsest=8, wall=0, transport=None):
    """Per level: the Coupled system, its Jacobian (CSR) for a BE step of
    size dt (inf: steady), the unknown indices of both colours."""
    from . import levels as _nlev
    nlev = _nlev(nr, nz, coarsest)
    dt_inv = 0.0 if not np.isfinite(dt) else 1.0 / dt
    out = []
    z = np.ascontiguousarray(z, dtype=np.float64)
    V, ne, np_ = (np.ascontiguousarray(a, dtype=np.float64) for a in (V, ne, np_))
    tr = transport
    for l in range(nlev):
        cp = Coupled(nr, nz, R, z, phys, wall=wall, transport=tr)
        zero = np.zeros_like(V)
        (_, (Ae, Ap)) = cp.residual(V, ne, np_, ne, np_, zero, zero, dt_inv)
        J = cp.jacobian(V, ne, np_, Ae, Ap).tocsr()
        colour = (cp.ii + cp.jj) % 2
        idx = [np.nonzero(np.repeat(colour == c, 3))[0] for c in (0, 1)]
        # zebra: lines of one parity do not couple to each other (the
        # five-point stencil reaches i +- 1 only), so the restriction of J to
        # them is one block-tridiagonal system per line
        lidx = [np.nonzero(np.repeat(cp.ii % 2 == c, 3))[0] for c in (0, 1)]
        out.append(dict(cp=cp, J=J, z=z, idx=idx,
                        lu=[spla.splu(J[ix][:, ix].tocsc()) for ix in idx],
                        lidx=lidx, llu=[spla.splu(J[ix][:, ix].tocsc()) for ix in lidx]))
        if l + 1 < nlev:
            nr, nz = nr // 2, nz // 2
            z = np.ascontiguousarray(z[::2])
            V, ne, np_ = (np.ascontiguousarray(a[::2, ::2]) for a in (V, ne, np_))
            if tr is not None:
                tr = {k: np.ascontiguousarray(v[::2, ::2]) for k, v in tr.items()}
    return out


def block_colour_sweep(L, f, x, colour, lines=False):
    """Every node of one colour takes the value that satisfies its three
    equations with the other colour's current values (the nodes of one
    colour do not couple to each other).  lines: the colours are the axial
    lines of even and odd i, and every line of the colour satisfies all its
    equations at once (block zebra z-line Gauss-Seidel)."""
    ix = (L["lidx"] if lines else L["idx"])[colour]
    r = f - L["J"] @ x
    x[ix] += (L["llu"] if lines else L["lu"])[colour].solve(r[ix])


def _fieldwise(L, vec, fn):
    planes = L["cp"].unpack(vec)
    return [fn(p) for p in planes]


def block_restrict(L, Lc, r):
    from . import restrict
    planes = _fieldwise(L, r, lambda p: restrict(L["z"], p))
    return Lc["cp"].pack(*[p for p in planes])


def block_prolong(L, Lc, xc):
    from . import prolong_add
    out = []
    for pc in Lc["cp"].unpack(xc):
        pf = np.zeros((L["cp"].nr + 1, L["cp"].nz + 1))
        prolong_add(L["z"], np.ascontiguousarray(pc), pf)
        out.append(pf)
    return L["cp"].pack(*out)


def block_vcycle(levels, f, l=0, nu1=2, nu2=2, lines=False):
    """One V(nu1, nu2) cycle for J x = f on level l from x = 0; returns x.
    lines: block zebra z-line smoothing on every level above the coarsest
    (else collective red-black point smoothing)."""
    L = levels[l]
    if l == len(levels) - 1:
        return spla.spsolve(L["J"].tocsc(), f)
    x = np.zeros_like(f)
    for _ in range(nu1):
        block_colour_sweep(L, f, x, 0, lines)
        block_colour_sweep(L, f, x, 1, lines)
    fc = block_restrict(L, levels[l + 1], f - L["J"] @ x)
    x += block_prolong(L, levels[l + 1], block_vcycle(levels, fc, l + 1, nu1, nu2, lines))
    for _ in range(nu2):
        block_colour_sweep(L, f, x, 0, lines)
        block_colour_sweep(L, f, x, 1, lines)
    return x
