"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module holds no arithmetic of the method: only the workload definition
(grid nodes, source profile, initial state, parameter draws).  The paper's
argon discharge data are not available, so these dimensionless inputs stand
in for the experiment of Sec. 3 with the same structure: an equidistant
radial grid, an axial grid refined towards both electrodes, a source peaked
in the discharge centre, Dirichlet electrodes and a potential drop between
them.
"""
import numpy as np

# Dimensionless physics of the synthetic workload (mobilities, diffusion
# coefficients and the Poisson coupling e*n0/eps0 of Eqs. 3-5).
PHYS = dict(mu_e=100.0, mu_p=1.0, D_e=1.0, D_p=0.01, k=1.0e3,
            V_bottom=0.0, V_top=1.0,
            ne_bottom=0.0, ne_top=0.0, np_bottom=0.0, np_top=0.0)
R = 1.0
D_GAP = 1.0


def z_cos(nz, d=D_GAP):
    """Axial nodes z_j = d/2 * (1 - cos(pi j / nz)), j = 0..nz (refined at
    both electrodes).  z_0 = 0 and z_nz = d exactly."""
    j = np.arange(nz + 1, dtype=np.float64)
    z = 0.5 * d * (1.0 - np.cos(np.pi * j / nz))
    z[0] = 0.0
    z[-1] = d
    return z


def source(nr, nz, z, R=R, amp=1.0e2, width=0.05, zc=0.5):
    """S[i, j] = amp * exp(-(r_i^2 + (z_j - zc)^2) / width), sampled at the
    nodes (r_i = i R / nr).  Used for both species (S_e = S_p)."""
    r = np.arange(nr + 1, dtype=np.float64) * (R / nr)
    return amp * np.exp(-(r[:, None] ** 2 + (z[None, :] - zc) ** 2) / width)


def initial_density(nr, nz, seed, level=1.0e-3, spread=0.01):
    """n[i, j] = level * (1 + spread * U(-1, 1)) from default_rng(seed),
    drawn as one (nr+1, nz+1) C-order array; electrode rows set to 0.
    Electrons and ions start from the same draw (no initial space charge)."""
    u = np.random.default_rng(seed).uniform(-1.0, 1.0, (nr + 1, nz + 1))
    n = level * (1.0 + spread * u)
    n[:, 0] = 0.0
    n[:, -1] = 0.0
    return n


def initial_potential(nr, nz, z, V_bottom=0.0, V_top=1.0, d=D_GAP):
    """V[i, j] = V_bottom + (V_top - V_bottom) z_j / d (linear in z)."""
    v = V_bottom + (V_top - V_bottom) * z / d
    return np.repeat(v[None, :], nr + 1, axis=0).copy()


def sweep_draws(n, seed, sizes=(64, 128, 256, 512)):
    """Parameter-sweep draws: grid size uniform over `sizes`, V_top ~ U(0.2, 5),
    mobility ratio mu_e/mu_p ~ logU(10, 1000).  mu_p = 1 and D_p = 0.01 stay
    fixed; mu_e = ratio and D_e = 0.01 * ratio keep D_e/D_p = mu_e/mu_p."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        N = int(rng.choice(sizes))
        vt = float(rng.uniform(0.2, 5.0))
        ratio = float(10.0 ** rng.uniform(1.0, 3.0))
        out.append(dict(N=N, V_top=vt, ratio=ratio, mu_e=ratio, D_e=0.01 * ratio,
                        mu_p=1.0, D_p=0.01))
    return out


# ---------------------------------------------------------------------------
# The paper's experiment (Sec. 3): obstructed glow discharge in argon, SI
# units.  d = 1.1 cm, R = 2.7 cm, 255.9 V across the gap, p = 0.514 torr;
# mu_e = 30/p m^2/(V s) (p in torr), D_e = mu_e kT_e/e with kT_e = 1 eV,
# D_p = mu_p kT_p/e with kT_p = 0.026 eV; Dirichlet wall at r = R
# (potential linear along it, densities 0).  The ion mobility comes from a
# reference the paper cites without giving a value; mu_p here is a stated
# substitute: the low-field reduced mobility of Ar+ in Ar, about 1.5 cm^2/(V s)
# at the standard gas density, scaled to the density at 0.514 torr and 300 K.
# ---------------------------------------------------------------------------
ELEMENTARY_CHARGE = 1.602176634e-19
EPSILON_0 = 8.8541878128e-12
ARGON_P_TORR = 0.514
ARGON_MU_P = 0.25  # m^2/(V s), substitute (see above)
ARGON = dict(mu_e=30.0 / ARGON_P_TORR, D_e=30.0 / ARGON_P_TORR * 1.0, mu_p=ARGON_MU_P, D_p=ARGON_MU_P * 0.026,
             k=ELEMENTARY_CHARGE / EPSILON_0, V_bottom=0.0, V_top=255.9,
             ne_bottom=0.0, ne_top=0.0, np_bottom=0.0, np_top=0.0)
ARGON_R = 0.027
ARGON_D = 0.011
# radial profile parameters (a, b) of the two cases shown in the paper
ARGON_CASES = ((30.0, 24.0), (10.0, 1.0))


def argon_sources(nr, nz, z, a, b, R=ARGON_R, d=ARGON_D):
    """S_e, S_p of Sec. 3 (m^-3 s^-1) at the nodes: radial profile
    1/(1 + exp(a r/R - b)) times the axial profiles
    S_p ~ 0.35e22 (z/d)^2 exp(-50 (z/d)^8) and
    S_e ~ 1.75e22 (z/d - 0.5) exp(-40 (z/d - 0.5)^2) for z/d > 0.5 (0 below);
    the paper's L is the gap d."""
    r = np.arange(nr + 1, dtype=np.float64) * (R / nr)
    x = np.asarray(z, dtype=np.float64) / d
    rad = 1.0 / (1.0 + np.exp(a * r / R - b))
    sp = 0.35e22 * x ** 2 * np.exp(-50.0 * x ** 8)
    se = np.where(x > 0.5, 1.75e22 * (x - 0.5) * np.exp(-40.0 * (x - 0.5) ** 2), 0.0)
    return np.ascontiguousarray(rad[:, None] * se[None, :]), np.ascontiguousarray(rad[:, None] * sp[None, :])


def argon_initial(nr, nz, z, n0=1.0e14, d=ARGON_D):
    """Initial state of the argon runs: uniform densities n0 (m^-3) inside,
    zero on the electrodes and the wall; potential linear in z."""
    n = np.full((nr + 1, nz + 1), n0)
    n[:, 0] = n[:, -1] = 0.0
    n[-1, :] = 0.0
    return initial_potential(nr, nz, z, 0.0, ARGON["V_top"], d), n, n.copy()


# ---------------------------------------------------------------------------
# Field-dependent transport of the synthetic workload (Sec. 2: mu(E), D(E)
# supplied by lookup tables, e.g. from a Monte Carlo code in a hybrid model):
# an electron mobility that saturates with the field, mu_e = mu0/(1 + E/Es),
# and an electron temperature that rises with it, D_e = mu_e T0 (1 + E/Et),
# tabulated on 41 field values in [0, 20] (dimensionless units of PHYS).
# ---------------------------------------------------------------------------
def electron_transport_table(mu0=100.0, T0=0.01, Es=2.0, Et=5.0, emax=20.0, n=41):
    """(E, mu_e(E), D_e(E)) sample arrays of the synthetic table."""
    E = np.linspace(0.0, emax, n)
    mu = mu0 / (1.0 + E / Es)
    return E, mu, mu * T0 * (1.0 + E / Et)
