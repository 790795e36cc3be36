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
