// HIP kernels for gfx950 (MI355X): assembly of the cylindrical 5-point
// operators, Gauss-Seidel smoothers, residual with wave64 reductions, grid
// transfer and the coarsest-grid direct solve.
//
// Fields are row-major (nr+1) x pitch with z (j) contiguous: a wavefront
// reads 64 consecutive axial nodes of one radial row, so every load and
// store is a coalesced 512-byte (FP64) segment.
#include <math.h>

#include "mg_internal.h"

namespace mgf {

namespace {

constexpr int kTX = 64;  // threads along z (one wavefront)

inline __device__ int64_t at(const Geom &g, int i, int j) { return (int64_t)i * g.pitch + j; }

inline dim3 blk2d(const Geom &g) { return dim3(kTX, g.ty); }
inline dim3 grid2d(const Geom &g) {
    return dim3((g.nz + 1 + kTX - 1) / kTX, (g.nr + 1 + g.ty - 1) / g.ty);
}

// Scharfetter-Gummel Bernoulli function F(x) = x/(exp(x)-1) (Sec. 2, after
// Eq. 11), evaluated in FP64.  For |x| < 1e-3 the quotient cancels and the
// Taylor series 1 - x/2 + x^2/12 - x^4/720 (truncation < 1e-22) is used.
// G(x) = x exp(x)/(exp(x)-1) = F(-x).
inline __device__ double bern_F(double x) {
    if (fabs(x) < 1e-3) {
        double x2 = x * x;
        return 1.0 - 0.5 * x + x2 * (1.0 / 12.0) - x2 * x2 * (1.0 / 720.0);
    }
    return x / expm1(x);
}

// ---------------------------------------------------------------------------
// Poisson, Eqs. (5), (12), (13) in finite-volume form.  Row of node (i, j):
//   sum over faces area/dist * (V - V_nb) = vol * k * (n_p - n_e)
// r-face i+1/2 has area r_{i+1/2} dzc_j and distance dr; z-face j+1/2 has
// area w_i (radial width) and distance dz_j.  The axis has no inner face;
// r = R has no outer face (zero radial flux), or, with the Dirichlet wall of
// Sec. 3, the wall nodes are fixed (identity rows, right-hand side the wall
// potential on the finest level, 0 on the coarse levels).
// ---------------------------------------------------------------------------
__device__ inline double wall_value(const Geom &g, int j, double lo, double hi) {
    return lo + (hi - lo) * ((g.z[j] - g.z[0]) / (g.z[g.nz] - g.z[0]));
}

__global__ void k_poisson_assemble(Geom g, Op<double> op, const double *__restrict__ ne,
                                   const double *__restrict__ np, double k, int charge, double vlo, double vhi) {
    int j = blockIdx.x * kTX + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > g.nr || j > g.nz) return;
    int64_t p = at(g, i, j);
    if (j == 0 || j == g.nz) {
        op.a[p] = op.b[p] = op.c[p] = op.d[p] = op.e[p] = op.f[p] = 0.0;
        return;
    }
    if (g.wall && i == g.nr) {
        op.a[p] = op.c[p] = op.d[p] = op.e[p] = 0.0;
        op.b[p] = 1.0;
        op.f[p] = charge ? wall_value(g, j, vlo, vhi) : 0.0;
        return;
    }
    double w = g.wr[i], dzc = g.dzc[j];
    double ca = (i > 0) ? g.fr[i - 1] * dzc / g.dr : 0.0;
    double cc = (i < g.nr) ? g.fr[i] * dzc / g.dr : 0.0;
    double cd = w / g.dz[j - 1];
    double ce = w / g.dz[j];
    op.a[p] = -ca;
    op.c[p] = -cc;
    op.d[p] = -cd;
    op.e[p] = -ce;
    op.b[p] = ((ca + cc) + cd) + ce;
    op.f[p] = charge ? w * dzc * k * (np[p] - ne[p]) : 0.0;
}

// ---------------------------------------------------------------------------
// Backward-Euler Scharfetter-Gummel continuity operator, Eqs. (7)-(11):
//   vol (n - n^k)/dt + sum over faces area * phi_out = vol S
// with the face flux (Eq. 8; Eq. 9 in z, second term with F)
//   phi_{i+1/2} = D/dr (n_i G(alpha) - n_{i+1} F(alpha)),
//   alpha = q (V_{i+1} - V_i),  q = -s mu/D.
// dt_inv = 0 gives the steady operator.
// ---------------------------------------------------------------------------
// Face coefficients (D, q = -sgn mu/D): from the node values (mean of the
// two nodes) when mun is given, else the constants.
__device__ inline void face_qd(const double *mun, const double *Dn, double sgn, int64_t p, int64_t pn, double q,
                               double D, double &qf, double &Df) {
    if (mun) {
        Df = 0.5 * (Dn[p] + Dn[pn]);
        qf = -sgn * (0.5 * (mun[p] + mun[pn])) / Df;
    } else {
        Df = D;
        qf = q;
    }
}

__global__ void k_sg_assemble(Geom g, Op<double> op, const double *__restrict__ V,
                              const double *__restrict__ nk, const double *__restrict__ S,
                              double q0, double D0, double dt_inv, const double *__restrict__ mun,
                              const double *__restrict__ Dn, double sgn) {
    int j = blockIdx.x * kTX + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > g.nr || j > g.nz) return;
    int64_t p = at(g, i, j);
    if (j == 0 || j == g.nz) {
        op.a[p] = op.b[p] = op.c[p] = op.d[p] = op.e[p] = op.f[p] = 0.0;
        return;
    }
    if (g.wall && i == g.nr) {  // Dirichlet wall: density 0
        op.a[p] = op.c[p] = op.d[p] = op.e[p] = op.f[p] = 0.0;
        op.b[p] = 1.0;
        return;
    }
    double w = g.wr[i], dzc = g.dzc[j];
    double vol = w * dzc;
    double vc = V[p];
    double diag = vol * dt_inv;
    double ca = 0.0, cc = 0.0, q, D;
    if (i < g.nr) {
        face_qd(mun, Dn, sgn, p, p + g.pitch, q0, D0, q, D);
        double gg = g.fr[i] * dzc * D / g.dr;
        double al = q * (V[p + g.pitch] - vc);
        double F = bern_F(al);
        cc = -gg * F;
        diag += gg * bern_F(-al);
    }
    if (i > 0) {
        face_qd(mun, Dn, sgn, p, p - g.pitch, q0, D0, q, D);
        double gg = g.fr[i - 1] * dzc * D / g.dr;
        double al = q * (vc - V[p - g.pitch]);
        double F = bern_F(al);
        ca = -gg * bern_F(-al);
        diag += gg * F;
    }
    double ce, cd;
    {
        face_qd(mun, Dn, sgn, p, p + 1, q0, D0, q, D);
        double gg = w * D / g.dz[j];
        double al = q * (V[p + 1] - vc);
        ce = -gg * bern_F(al);
        diag += gg * bern_F(-al);
    }
    {
        face_qd(mun, Dn, sgn, p, p - 1, q0, D0, q, D);
        double gg = w * D / g.dz[j - 1];
        double al = q * (vc - V[p - 1]);
        cd = -gg * bern_F(-al);
        diag += gg * bern_F(al);
    }
    op.a[p] = ca;
    op.c[p] = cc;
    op.d[p] = cd;
    op.e[p] = ce;
    op.b[p] = diag;
    double src = S ? S[p] : 0.0;
    double old = nk ? nk[p] * dt_inv : 0.0;
    op.f[p] = vol * (src + old);
}

// Coarse potential = coincident fine value (nested grids).
__global__ void k_inject(Geom gf, const double *__restrict__ vf, Geom gc, double *__restrict__ vc) {
    int J = blockIdx.x * kTX + threadIdx.x;
    int I = blockIdx.y * blockDim.y + threadIdx.y;
    if (I > gc.nr || J > gc.nz) return;
    vc[at(gc, I, J)] = vf[at(gf, 2 * I, 2 * J)];
}

__global__ void k_set_electrodes(Geom g, double *u, double lo, double hi, const double *lohi, Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    u = boff(u, bo_);
    if (lohi) {
        lo = lohi[2 * blockIdx.z];
        hi = lohi[2 * blockIdx.z + 1];
    }

    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > g.nr) return;
    u[at(g, i, 0)] = lo;
    u[at(g, i, g.nz)] = hi;
}

__global__ void k_set_wall(Geom g, double *u, double lo, double hi, const double *lohi, Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    u = boff(u, bo_);
    g = geom_off(g, bo_);
    if (lohi) {
        lo = lohi[2 * blockIdx.z];
        hi = lohi[2 * blockIdx.z + 1];
    }
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j > g.nz) return;
    u[at(g, g.nr, j)] = wall_value(g, j, lo, hi);
}

// Particle flow (per radian of azimuth) out of the domain through the
// boundaries, from the SG face fluxes of Eqs. (8)-(9) at the state (V, n):
// out[0] cathode (face z_{1/2}, cells i < nr, or i <= nr without a wall),
// out[1] anode (face z_{nz-1/2}), out[2] wall (face r_{nr-1/2}, j = 1..nz-1,
// Dirichlet wall only).  One workgroup; fixed-order tree sums.
__global__ __launch_bounds__(1024) void k_boundary_flow(Geom g, const double *__restrict__ V,
                                                         const double *__restrict__ n, double q0, double D0,
                                                         double *__restrict__ out, const double *__restrict__ mun,
                                                         const double *__restrict__ Dn, double sgn) {
    __shared__ double sh[3][1024];
    const int t = threadIdx.x;
    double c0 = 0.0, c1 = 0.0, c2 = 0.0;
    const int imax = g.wall ? g.nr - 1 : g.nr;
    for (int i = t; i <= imax; i += 1024) {
        const double w = g.wr[i];
        double q, D;
        {
            const int64_t p0 = at(g, i, 0), p1 = at(g, i, 1);
            face_qd(mun, Dn, sgn, p0, p1, q0, D0, q, D);
            const double al = q * (V[p1] - V[p0]);
            const double phi = D / g.dz[0] * (n[p0] * bern_F(-al) - n[p1] * bern_F(al));
            c0 += -phi * w;
        }
        {
            const int64_t pa = at(g, i, g.nz - 1), pb = at(g, i, g.nz);
            face_qd(mun, Dn, sgn, pa, pb, q0, D0, q, D);
            const double al = q * (V[pb] - V[pa]);
            const double phi = D / g.dz[g.nz - 1] * (n[pa] * bern_F(-al) - n[pb] * bern_F(al));
            c1 += phi * w;
        }
    }
    if (g.wall)
        for (int j = 1 + t; j < g.nz; j += 1024) {
            const int64_t pa = at(g, g.nr - 1, j), pb = at(g, g.nr, j);
            double q, D;
            face_qd(mun, Dn, sgn, pa, pb, q0, D0, q, D);
            const double al = q * (V[pb] - V[pa]);
            const double phi = D / g.dr * (n[pa] * bern_F(-al) - n[pb] * bern_F(al));
            c2 += phi * g.fr[g.nr - 1] * g.dzc[j];
        }
    sh[0][t] = c0;
    sh[1][t] = c1;
    sh[2][t] = c2;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if (t < h)
            for (int k = 0; k < 3; ++k) sh[k][t] += sh[k][t + h];
        __syncthreads();
    }
    if (t < 3) out[t] = sh[t][0];
}

// Node transport from tables of |E| (see mg_transport_table): the field
// strength from central differences of V (one-sided at the electrodes and
// at r = R; the radial component vanishes on the axis), then linear
// interpolation between the bracketing table entries (clamped).
__global__ void k_transport_table(Geom g, const double *__restrict__ V, const double *__restrict__ Et,
                                  const double *__restrict__ mut, const double *__restrict__ Dt, int ntab,
                                  double *__restrict__ mu, double *__restrict__ Dv) {
    int j = blockIdx.x * kTX + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > g.nr || j > g.nz) return;
    const int64_t p = at(g, i, j);
    double er = 0.0, ez;
    if (i > 0 && i < g.nr)
        er = (V[p + g.pitch] - V[p - g.pitch]) / (2.0 * g.dr);
    else if (i == g.nr)
        er = (V[p] - V[p - g.pitch]) / g.dr;
    if (j == 0)
        ez = (V[p + 1] - V[p]) / g.dz[0];
    else if (j == g.nz)
        ez = (V[p] - V[p - 1]) / g.dz[g.nz - 1];
    else
        ez = (V[p + 1] - V[p - 1]) / (g.dz[j - 1] + g.dz[j]);
    const double E = sqrt(er * er + ez * ez);
    double m, d;
    if (E <= Et[0]) {
        m = mut[0];
        d = Dt[0];
    } else if (E >= Et[ntab - 1]) {
        m = mut[ntab - 1];
        d = Dt[ntab - 1];
    } else {
        int lo = 0, hi = ntab - 1;  // Et[lo] < E < Et[hi]
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (Et[mid] <= E)
                lo = mid;
            else
                hi = mid;
        }
        const double t = (E - Et[lo]) / (Et[hi] - Et[lo]);
        m = mut[lo] + t * (mut[hi] - mut[lo]);
        d = Dt[lo] + t * (Dt[hi] - Dt[lo]);
    }
    mu[p] = m;
    Dv[p] = d;
}

template <class T>
__global__ void k_fill(T *p, int64_t n, T v, Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    p = boff(p, bo_);

    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; t < n; t += stride) p[t] = v;
}

// ---------------------------------------------------------------------------
// Red-black point Gauss-Seidel half-sweep: nodes with (i+j)%2 == colour.
// Nodes of one colour only read nodes of the other colour, so the order of
// updates inside a half-sweep does not matter.
// ---------------------------------------------------------------------------
// The five coefficients and right-hand side of one node, in registers.
template <class T>
struct SRow {
    T a, b, c, d, e, f;
};
template <class T>
inline __device__ void load_srow(const Op<T> &op, int64_t p, SRow<T> &R) {
    R.a = op.a[p];
    R.b = op.b[p];
    R.c = op.c[p];
    R.d = op.d[p];
    R.e = op.e[p];
    R.f = op.f[p];
}
// Gauss-Seidel value of one node; xnb(t): neighbour t (0: i-1, 1: i+1,
// 2: j-1, 3: j+1).
template <class T, class XNb>
inline __device__ T solve_srow(const SRow<T> &R, bool has_im, bool has_ip, XNb xnb) {
    T s = R.f - R.d * xnb(2) - R.e * xnb(3);
    if (has_im) s -= R.a * xnb(0);
    if (has_ip) s -= R.c * xnb(1);
    return s / R.b;
}

template <class T>
__global__ void k_rbgs(Geom g, Op<T> op, T *__restrict__ x, int colour) {
    int j = blockIdx.x * kTX + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > g.nr || j < 1 || j >= g.nz) return;
    if (((i + j) & 1) != colour) return;
    int64_t p = at(g, i, j);
    SRow<T> R;
    load_srow(op, p, R);
    const int64_t nbp[4] = {p - g.pitch, p + g.pitch, p - 1, p + 1};
    x[p] = solve_srow(R, i > 0, i < g.nr, [&](int t) { return x[nbp[t]]; });
}

// ---------------------------------------------------------------------------
// Zebra z-line Gauss-Seidel half-sweep.  Every radial line i with
// i%2 == parity solves its tridiagonal system over j = 1..nz-1 exactly, the
// neighbouring lines held fixed.  One wavefront per line:
//   1. coalesced load of the line into LDS as (lower, diag, upper, rhs) with
//      the neighbour-line and electrode terms folded into rhs;
//   2. lane t owns CH consecutive rows; it eliminates its first CH-1 rows in
//      registers, expressing them through y_{t-1} (last unknown of lane t-1)
//      and its own last unknown y_t;
//   3. the 64 unknowns y_t satisfy a tridiagonal system that is solved by
//      parallel cyclic reduction over the lanes (6 shuffle steps);
//   4. each lane recovers its rows and the line is stored coalesced.
// Diagonal dominance of the line systems (M-matrices) makes the pivot-free
// elimination stable.  LDS rows are padded by one element every 16 so that
// the lanes' chunk reads spread over the banks.
// ---------------------------------------------------------------------------
inline __device__ int lds_pad(int q) { return q + (q >> 4); }

template <class T, int CH>
__global__ __launch_bounds__(64) void k_zline(Geom g, Op<T> op, T *__restrict__ x, int parity) {
    constexpr int NQ = 64 * CH;
    constexpr int NP = NQ + NQ / 16 + 1;
    __shared__ T sl[NP], sm[NP], su[NP], sr[NP];
    const int lane = threadIdx.x;
    const int i = parity + 2 * blockIdx.x;
    if (i > g.nr) return;
    const int m = g.nz - 1;  // unknowns on the line
    const int64_t row = (int64_t)i * g.pitch;
    const bool has_lo = i > 0, has_hi = i < g.nr;

    for (int q = lane; q < NQ; q += 64) {
        T l = 0, dg = 1, u = 0, rh = 0;
        if (q < m) {
            int64_t p = row + q + 1;
            l = op.d[p];
            dg = op.b[p];
            u = op.e[p];
            rh = op.f[p];
            if (has_lo) rh -= op.a[p] * x[p - g.pitch];
            if (has_hi) rh -= op.c[p] * x[p + g.pitch];
            if (q == 0) {
                rh -= l * x[p - 1];
                l = 0;
            }
            if (q == m - 1) {
                rh -= u * x[p + 1];
                u = 0;
            }
        }
        int s = lds_pad(q);
        sl[s] = l;
        sm[s] = dg;
        su[s] = u;
        sr[s] = rh;
    }
    __syncthreads();

    // Step 2: rows k = 0..CH-2 of this lane's chunk as
    // x_k = al[k] + be[k] * y_{t-1} + ga[k] * y_t.
    const int q0 = lane * CH;
    T al[CH > 1 ? CH - 1 : 1], be[CH > 1 ? CH - 1 : 1], ga[CH > 1 ? CH - 1 : 1];
    T lastA, lastB, lastC, lastD;  // reduced row, before neighbour terms
    {
        T cprev = 0, rprev = 0, sprev = 0;
#pragma unroll
        for (int k = 0; k < CH - 1; ++k) {
            int s = lds_pad(q0 + k);
            T l = sl[s], dg = sm[s], u = su[s], rh = sr[s];
            T den = dg - l * cprev;
            T inv = T(1) / den;
            T cp = u * inv;
            T rp = (rh - l * rprev) * inv;
            T sp = (k == 0 ? -l : -l * sprev) * inv;
            ga[k] = cp;  // hold c' here until back substitution
            al[k] = rp;
            be[k] = sp;
            cprev = cp;
            rprev = rp;
            sprev = sp;
        }
        // back substitution: row CH-2 couples to y_t through its upper entry
        if (CH > 1) {
            T c_last = ga[CH - 2];
            ga[CH - 2] = -c_last;
#pragma unroll
            for (int k = CH - 3; k >= 0; --k) {
                T cp = ga[k];
                al[k] = al[k] - cp * al[k + 1];
                be[k] = be[k] - cp * be[k + 1];
                ga[k] = -cp * ga[k + 1];
            }
        }
        int s = lds_pad(q0 + CH - 1);
        T l = sl[s], dg = sm[s], u = su[s], rh = sr[s];
        // x_{CH-2} in terms of (y_{t-1}, y_t)
        T a2 = (CH > 1) ? al[CH > 1 ? CH - 2 : 0] : T(0);
        T b2 = (CH > 1) ? be[CH > 1 ? CH - 2 : 0] : T(1);
        T g2 = (CH > 1) ? ga[CH > 1 ? CH - 2 : 0] : T(0);
        lastA = l * b2;
        lastB = dg + l * g2;
        lastC = u;
        lastD = rh - l * a2;
    }
    // first row of lane t+1 in terms of (y_t, y_{t+1})
    T a0 = (CH > 1) ? al[0] : T(0);
    T b0 = (CH > 1) ? be[0] : T(0);
    T g0 = (CH > 1) ? ga[0] : T(1);
    T na0 = __shfl_down(a0, 1);
    T nb0 = __shfl_down(b0, 1);
    T ng0 = __shfl_down(g0, 1);
    T A = lastA;
    T B = lastB + lastC * nb0;
    T C = lastC * ng0;
    T Dd = lastD - lastC * na0;
    if (lane == 63) C = 0;  // the last row of the line has no upper neighbour

    // Step 3: parallel cyclic reduction over the 64 lanes.
#pragma unroll
    for (int s = 1; s < 64; s <<= 1) {
        T Am = __shfl_up(A, s), Bm = __shfl_up(B, s), Cm = __shfl_up(C, s), Dm = __shfl_up(Dd, s);
        T Ap = __shfl_down(A, s), Bp = __shfl_down(B, s), Cp = __shfl_down(C, s), Dp = __shfl_down(Dd, s);
        bool lo = lane >= s, hi = lane + s < 64;
        if (!lo) { Am = 0; Bm = 1; Cm = 0; Dm = 0; }
        if (!hi) { Ap = 0; Bp = 1; Cp = 0; Dp = 0; }
        T k1 = A / Bm;
        T k2 = C / Bp;
        T nA = -Am * k1;
        T nC = -Cp * k2;
        T nB = B - Cm * k1 - Ap * k2;
        T nD = Dd - Dm * k1 - Dp * k2;
        A = nA;
        B = nB;
        C = nC;
        Dd = nD;
    }
    T y = Dd / B;
    T yprev = __shfl_up(y, 1);
    if (lane == 0) yprev = 0;

    // Step 4: recover the chunk and store the line.
    __syncthreads();
#pragma unroll
    for (int k = 0; k < CH - 1; ++k) sr[lds_pad(q0 + k)] = al[k] + be[k] * yprev + ga[k] * y;
    sr[lds_pad(q0 + CH - 1)] = y;
    __syncthreads();
    for (int q = lane; q < m; q += 64) x[row + q + 1] = sr[lds_pad(q)];
}

// ---------------------------------------------------------------------------
// Residual r = f - A x on the unknown nodes (0 on the electrode rows), and
// optionally per-block sums of (r/vol)^2 and (b_eff/vol)^2, where b_eff is f
// minus the electrode terms of the rows next to the electrodes.  Sums use a
// wave64 shuffle tree and a fixed-order combination of the block's waves,
// so they are deterministic.
// ---------------------------------------------------------------------------
template <class TA, class TX, class TR>
__global__ __launch_bounds__(1024) void k_residual(Geom g, Op<TA> op, const TX *__restrict__ fo,
                                                   const TX *__restrict__ x, TR *__restrict__ r,
                                                   double *__restrict__ partials) {
    int j = blockIdx.x * kTX + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    double rr = 0.0, bb = 0.0;
    if (i <= g.nr && j <= g.nz) {
        int64_t p = at(g, i, j);
        if (j == 0 || j == g.nz) {
            if (r) r[p] = TR(0);
        } else {
            double f = fo ? (double)fo[p] : (double)op.f[p];
            double xd = (double)x[p - 1], xu = (double)x[p + 1];
            double ax = (double)op.b[p] * (double)x[p] + (double)op.d[p] * xd + (double)op.e[p] * xu;
            if (i > 0) ax += (double)op.a[p] * (double)x[p - g.pitch];
            if (i < g.nr) ax += (double)op.c[p] * (double)x[p + g.pitch];
            double res = f - ax;
            if (r) r[p] = (TR)res;
            if (partials) {
                double be = f;
                if (j == 1) be -= (double)op.d[p] * xd;
                if (j == g.nz - 1) be -= (double)op.e[p] * xu;
                double vol = g.wr[i] * g.dzc[j];
                rr = (res / vol) * (res / vol);
                bb = (be / vol) * (be / vol);
            }
        }
    }
    if (!partials) return;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        rr += __shfl_xor(rr, off);
        bb += __shfl_xor(bb, off);
    }
    __shared__ double srr[kMaxTY], sbb[kMaxTY];
    if (threadIdx.x == 0) {
        srr[threadIdx.y] = rr;
        sbb[threadIdx.y] = bb;
    }
    __syncthreads();
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < (int)blockDim.y; ++w) {
            a += srr[w];
            b += sbb[w];
        }
        int blk = blockIdx.y * gridDim.x + blockIdx.x;
        partials[2 * blk] = a;
        partials[2 * blk + 1] = b;
    }
}

// Sum `ncomp`-component partials of nblocks blocks in a fixed order.
__global__ __launch_bounds__(256) void k_sum_partials(const double *__restrict__ part, int nblocks,
                                                       int ncomp, double *__restrict__ out, Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    part = boff(part, bo_);
    out = boff(out, bo_);

    __shared__ double sh[256 * 4];
    for (int c = 0; c < ncomp; ++c) {
        double acc = sum_strided(part, nblocks, threadIdx.x, 256, ncomp, c);
        sh[c * 256 + threadIdx.x] = acc;
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < ncomp; ++c) sh[c * 256 + threadIdx.x] += sh[c * 256 + threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int c = 0; c < ncomp; ++c) out[c] = sh[c * 256];
}

// Per-block sums of (a-b)^2 and a^2 over the unknown nodes (steady test).
__global__ __launch_bounds__(1024) void k_diff_norms(Geom g, const double *__restrict__ a,
                                                     const double *__restrict__ b,
                                                     double *__restrict__ partials, Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    a = boff(a, bo_);
    b = boff(b, bo_);
    partials = boff(partials, bo_);
    int j = blockIdx.x * kTX + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    double dd = 0.0, aa = 0.0;

    if (i <= g.nr && j >= 1 && j < g.nz) {
        int64_t p = at(g, i, j);
        double t = a[p] - b[p];
        dd = t * t;
        aa = a[p] * a[p];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        dd += __shfl_xor(dd, off);
        aa += __shfl_xor(aa, off);
    }
    __shared__ double s1[kMaxTY], s2[kMaxTY];
    if (threadIdx.x == 0) {
        s1[threadIdx.y] = dd;
        s2[threadIdx.y] = aa;
    }
    __syncthreads();
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        double u = 0.0, v = 0.0;
        for (int w = 0; w < (int)blockDim.y; ++w) {
            u += s1[w];
            v += s2[w];
        }
        int blk = blockIdx.y * gridDim.x + blockIdx.x;
        partials[2 * blk] = u;
        partials[2 * blk + 1] = v;
    }
}

// ---------------------------------------------------------------------------
// Restriction = transpose of the bilinear prolongation, applied to the
// finite-volume residual: coarse node (I, J) gathers fine nodes
// (2I+di, 2J+dj), weights 1/2 for di = +-1 (equidistant r), and for dj = +-1
// the z-distance weights of the interpolation that feeds those fine nodes.
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_restrict(Geom gf, const T *__restrict__ rf, Geom gc, T *__restrict__ fc) {
    int J = blockIdx.x * kTX + threadIdx.x;
    int I = blockIdx.y * blockDim.y + threadIdx.y;
    if (I > gc.nr || J > gc.nz) return;
    int64_t pc = at(gc, I, J);
    if (J == 0 || J == gc.nz) {
        fc[pc] = T(0);
        return;
    }
    T wdn = T(1) - (T)gf.wl[J - 1];  // fine node 2J-1 -> upper coarse node J
    T wup = (T)gf.wl[J];             // fine node 2J+1 -> lower coarse node J
    T acc = 0;
    for (int di = -1; di <= 1; ++di) {
        int i = 2 * I + di;
        if (i < 0 || i > gf.nr) continue;
        T wi = (di == 0) ? T(1) : T(0.5);
        int64_t p = at(gf, i, 2 * J);
        acc += wi * (wdn * rf[p - 1] + rf[p] + wup * rf[p + 1]);
    }
    fc[pc] = acc;
}

// Bilinear prolongation of the coarse correction, added on fine unknowns.
template <class T>
inline __device__ T prolong_s(const Geom &gf, const Geom &gc, const T *xc, int i, int j) {
    int I0 = i >> 1, I1 = (i + 1) >> 1;
    T v0, v1;
    if ((j & 1) == 0) {
        v0 = xc[at(gc, I0, j >> 1)];
        v1 = xc[at(gc, I1, j >> 1)];
    } else {
        int J = j >> 1;
        T wl = (T)gf.wl[J];
        T wu = T(1) - wl;
        v0 = wl * xc[at(gc, I0, J)] + wu * xc[at(gc, I0, J + 1)];
        v1 = wl * xc[at(gc, I1, J)] + wu * xc[at(gc, I1, J + 1)];
    }
    return (i & 1) ? T(0.5) * (v0 + v1) : v0;
}

template <class T>
__global__ void k_prolong(Geom gf, T *__restrict__ xf, Geom gc, const T *__restrict__ xc) {
    int j = blockIdx.x * kTX + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > gf.nr || j < 1 || j >= gf.nz) return;
    T v = xf[at(gf, i, j)];
    v += prolong_s(gf, gc, xc, i, j);
    xf[at(gf, i, j)] = v;
}

// ---------------------------------------------------------------------------
// One full red-black sweep in one launch (scalar operator), from the input to
// xout (distinct buffers).  The input is xin, or zero (zin != 0, xin not
// read), or xin plus the bilinear prolongation of the coarse correction xc
// (xc != nullptr).  A workgroup owns a kSWs x SH tile and ring threads; the
// input over the tile and a 2-node ring is staged in LDS, every thread holds
// its node's coefficients in registers, the colour-0 nodes of tile and
// 1-node ring are updated into LDS, then the tile's colour-1 nodes.  The
// electrode rows of the tile are copied from the input, so xout is a whole
// field.  Values equal two k_rbgs launches (after k_prolong).
// ---------------------------------------------------------------------------
constexpr int kSWs = 32;
template <int SH>
struct STile {
    static constexpr int kSR = (2 * kSWs + 2 * SH + kSWs - 1) / kSWs;
};
template <class T, int SH>
__global__ __launch_bounds__(kSWs *(SH + STile<SH>::kSR)) void k_rb_sweep_s(Geom g, Op<T> op,
                                                                           const T *__restrict__ xin,
                                                                           T *__restrict__ xout, int zin, Geom gc,
                                                                           const T *__restrict__ xc) {
    constexpr int kSH = SH, kSR = STile<SH>::kSR;
    constexpr int W = kSWs + 2, W2 = kSWs + 4;
    __shared__ T lx[(kSH + 2) * W];
    __shared__ T lin[(kSH + 4) * W2];
    int tx = blockIdx.x, ty = blockIdx.y;
    if (g.xcd) {  // tiles in XCD-contiguous order (neighbouring tiles share ring lines in one L2)
        const int nx = gridDim.x, n = gridDim.x * gridDim.y;
        const int b = blockIdx.y * nx + blockIdx.x;
        const int k = b & 7, q = n >> 3, r = n & 7;
        const int t = k * q + (k < r ? k : r) + (b >> 3);
        tx = t % nx;
        ty = t / nx;
    }
    const int i0 = ty * kSH, j0 = tx * kSWs;
    const int ti = threadIdx.y, tj = threadIdx.x, tid = ti * kSWs + tj;
    for (int t = tid; t < (kSH + 4) * W2; t += kSWs * (kSH + kSR)) {
        const int ii = i0 - 2 + t / W2, jj = j0 - 2 + t % W2;
        if (ii < 0 || ii > g.nr || jj < 0 || jj > g.nz) continue;
        T v = zin ? T(0) : xin[at(g, ii, jj)];
        if (xc && jj >= 1 && jj < g.nz) v += prolong_s(g, gc, xc, ii, jj);
        lin[t] = v;
    }
    int ni, nj;
    if (ti < kSH) {
        ni = i0 + ti;
        nj = j0 + tj;
    } else {
        const int k = (ti - kSH) * kSWs + tj;
        if (k < kSWs) {
            ni = i0 - 1;
            nj = j0 + k;
        } else if (k < 2 * kSWs) {
            ni = i0 + kSH;
            nj = j0 + k - kSWs;
        } else if (k < 2 * kSWs + kSH) {
            ni = i0 + k - 2 * kSWs;
            nj = j0 - 1;
        } else if (k < 2 * kSWs + 2 * kSH) {
            ni = i0 + k - 2 * kSWs - kSH;
            nj = j0 + kSWs;
        } else {
            ni = -1;  // spare ring thread
            nj = 0;
        }
    }
    const bool tile = ti < kSH;
    const bool valid = ni >= 0 && ni <= g.nr && nj >= 1 && nj < g.nz;
    const bool red = ((ni + nj) & 1) == 0;
    const int64_t p = at(g, ni, nj);
    SRow<T> R;
    if (valid && (tile || red)) load_srow(op, p, R);
    __syncthreads();
    auto in_at = [&](int ii, int jj) { return lin[(ii - i0 + 2) * W2 + (jj - j0 + 2)]; };
    const int dni[4] = {-1, 1, 0, 0}, dnj[4] = {0, 0, -1, 1};
    if (tile && ni <= g.nr && (nj == 0 || nj == g.nz)) xout[p] = in_at(ni, nj);  // electrode rows
    if (valid && red) {
        const T v = solve_srow(R, ni > 0, ni < g.nr, [&](int t) { return in_at(ni + dni[t], nj + dnj[t]); });
        lx[(ni - i0 + 1) * W + (nj - j0 + 1)] = v;
        if (tile) xout[p] = v;
    }
    __syncthreads();
    if (!tile || !valid || red) return;
    const bool fixed[4] = {false, false, nj - 1 == 0, nj + 1 == g.nz};
    xout[p] = solve_srow(R, ni > 0, ni < g.nr, [&](int t) {
        const int ii = ni + dni[t], jj = nj + dnj[t];
        return fixed[t] ? in_at(ii, jj) : lx[(ii - i0 + 1) * W + (jj - j0 + 1)];
    });
}

// Fine residual (as k_residual: FP64 arithmetic, stored as T) at node (i, j).
template <class T>
inline __device__ T residual_s(const Geom &g, const Op<T> &op, const T *x, int i, int j) {
    const int64_t p = at(g, i, j);
    double f = (double)op.f[p];
    double xd = (double)x[p - 1], xu = (double)x[p + 1];
    double ax = (double)op.b[p] * (double)x[p] + (double)op.d[p] * xd + (double)op.e[p] * xu;
    if (i > 0) ax += (double)op.a[p] * (double)x[p - g.pitch];
    if (i < g.nr) ax += (double)op.c[p] * (double)x[p + g.pitch];
    return (T)(f - ax);
}

// Restriction of a fine residual held in LDS (window origin fi0, fj0, row
// length FW) to coarse node (I, J), as k_restrict.
template <class T>
inline __device__ T restrict_s(const Geom &gf, const Geom &gc, const T *lr, int fi0, int fj0, int FW, int I, int J) {
    if (J == 0 || J == gc.nz) return T(0);
    T wdn = T(1) - (T)gf.wl[J - 1];
    T wup = (T)gf.wl[J];
    T acc = 0;
    for (int di = -1; di <= 1; ++di) {
        int i = 2 * I + di;
        if (i < 0 || i > gf.nr) continue;
        T wi = (di == 0) ? T(1) : T(0.5);
        const int l = (i - fi0) * FW + (2 * J - fj0);
        acc += wi * (wdn * lr[l - 1] + lr[l] + wup * lr[l + 1]);
    }
    return acc;
}

// Residual and restriction in one launch: coarse tile kCWs x kCHs, fine
// window (2 kCHs + 1) x (2 kCWs + 1) of residuals in LDS, one fine node per
// thread of a 64 x 10 workgroup.  Values equal k_residual + k_restrict.
constexpr int kCWs = 32, kCHs = 4;
static_assert((2 * kCWs + 1) * (2 * kCHs + 1) <= 64 * 10, "one fine node per thread");
template <class T>
__global__ __launch_bounds__(640) void k_residual_restrict_s(Geom gf, Op<T> op, const T *__restrict__ x, Geom gc,
                                                             T *__restrict__ fc) {
    constexpr int FW = 2 * kCWs + 1, FH = 2 * kCHs + 1;
    __shared__ T lr[FH * FW];
    const int I0 = blockIdx.y * kCHs, J0 = blockIdx.x * kCWs;
    const int fi0 = 2 * I0 - 1, fj0 = 2 * J0 - 1;
    const int tid = threadIdx.y * blockDim.x + threadIdx.x;
    if (tid < FH * FW) {
        const int i = fi0 + tid / FW, j = fj0 + tid % FW;
        if (i >= 0 && i <= gf.nr && j >= 0 && j <= gf.nz)
            lr[tid] = (j == 0 || j == gf.nz) ? T(0) : residual_s(gf, op, x, i, j);
    }
    __syncthreads();
    if (tid >= kCWs * kCHs) return;
    const int I = I0 + tid / kCWs, J = J0 + tid % kCWs;
    if (I > gc.nr || J > gc.nz) return;
    fc[at(gc, I, J)] = restrict_s(gf, gc, lr, fi0, fj0, FW, I, J);
}

// ---------------------------------------------------------------------------
// The coarse end of the scalar V-cycle (levels 0..n-1 of F, the last the
// coarsest) in one workgroup, every level's coefficients, right-hand side,
// correction and residual staged in LDS (compact, pitch nz+1); the top
// level's correction is written back.  Node by node the arithmetic of the
// per-level kernels (red-black half-sweeps, residual, restriction, explicit
// coarsest inverse, prolongation).  Corrections start from zero.
// ---------------------------------------------------------------------------
constexpr int kSubPoolS = 15360;
template <class T>
__global__ __launch_bounds__(1024) void k_subcycle_s(FusedScalar<T> F) {
    __shared__ T pool[kSubPoolS];
    __shared__ T rhs[kMaxCoarseUnknowns];
    const int n = F.n, nt = blockDim.x;
    auto nodes = [&](int q) { return (F.g[q].nr + 1) * (F.g[q].nz + 1); };
    auto off = [&](int q) {
        int o = 0;
        for (int t = 0; t < q; ++t) o += 8 * nodes(t);
        return o;
    };
    auto geom = [&](int q) {
        Geom g = F.g[q];
        g.pitch = g.nz + 1;
        return g;
    };
    auto opq = [&](int q) {
        T *b = pool + off(q);
        const int nn = nodes(q);
        return Op<T>{b, b + nn, b + 2 * nn, b + 3 * nn, b + 4 * nn, b + 5 * nn};
    };
    auto xq = [&](int q) { return pool + off(q) + 6 * nodes(q); };
    auto rq = [&](int q) { return pool + off(q) + 7 * nodes(q); };
    // stage coefficients and right-hand sides; zero the corrections
    for (int q = 0; q < n; ++q) {
        const Geom &gg = F.g[q];
        const int w = gg.nz + 1, nn = nodes(q);
        const Op<T> &src = F.op[q];
        const T *arr[6] = {src.a, src.b, src.c, src.d, src.e, src.f};
        T *dst = pool + off(q);
        for (int t = threadIdx.x; t < 6 * nn; t += nt) {
            const int k = t / nn, node = t % nn;
            dst[t] = arr[k][(int64_t)(node / w) * gg.pitch + node % w];
        }
        T *x = xq(q);
        for (int t = threadIdx.x; t < nn; t += nt) x[t] = T(0);
    }
    __syncthreads();
    for (int q = 0; q < n - 1; ++q) {
        const Geom g = geom(q);
        const Op<T> op = opq(q);
        T *x = xq(q);
        T *r = rq(q);
        const int nn = nodes(q);
        for (int s = 0; s < F.nu1; ++s)
            for (int col = 0; col < 2; ++col) {
                for (int t = threadIdx.x; t < nn; t += nt) {
                    const int i = t / (g.nz + 1), j = t % (g.nz + 1);
                    if (j < 1 || j >= g.nz || ((i + j) & 1) != col) continue;
                    const int64_t p = at(g, i, j);
                    SRow<T> R;
                    load_srow(op, p, R);
                    const int64_t nbp[4] = {p - g.pitch, p + g.pitch, p - 1, p + 1};
                    x[p] = solve_srow(R, i > 0, i < g.nr, [&](int k) { return x[nbp[k]]; });
                }
                __syncthreads();
            }
        for (int t = threadIdx.x; t < nn; t += nt) {
            const int i = t / (g.nz + 1), j = t % (g.nz + 1);
            r[t] = (j == 0 || j == g.nz) ? T(0) : residual_s(g, op, x, i, j);
        }
        __syncthreads();
        const Geom gc = geom(q + 1);
        const Op<T> oc = opq(q + 1);
        for (int t = threadIdx.x; t < nodes(q + 1); t += nt) {
            const int I = t / (gc.nz + 1), J = t % (gc.nz + 1);
            // the fine residual window is the whole level: origin (0, 0), row length nz + 1
            oc.f[t] = (J == 0 || J == gc.nz) ? T(0) : restrict_s(g, gc, r, 0, 0, g.nz + 1, I, J);
        }
        __syncthreads();
    }
    {
        // coarsest level: x = A^{-1} f (electrode terms with the zero correction)
        const int q = n - 1;
        const Geom g = geom(q);
        const Op<T> op = opq(q);
        T *x = xq(q);
        const int m = g.nz - 1, nc = (g.nr + 1) * m;
        for (int row = threadIdx.x; row < nc; row += nt) {
            const int i = row / m, j = row % m + 1;
            const int64_t p = at(g, i, j);
            T v = op.f[p];
            if (j == 1) v -= op.d[p] * x[p - 1];
            if (j == m) v -= op.e[p] * x[p + 1];
            rhs[row] = v;
        }
        __syncthreads();
        for (int row = threadIdx.x; row < nc; row += nt) {
            T acc = 0;
            for (int k = 0; k < nc; ++k) acc += F.invT[(int64_t)k * nc + row] * rhs[k];
            const int i = row / m, j = row % m + 1;
            x[at(g, i, j)] = acc;
        }
        __syncthreads();
    }
    for (int q = n - 2; q >= 0; --q) {
        const Geom g = geom(q), gc = geom(q + 1);
        const Op<T> op = opq(q);
        T *x = xq(q);
        const T *xcq = xq(q + 1);
        const int nn = nodes(q);
        for (int t = threadIdx.x; t < nn; t += nt) {
            const int i = t / (g.nz + 1), j = t % (g.nz + 1);
            if (j < 1 || j >= g.nz) continue;
            T v = x[t];
            v += prolong_s(g, gc, xcq, i, j);
            x[t] = v;
        }
        __syncthreads();
        for (int s = 0; s < F.nu2; ++s)
            for (int col = 0; col < 2; ++col) {
                for (int t = threadIdx.x; t < nn; t += nt) {
                    const int i = t / (g.nz + 1), j = t % (g.nz + 1);
                    if (j < 1 || j >= g.nz || ((i + j) & 1) != col) continue;
                    const int64_t p = at(g, i, j);
                    SRow<T> R;
                    load_srow(op, p, R);
                    const int64_t nbp[4] = {p - g.pitch, p + g.pitch, p - 1, p + 1};
                    x[p] = solve_srow(R, i > 0, i < g.nr, [&](int k) { return x[nbp[k]]; });
                }
                __syncthreads();
            }
    }
    // the top level's correction back to its field (whole field, electrode rows zero)
    const Geom &g0 = F.g[0];
    const int w = g0.nz + 1, nn = nodes(0);
    const T *x0 = xq(0);
    for (int t = threadIdx.x; t < nn; t += nt) F.x0[(int64_t)(t / w) * g0.pitch + t % w] = x0[t];
}

// Full-field bilinear interpolation (used for the multilevel prolongation of
// a whole state, electrode rows included).
__global__ void k_prolong_state(Geom gf, double *__restrict__ xf, Geom gc, const double *__restrict__ xc) {
    int j = blockIdx.x * kTX + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > gf.nr || j > gf.nz) return;
    int I0 = i >> 1, I1 = (i + 1) >> 1;
    double v0, v1;
    if ((j & 1) == 0) {
        v0 = xc[at(gc, I0, j >> 1)];
        v1 = xc[at(gc, I1, j >> 1)];
    } else {
        int J = j >> 1;
        double wl = gf.wl[J];
        double wu = 1.0 - wl;
        v0 = wl * xc[at(gc, I0, J)] + wu * xc[at(gc, I0, J + 1)];
        v1 = wl * xc[at(gc, I1, J)] + wu * xc[at(gc, I1, J + 1)];
    }
    xf[at(gf, i, j)] = (i & 1) ? 0.5 * (v0 + v1) : v0;
}

// ---------------------------------------------------------------------------
// Coarsest grid: explicit inverse by Gauss-Jordan elimination with partial
// pivoting (one workgroup), stored transposed so that the per-cycle solve
// x = A^{-1} b reads it coalesced.  Unknown (i, j) has index i*(nz-1)+j-1.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_coarse_factor(Geom g, Op<double> op, double *__restrict__ M,
                                                        double *__restrict__ invT, float *__restrict__ invT32) {
    const int m = g.nz - 1;
    const int n = (g.nr + 1) * m;
    const int n2 = 2 * n;
    // [A | I]
    for (int t = threadIdx.x; t < n * n2; t += blockDim.x) M[t] = 0.0;
    __syncthreads();
    for (int row = threadIdx.x; row < n; row += blockDim.x) {
        int i = row / m, j = row % m + 1;
        int64_t p = at(g, i, j);
        double *Mr = M + (int64_t)row * n2;
        Mr[row] = op.b[p];
        if (i > 0) Mr[row - m] = op.a[p];
        if (i < g.nr) Mr[row + m] = op.c[p];
        if (j > 1) Mr[row - 1] = op.d[p];
        if (j < m) Mr[row + 1] = op.e[p];
        Mr[n + row] = 1.0;
    }
    __syncthreads();
    __shared__ int piv;
    __shared__ double fcol[kMaxCoarseUnknowns];
    for (int col = 0; col < n; ++col) {
        pivot_search_wave0(M, n2, col, n, &piv);
        __syncthreads();
        const int pv = piv;
        if (pv != col)
            for (int t = threadIdx.x; t < n2; t += blockDim.x) {
                double tmp = M[(int64_t)col * n2 + t];
                M[(int64_t)col * n2 + t] = M[(int64_t)pv * n2 + t];
                M[(int64_t)pv * n2 + t] = tmp;
            }
        __syncthreads();
        const double pinv = 1.0 / M[(int64_t)col * n2 + col];
        __syncthreads();
        for (int t = threadIdx.x; t < n2; t += blockDim.x) M[(int64_t)col * n2 + t] *= pinv;
        for (int rr = threadIdx.x; rr < n; rr += blockDim.x) fcol[rr] = M[(int64_t)rr * n2 + col];
        __syncthreads();
        // eliminate column `col` from every other row
        for (int64_t t = threadIdx.x; t < (int64_t)n * n2; t += blockDim.x) {
            int rr = (int)(t / n2), cc = (int)(t % n2);
            if (rr == col) continue;
            double fct = fcol[rr];
            if (fct != 0.0) M[(int64_t)rr * n2 + cc] -= fct * M[(int64_t)col * n2 + cc];
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
        int row = t / n, k = t % n;
        double v = M[(int64_t)row * n2 + n + k];
        invT[(int64_t)k * n + row] = v;
        if (invT32) invT32[(int64_t)k * n + row] = (float)v;
    }
}

// Same factorisation with the augmented matrix resident in LDS (n <= 63).
constexpr int kLdsGJ = 63;
__global__ __launch_bounds__(1024) void k_coarse_factor_lds(Geom g, Op<double> op, double *__restrict__ invT,
                                                             float *__restrict__ invT32) {
    const int m = g.nz - 1;
    const int n = (g.nr + 1) * m;
    const int n2 = 2 * n;
    // two copies of the augmented matrix: column step k reads one, writes the other
    __shared__ double Mb[2][kLdsGJ * 2 * kLdsGJ];
    __shared__ int piv;
    double *M = Mb[0];
    for (int t = threadIdx.x; t < n * n2; t += blockDim.x) M[t] = 0.0;
    __syncthreads();
    for (int row = threadIdx.x; row < n; row += blockDim.x) {
        int i = row / m, j = row % m + 1;
        int64_t p = at(g, i, j);
        double *Mr = M + row * n2;
        Mr[row] = op.b[p];
        if (i > 0) Mr[row - m] = op.a[p];
        if (i < g.nr) Mr[row + m] = op.c[p];
        if (j > 1) Mr[row - 1] = op.d[p];
        if (j < m) Mr[row + 1] = op.e[p];
        Mr[n + row] = 1.0;
    }
    __syncthreads();
    // Gauss-Jordan with partial pivoting, two barriers per column: the pivot
    // search, then every element of the next copy in one pass (scaled pivot
    // row, exchanged row, other rows eliminated against the scaled pivot row).
    constexpr int kPer = (kLdsGJ * 2 * kLdsGJ + 1023) / 1024;
    const int total = n * n2;
    int cur = 0;
    for (int col = 0; col < n; ++col) {
        const double *A = Mb[cur];
        double *B = Mb[cur ^ 1];
        pivot_search_wave0(A, n2, col, n, &piv);
        __syncthreads();
        const int pv = piv;
        const double pinv = 1.0 / A[pv * n2 + col];
        const double fpv = A[col * n2 + col];
        double v[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int t = threadIdx.x + k * 1024;
            if (t >= total) break;
            const int rr = t / n2, cc = t - rr * n2;
            const double prc = A[pv * n2 + cc] * pinv;
            if (rr == col) {
                v[k] = prc;
            } else {
                const double src = (rr == pv) ? A[col * n2 + cc] : A[rr * n2 + cc];
                const double fct = (rr == pv) ? fpv : A[rr * n2 + col];
                v[k] = (fct != 0.0) ? src - fct * prc : src;
            }
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int t = threadIdx.x + k * 1024;
            if (t >= total) break;
            B[t] = v[k];
        }
        __syncthreads();
        cur ^= 1;
    }
    M = Mb[cur];
    for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
        int row = t / n, k = t % n;
        double v = M[row * n2 + n + k];
        invT[(int64_t)k * n + row] = v;
        if (invT32) invT32[(int64_t)k * n + row] = (float)v;
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_coarse_solve(Geom g, Op<T> op, const T *__restrict__ invT,
                                                       T *__restrict__ x) {
    const int m = g.nz - 1;
    const int n = (g.nr + 1) * m;
    __shared__ T rhs[kMaxCoarseUnknowns];
    for (int row = threadIdx.x; row < n; row += blockDim.x) {
        int i = row / m, j = row % m + 1;
        int64_t p = at(g, i, j);
        T v = op.f[p];
        if (j == 1) v -= op.d[p] * x[p - 1];
        if (j == m) v -= op.e[p] * x[p + 1];
        rhs[row] = v;
    }
    __syncthreads();
    for (int row = threadIdx.x; row < n; row += blockDim.x) {
        T acc = 0;
        for (int k = 0; k < n; ++k) acc += invT[(int64_t)k * n + row] * rhs[k];
        int i = row / m, j = row % m + 1;
        x[at(g, i, j)] = acc;
    }
}

__global__ void k_copy_field(Geom g, const double *__restrict__ s, double *__restrict__ d, Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    s = boff(s, bo_);
    d = boff(d, bo_);

    int j = blockIdx.x * kTX + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > g.nr || j > g.nz) return;
    d[at(g, i, j)] = s[at(g, i, j)];
}

__global__ void k_to_f32(Geom g, const double *__restrict__ s, float *__restrict__ d) {
    int j = blockIdx.x * kTX + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > g.nr || j > g.nz) return;
    d[at(g, i, j)] = (float)s[at(g, i, j)];
}

__global__ void k_add_f32(Geom g, double *__restrict__ x, const float *__restrict__ e) {
    int j = blockIdx.x * kTX + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > g.nr || j < 1 || j >= g.nz) return;
    x[at(g, i, j)] += (double)e[at(g, i, j)];
}

// FP32 copy of a five-point operator that keeps its column sums.  Rounding
// b on its own would bury the small part of the diagonal that makes the
// matrix non-singular (vol/dt plus electrode outflow, next to fluxes many
// orders larger), so b is rebuilt from the exact FP64 column excess
// delta_i = b_i + sum of the entries of column i in the neighbour rows,
// minus those neighbour entries as rounded to FP32.
__device__ inline double col_nb_sum(const Geom &g, const double *a, const double *c, const double *d,
                                    const double *e, int i, int j, bool f32round) {
    double s = 0.0;
    auto rd = [&](double v) { return f32round ? (double)(float)v : v; };
    if (i > 0) s += rd(c[at(g, i - 1, j)]);       // row (i-1, j) couples to (i, j) through c
    if (i < g.nr) s += rd(a[at(g, i + 1, j)]);    // row (i+1, j) through a
    if (j > 1) s += rd(e[at(g, i, j - 1)]);       // row (i, j-1) through e
    if (j < g.nz - 1) s += rd(d[at(g, i, j + 1)]);  // row (i, j+1) through d
    return s;
}

__global__ void k_op_to_f32(Geom g, Op<double> o, Op<float> o32) {
    int j = blockIdx.x * kTX + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > g.nr || j > g.nz) return;
    int64_t p = at(g, i, j);
    o32.a[p] = (float)o.a[p];
    o32.c[p] = (float)o.c[p];
    o32.d[p] = (float)o.d[p];
    o32.e[p] = (float)o.e[p];
    o32.f[p] = 0.0f;
    if (j == 0 || j == g.nz) {
        o32.b[p] = (float)o.b[p];
        return;
    }
    double excess = o.b[p] + col_nb_sum(g, o.a, o.c, o.d, o.e, i, j, false);
    o32.b[p] = (float)(excess - col_nb_sum(g, o.a, o.c, o.d, o.e, i, j, true));
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

void launch_poisson_assemble(const Geom &g, Op<double> op, const double *ne, const double *np,
                             double k, bool charge, double vlo, double vhi, hipStream_t s) {
    k_poisson_assemble<<<grid2d(g), blk2d(g), 0, s>>>(g, op, ne, np, k, charge ? 1 : 0, vlo, vhi);
}

void launch_sg_assemble(const Geom &g, Op<double> op, const double *V, const double *nk,
                        const double *S, double q, double D, double dt_inv, hipStream_t s, const double *mun,
                        const double *Dn, double sgn) {
    k_sg_assemble<<<grid2d(g), blk2d(g), 0, s>>>(g, op, V, nk, S, q, D, dt_inv, mun, Dn, sgn);
}

void launch_transport_table(const Geom &g, const double *V, const double *Et, const double *mut, const double *Dt,
                            int ntab, double *mu, double *D, hipStream_t s) {
    k_transport_table<<<grid2d(g), blk2d(g), 0, s>>>(g, V, Et, mut, Dt, ntab, mu, D);
}

void launch_inject(const Geom &gf, const double *vf, const Geom &gc, double *vc, hipStream_t s) {
    k_inject<<<grid2d(gc), blk2d(gc), 0, s>>>(gf, vf, gc, vc);
}

void launch_set_electrodes(const Geom &g, double *u, double lo, double hi, hipStream_t s, const double *lohi,
                           const Batch &bt) {
    k_set_electrodes<<<dim3((g.nr + 1 + 255) / 256, 1, bt.n), 256, 0, s>>>(g, u, lo, hi, lohi, bt);
}

void launch_set_wall(const Geom &g, double *u, double lo, double hi, hipStream_t s, const double *lohi,
                     const Batch &bt) {
    if (!g.wall) return;
    k_set_wall<<<dim3((g.nz + 1 + 255) / 256, 1, bt.n), 256, 0, s>>>(g, u, lo, hi, lohi, bt);
}

void launch_boundary_flow(const Geom &g, const double *V, const double *n, double q, double D, double *out,
                          hipStream_t s, const double *mun, const double *Dn, double sgn) {
    k_boundary_flow<<<1, 1024, 0, s>>>(g, V, n, q, D, out, mun, Dn, sgn);
}

void set_boundary(const Geom &g, double *V, double *ne, double *np, const mg_physics &ph, hipStream_t s) {
    launch_set_electrodes(g, V, ph.V_bottom, ph.V_top, s);
    launch_set_electrodes(g, ne, ph.ne_bottom, ph.ne_top, s);
    launch_set_electrodes(g, np, ph.np_bottom, ph.np_top, s);
    launch_set_wall(g, V, ph.V_bottom, ph.V_top, s);
    launch_set_wall(g, ne, 0.0, 0.0, s);
    launch_set_wall(g, np, 0.0, 0.0, s);
}

void launch_fill(double *p, int64_t n, double v, hipStream_t s, const Batch &bt) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    k_fill<double><<<dim3((unsigned)blocks, 1, bt.n), 256, 0, s>>>(p, n, v, bt);
}

void launch_fill(float *p, int64_t n, float v, hipStream_t s, const Batch &bt) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    k_fill<float><<<dim3((unsigned)blocks, 1, bt.n), 256, 0, s>>>(p, n, v, bt);
}

template <class T>
void launch_rbgs(const Geom &g, Op<T> op, T *x, int colour, hipStream_t s) {
    k_rbgs<T><<<grid2d(g), blk2d(g), 0, s>>>(g, op, x, colour);
}

template <class T>
void launch_zline(const Geom &g, Op<T> op, T *x, int parity, hipStream_t s) {
    int m = g.nz - 1;
    int lines = (g.nr - parity) / 2 + 1;
    if (lines <= 0) return;
    if (m <= 64)
        k_zline<T, 1><<<lines, 64, 0, s>>>(g, op, x, parity);
    else if (m <= 128)
        k_zline<T, 2><<<lines, 64, 0, s>>>(g, op, x, parity);
    else if (m <= 256)
        k_zline<T, 4><<<lines, 64, 0, s>>>(g, op, x, parity);
    else if (m <= 512)
        k_zline<T, 8><<<lines, 64, 0, s>>>(g, op, x, parity);
    else
        k_zline<T, 16><<<lines, 64, 0, s>>>(g, op, x, parity);
}

int residual_blocks(const Geom &g) {
    dim3 gr = grid2d(g);
    return (int)(gr.x * gr.y);
}

template <class TA, class TX, class TR>
void launch_residual(const Geom &g, Op<TA> op, const TX *fo, const TX *x, TR *r, double *partials,
                     int *nblocks_out, hipStream_t s) {
    dim3 gr = grid2d(g);
    if (nblocks_out) *nblocks_out = (int)(gr.x * gr.y);
    k_residual<TA, TX, TR><<<gr, blk2d(g), 0, s>>>(g, op, fo, x, r, partials);
}

template <class T>
void launch_restrict(const Geom &gf, const T *rf, const Geom &gc, T *fc, hipStream_t s) {
    k_restrict<T><<<grid2d(gc), blk2d(gc), 0, s>>>(gf, rf, gc, fc);
}

template <class T>
void launch_rb_sweep(const Geom &g, Op<T> op, const T *xin, T *xout, bool zin, const Geom *gc, const T *xc,
                     hipStream_t s) {
    const Geom &gcc = gc ? *gc : g;
    if (g.sh == 16) {
        dim3 grid((g.nz + 1 + kSWs - 1) / kSWs, (g.nr + 1 + 15) / 16);
        k_rb_sweep_s<T, 16><<<grid, dim3(kSWs, 16 + STile<16>::kSR), 0, s>>>(g, op, xin, xout, zin ? 1 : 0, gcc, xc);
    } else {
        dim3 grid((g.nz + 1 + kSWs - 1) / kSWs, (g.nr + 1 + 7) / 8);
        k_rb_sweep_s<T, 8><<<grid, dim3(kSWs, 8 + STile<8>::kSR), 0, s>>>(g, op, xin, xout, zin ? 1 : 0, gcc, xc);
    }
}

template <class T>
void launch_residual_restrict_s(const Geom &gf, Op<T> op, const T *x, const Geom &gc, T *fc, hipStream_t s) {
    dim3 grid((gc.nz + 1 + kCWs - 1) / kCWs, (gc.nr + 1 + kCHs - 1) / kCHs);
    k_residual_restrict_s<T><<<grid, dim3(64, 10), 0, s>>>(gf, op, x, gc, fc);
}

template <class T>
bool launch_subcycle_s(const FusedScalar<T> &F, hipStream_t s) {
    int64_t need = 0;
    for (int q = 0; q < F.n; ++q) need += 8 * (int64_t)(F.g[q].nr + 1) * (F.g[q].nz + 1);
    const Geom &gl = F.g[F.n - 1];
    if (need > kSubPoolS || (int64_t)(gl.nr + 1) * (gl.nz - 1) > kMaxCoarseUnknowns) return false;
    k_subcycle_s<T><<<1, 1024, 0, s>>>(F);
    return true;
}

template <class T>
void launch_prolong(const Geom &gf, T *xf, const Geom &gc, const T *xc, hipStream_t s) {
    k_prolong<T><<<grid2d(gf), blk2d(gf), 0, s>>>(gf, xf, gc, xc);
}

void launch_prolong_state(const Geom &gf, double *xf, const Geom &gc, const double *xc, hipStream_t s) {
    k_prolong_state<<<grid2d(gf), blk2d(gf), 0, s>>>(gf, xf, gc, xc);
}

void launch_coarse_factor(const Geom &g, Op<double> op, double *scratch, double *invT, float *invT32,
                          hipStream_t s) {
    int n = (g.nr + 1) * (g.nz - 1);
    if (n <= kLdsGJ)
        k_coarse_factor_lds<<<1, 1024, 0, s>>>(g, op, invT, invT32);
    else
        k_coarse_factor<<<1, 256, 0, s>>>(g, op, scratch, invT, invT32);
}

template <class T>
void launch_coarse_solve(const Geom &g, Op<T> op, const T *invT, T *x, hipStream_t s) {
    k_coarse_solve<T><<<1, 256, 0, s>>>(g, op, invT, x);
}

void launch_sum_partials(const double *partials, int nblocks, int ncomp, double *out, hipStream_t s,
                         const Batch &bt) {
    k_sum_partials<<<dim3(1, 1, bt.n), 256, 0, s>>>(partials, nblocks, ncomp, out, bt);
}

void launch_diff_norms(const Geom &g, const double *a, const double *b, double *partials,
                       int *nblocks_out, hipStream_t s, const Batch &bt) {
    dim3 gr = grid2d(g);
    if (nblocks_out) *nblocks_out = (int)(gr.x * gr.y);
    k_diff_norms<<<dim3(gr.x, gr.y, bt.n), blk2d(g), 0, s>>>(g, a, b, partials, bt);
}

void launch_copy_field(const Geom &g, const double *src, double *dst, hipStream_t s, const Batch &bt) {
    k_copy_field<<<dim3(grid2d(g).x, grid2d(g).y, bt.n), blk2d(g), 0, s>>>(g, src, dst, bt);
}

void launch_to_f32(const Geom &g, const double *src, float *dst, hipStream_t s) {
    k_to_f32<<<grid2d(g), blk2d(g), 0, s>>>(g, src, dst);
}

void launch_add_f32(const Geom &g, double *x, const float *e, hipStream_t s) {
    k_add_f32<<<grid2d(g), blk2d(g), 0, s>>>(g, x, e);
}

void launch_op_to_f32(const Geom &g, Op<double> op, Op<float> o32, hipStream_t s) {
    k_op_to_f32<<<grid2d(g), blk2d(g), 0, s>>>(g, op, o32);
}

template void launch_rbgs<double>(const Geom &, Op<double>, double *, int, hipStream_t);
template void launch_rbgs<float>(const Geom &, Op<float>, float *, int, hipStream_t);
template void launch_zline<double>(const Geom &, Op<double>, double *, int, hipStream_t);
template void launch_zline<float>(const Geom &, Op<float>, float *, int, hipStream_t);
template void launch_residual<double, double, double>(const Geom &, Op<double>, const double *,
                                                      const double *, double *, double *, int *,
                                                      hipStream_t);
template void launch_residual<double, double, float>(const Geom &, Op<double>, const double *,
                                                     const double *, float *, double *, int *,
                                                     hipStream_t);
template void launch_residual<float, float, float>(const Geom &, Op<float>, const float *, const float *,
                                                   float *, double *, int *, hipStream_t);
template void launch_restrict<double>(const Geom &, const double *, const Geom &, double *, hipStream_t);
template void launch_restrict<float>(const Geom &, const float *, const Geom &, float *, hipStream_t);
template void launch_prolong<double>(const Geom &, double *, const Geom &, const double *, hipStream_t);
template void launch_rb_sweep<double>(const Geom &, Op<double>, const double *, double *, bool, const Geom *,
                                      const double *, hipStream_t);
template void launch_rb_sweep<float>(const Geom &, Op<float>, const float *, float *, bool, const Geom *,
                                     const float *, hipStream_t);
template void launch_residual_restrict_s<double>(const Geom &, Op<double>, const double *, const Geom &, double *,
                                                 hipStream_t);
template void launch_residual_restrict_s<float>(const Geom &, Op<float>, const float *, const Geom &, float *,
                                                hipStream_t);
template bool launch_subcycle_s<double>(const FusedScalar<double> &, hipStream_t);
template bool launch_subcycle_s<float>(const FusedScalar<float> &, hipStream_t);
template void launch_prolong<float>(const Geom &, float *, const Geom &, const float *, hipStream_t);
template void launch_coarse_solve<double>(const Geom &, Op<double>, const double *, double *, hipStream_t);
template void launch_coarse_solve<float>(const Geom &, Op<float>, const float *, float *, hipStream_t);

}  // namespace mgf
