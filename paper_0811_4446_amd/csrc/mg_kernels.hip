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
// r = R has no outer face (zero radial flux).
// ---------------------------------------------------------------------------
__global__ void k_poisson_assemble(Geom g, Op<double> op, const double *__restrict__ ne,
                                   const double *__restrict__ np, double k, int charge) {
    int j = blockIdx.x * kTX + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > g.nr || j > g.nz) return;
    int64_t p = at(g, i, j);
    if (j == 0 || j == g.nz) {
        op.a[p] = op.b[p] = op.c[p] = op.d[p] = op.e[p] = op.f[p] = 0.0;
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
__global__ void k_sg_assemble(Geom g, Op<double> op, const double *__restrict__ V,
                              const double *__restrict__ nk, const double *__restrict__ S,
                              double q, double D, double dt_inv) {
    int j = blockIdx.x * kTX + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > g.nr || j > g.nz) return;
    int64_t p = at(g, i, j);
    if (j == 0 || j == g.nz) {
        op.a[p] = op.b[p] = op.c[p] = op.d[p] = op.e[p] = op.f[p] = 0.0;
        return;
    }
    double w = g.wr[i], dzc = g.dzc[j];
    double vol = w * dzc;
    double vc = V[p];
    double diag = vol * dt_inv;
    double ca = 0.0, cc = 0.0;
    if (i < g.nr) {
        double gg = g.fr[i] * dzc * D / g.dr;
        double al = q * (V[p + g.pitch] - vc);
        double F = bern_F(al);
        cc = -gg * F;
        diag += gg * bern_F(-al);
    }
    if (i > 0) {
        double gg = g.fr[i - 1] * dzc * D / g.dr;
        double al = q * (vc - V[p - g.pitch]);
        double F = bern_F(al);
        ca = -gg * bern_F(-al);
        diag += gg * F;
    }
    double ce, cd;
    {
        double gg = w * D / g.dz[j];
        double al = q * (V[p + 1] - vc);
        ce = -gg * bern_F(al);
        diag += gg * bern_F(-al);
    }
    {
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
template <class T>
__global__ void k_rbgs(Geom g, Op<T> op, T *__restrict__ x, int colour) {
    int j = blockIdx.x * kTX + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > g.nr || j < 1 || j >= g.nz) return;
    if (((i + j) & 1) != colour) return;
    int64_t p = at(g, i, j);
    T s = op.f[p] - op.d[p] * x[p - 1] - op.e[p] * x[p + 1];
    if (i > 0) s -= op.a[p] * x[p - g.pitch];
    if (i < g.nr) s -= op.c[p] * x[p + g.pitch];
    x[p] = s / op.b[p];
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
        double acc = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += 256) acc += part[b * ncomp + c];
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
__global__ void k_prolong(Geom gf, T *__restrict__ xf, Geom gc, const T *__restrict__ xc) {
    int j = blockIdx.x * kTX + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > gf.nr || j < 1 || j >= gf.nz) return;
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
    T v = (i & 1) ? T(0.5) * (v0 + v1) : v0;
    xf[at(gf, i, j)] += v;
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
__global__ __launch_bounds__(256) void k_coarse_factor_lds(Geom g, Op<double> op, double *__restrict__ invT,
                                                            float *__restrict__ invT32) {
    const int m = g.nz - 1;
    const int n = (g.nr + 1) * m;
    const int n2 = 2 * n;
    __shared__ double M[kLdsGJ * 2 * kLdsGJ];
    __shared__ double fcol[kLdsGJ];
    __shared__ int piv;
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
    for (int col = 0; col < n; ++col) {
        pivot_search_wave0(M, n2, col, n, &piv);
        __syncthreads();
        const int pv = piv;
        if (pv != col)
            for (int t = threadIdx.x; t < n2; t += blockDim.x) {
                double tmp = M[col * n2 + t];
                M[col * n2 + t] = M[pv * n2 + t];
                M[pv * n2 + t] = tmp;
            }
        __syncthreads();
        const double pinv = 1.0 / M[col * n2 + col];
        __syncthreads();
        for (int t = threadIdx.x; t < n2; t += blockDim.x) M[col * n2 + t] *= pinv;
        for (int rr = threadIdx.x; rr < n; rr += blockDim.x) fcol[rr] = M[rr * n2 + col];
        __syncthreads();
        for (int t = threadIdx.x; t < n * n2; t += blockDim.x) {
            int rr = t / n2, cc = t % n2;
            if (rr == col) continue;
            double fct = fcol[rr];
            if (fct != 0.0) M[rr * n2 + cc] -= fct * M[col * n2 + cc];
        }
        __syncthreads();
    }
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
                             double k, bool charge, hipStream_t s) {
    k_poisson_assemble<<<grid2d(g), blk2d(g), 0, s>>>(g, op, ne, np, k, charge ? 1 : 0);
}

void launch_sg_assemble(const Geom &g, Op<double> op, const double *V, const double *nk,
                        const double *S, double q, double D, double dt_inv, hipStream_t s) {
    k_sg_assemble<<<grid2d(g), blk2d(g), 0, s>>>(g, op, V, nk, S, q, D, dt_inv);
}

void launch_inject(const Geom &gf, const double *vf, const Geom &gc, double *vc, hipStream_t s) {
    k_inject<<<grid2d(gc), blk2d(gc), 0, s>>>(gf, vf, gc, vc);
}

void launch_set_electrodes(const Geom &g, double *u, double lo, double hi, hipStream_t s, const double *lohi,
                           const Batch &bt) {
    k_set_electrodes<<<dim3((g.nr + 1 + 255) / 256, 1, bt.n), 256, 0, s>>>(g, u, lo, hi, lohi, bt);
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
        k_coarse_factor_lds<<<1, 256, 0, s>>>(g, op, invT, invT32);
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
template void launch_prolong<float>(const Geom &, float *, const Geom &, const float *, hipStream_t);
template void launch_coarse_solve<double>(const Geom &, Op<double>, const double *, double *, hipStream_t);
template void launch_coarse_solve<float>(const Geom &, Op<float>, const float *, float *, hipStream_t);

}  // namespace mgf
