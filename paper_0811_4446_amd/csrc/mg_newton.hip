// Coupled Newton-Raphson path (Sec. 2, Eq. 14): the 3x3-block five-point
// Jacobian of the backward-Euler system in u = (n_e, n_p, V), its block
// multigrid (collective red-black Gauss-Seidel: the three unknowns of a
// node are relaxed together), and the BLAS-1 kernels of the FGMRES solver
// it preconditions.  FP64 throughout.
//
// Block coefficient planes (each (nr+1) x pitch, FV-integrated rows):
//   kind*5 + w   kind: 0 ee, 1 eV, 2 pp, 3 pV, 4 VV;  w: 0 a (i-1), 1 b
//                (centre), 2 c (i+1), 3 d (j-1), 4 e (j+1)
//   25 Ve, 26 Vp (centre couplings of the Poisson row to the densities)
//   27..29  right-hand side of the e, p and V rows
// A 3-field vector is three consecutive planes (n_e, n_p, V).
#include <math.h>

#include "mg_newton.h"

namespace mgf {

namespace {

constexpr int kTX = 64;

inline dim3 grid2d(const Geom &g) { return dim3((g.nz + 1 + kTX - 1) / kTX, (g.nr + 1 + g.ty - 1) / g.ty); }
inline dim3 blk2d(const Geom &g) { return dim3(kTX, g.ty); }
inline __device__ int64_t at(const Geom &g, int i, int j) { return (int64_t)i * g.pitch + j; }

inline __device__ double bF(double x) {
    if (fabs(x) < 1e-3) {
        double x2 = x * x;
        return 1.0 - 0.5 * x + x2 * (1.0 / 12.0) - x2 * x2 * (1.0 / 720.0);
    }
    return x / expm1(x);
}

// F'(x) = F(x) (1 - G(x)) / x with G(x) = F(-x); for |x| < 0.1 the Taylor
// series from the Bernoulli numbers (the closed form cancels there).
inline __device__ double bdF(double x) {
    if (fabs(x) < 0.1) {
        double x2 = x * x;
        return -0.5 + x * (1.0 / 6.0 + x2 * (-1.0 / 180.0 + x2 * (1.0 / 5040.0 +
                     x2 * (-1.0 / 151200.0 + x2 * (1.0 / 4790016.0)))));
    }
    return bF(x) * (1.0 - bF(-x)) / x;
}

struct Face {
    double nb_n, c_n;   // neighbour coefficient and centre contribution (density column)
    double nb_V, c_V;   // same for the potential column
};

// Face between the centre node and a neighbour.  `plus` = neighbour in +r/+z.
// q = -s mu/D, gd = area * D / distance.
inline __device__ Face sg_face(bool plus, double q, double gd, double Vc, double Vn, double nc, double nn) {
    Face f;
    if (plus) {  // outward flux gd (nc G(al) - nn F(al)), al = q (Vn - Vc)
        double al = q * (Vn - Vc);
        double F = bF(al), G = bF(-al), dF = bdF(al);
        f.nb_n = -gd * F;
        f.c_n = gd * G;
        double sl = gd * ((dF + 1.0) * nc - dF * nn);
        f.nb_V = q * sl;
        f.c_V = -q * sl;
    } else {     // outward flux gd (nc F(al) - nn G(al)), al = q (Vc - Vn)
        double al = q * (Vc - Vn);
        double F = bF(al), G = bF(-al), dF = bdF(al);
        f.nb_n = -gd * G;
        f.c_n = gd * F;
        double sl = gd * (dF * nc - (dF + 1.0) * nn);
        f.nb_V = -q * sl;
        f.c_V = q * sl;
    }
    return f;
}

// ---------------------------------------------------------------------------
// Jacobian (Eq. 14) and Newton right-hand side -F at the state (V, ne, np).
// Continuity rows: F = sum over faces area*phi_out + vol (n - n^k)/dt - vol S
// (Eqs. 7-11); Poisson row: F = A_P V - vol k (n_p - n_e) (Eqs. 12-13).
// ---------------------------------------------------------------------------
// One node (i, j) of a level's Jacobian and, with_rhs, of -F.  The state
// (V, ne, np) and the rhs inputs are read at sidx(i', j') for node (i', j')
// of this level: the level's own layout on the finest grid, and the finest
// grid's node (i' 2^l, j' 2^l) on level l (repeated injection).
template <class Ix>
inline __device__ void assemble_node(const Geom &g, const BOp &J, int i, int j, Ix sidx, const double *V,
                                     const double *ne, const double *np, const double *nek, const double *npk,
                                     const double *Se, const double *Sp, const NewtonPhys &ph, bool with_rhs,
                                     const NodeTransport &tr) {
    int64_t p = at(g, i, j);
    if (j == 0 || j == g.nz) {
        for (int k = 0; k < kBPlanes; ++k) J.pl(k)[p] = 0.0;
        return;
    }
    if (g.wall && i == g.nr) {
        // Dirichlet wall (Sec. 3): u = u_wall, identity block; the driver
        // keeps the state's wall row at u_wall, so -F = 0 there
        for (int k = 0; k < kBPlanes; ++k) J.pl(k)[p] = 0.0;
        J.pl(kEE + 1)[p] = 1.0;
        J.pl(kPP + 1)[p] = 1.0;
        J.pl(kVV + 1)[p] = 1.0;
        return;
    }
    int64_t s = sidx(i, j);
    double w = g.wr[i], dzc = g.dzc[j], vol = w * dzc;
    double Vc = V[s], ec = ne[s], pc = np[s];
    double ee[5] = {0, 0, 0, 0, 0}, eV[5] = {0, 0, 0, 0, 0}, pp[5] = {0, 0, 0, 0, 0}, pV[5] = {0, 0, 0, 0, 0},
           VV[5] = {0, 0, 0, 0, 0};
    int64_t nbp[5] = {sidx(i - 1, j), s, sidx(i + 1, j), sidx(i, j - 1), sidx(i, j + 1)};
    bool has[5] = {i > 0, false, i < g.nr, true, true};
    double geo[5];
    geo[0] = (i > 0) ? g.fr[i - 1] * dzc / g.dr : 0.0;
    geo[2] = (i < g.nr) ? g.fr[i] * dzc / g.dr : 0.0;
    geo[3] = w / g.dz[j - 1];
    geo[4] = w / g.dz[j];
#pragma unroll
    for (int d = 0; d < 5; ++d) {
        if (d == 1 || !has[d]) continue;
        bool plus = (d == 2 || d == 4);
        int64_t q = nbp[d];
        double Vn = V[q];
        // face transport: the constants, or the mean of the two nodes' values
        double qe = ph.qe, De = ph.De, qp = ph.qp, Dp = ph.Dp;
        if (tr.mue) {
            De = 0.5 * (tr.De[s] + tr.De[q]);
            qe = (0.5 * (tr.mue[s] + tr.mue[q])) / De;  // -s mu/D, s = -1
        }
        if (tr.mup) {
            Dp = 0.5 * (tr.Dp[s] + tr.Dp[q]);
            qp = -(0.5 * (tr.mup[s] + tr.mup[q])) / Dp;  // s = +1
        }
        Face fe = sg_face(plus, qe, geo[d] * De, Vc, Vn, ec, ne[q]);
        Face fp = sg_face(plus, qp, geo[d] * Dp, Vc, Vn, pc, np[q]);
        ee[d] = fe.nb_n;
        ee[1] += fe.c_n;
        eV[d] = fe.nb_V;
        eV[1] += fe.c_V;
        pp[d] = fp.nb_n;
        pp[1] += fp.c_n;
        pV[d] = fp.nb_V;
        pV[1] += fp.c_V;
        VV[d] = -geo[d];
        VV[1] += geo[d];
    }
    ee[1] += vol * ph.dt_inv;
    pp[1] += vol * ph.dt_inv;
#pragma unroll
    for (int d = 0; d < 5; ++d) {
        J.pl(kEE + d)[p] = ee[d];
        J.pl(kEV + d)[p] = eV[d];
        J.pl(kPP + d)[p] = pp[d];
        J.pl(kPV + d)[p] = pV[d];
        J.pl(kVV + d)[p] = VV[d];
    }
    double kv = vol * ph.k;
    J.pl(kVe)[p] = kv;
    J.pl(kVp)[p] = -kv;
    if (with_rhs) {
        double Fe = ee[1] * ec - vol * (Se[s] + nek[s] * ph.dt_inv);
        double Fp = pp[1] * pc - vol * (Sp[s] + npk[s] * ph.dt_inv);
        double FV = VV[1] * Vc - kv * (pc - ec);
#pragma unroll
        for (int d = 0; d < 5; ++d) {
            if (d == 1 || !has[d]) continue;
            int64_t q = nbp[d];
            Fe += ee[d] * ne[q];
            Fp += pp[d] * np[q];
            FV += VV[d] * V[q];
        }
        J.pl(kFe)[p] = -Fe;
        J.pl(kFp)[p] = -Fp;
        J.pl(kFV)[p] = -FV;
    } else {
        J.pl(kFe)[p] = 0.0;
        J.pl(kFp)[p] = 0.0;
        J.pl(kFV)[p] = 0.0;
    }
}

__global__ void k_newton_assemble(Geom g, BOp J, const double *__restrict__ V, const double *__restrict__ ne,
                                  const double *__restrict__ np, const double *__restrict__ nek,
                                  const double *__restrict__ npk, const double *__restrict__ Se,
                                  const double *__restrict__ Sp, NewtonPhys ph, int with_rhs,
                                  const NewtonPhys *__restrict__ php, Batch bt, NodeTransport tr) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    g = geom_off(g, bo_);
    J.base = boff(J.base, bo_);
    V = boff(V, bo_);
    ne = boff(ne, bo_);
    np = boff(np, bo_);
    nek = boff(nek, bo_);
    npk = boff(npk, bo_);
    Se = boff(Se, bo_);
    Sp = boff(Sp, bo_);
    if (php) ph = php[blockIdx.z];

    int j = blockIdx.x * kTX + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > g.nr || j > g.nz) return;
    const int64_t pitch = g.pitch;
    assemble_node(g, J, i, j, [pitch](int a, int b) { return (int64_t)a * pitch + b; }, V, ne, np, nek, npk, Se, Sp,
                  ph, with_rhs != 0, tr);
}

// Levels 1..n of the hierarchy in one launch: blockIdx.y ranges over the
// row blocks of every level in turn (LevTab::y0), and level l reads the
// finest state at (i 2^l, j 2^l), the node that repeated injection
// carries to its node (i, j).
__global__ __launch_bounds__(kTX *kLevTabTY) void k_newton_assemble_coarse(LevTab t, const double *__restrict__ V,
                                                                          const double *__restrict__ ne,
                                                                          const double *__restrict__ np,
                                                                          int64_t pitch0, NewtonPhys ph,
                                                                          const NewtonPhys *__restrict__ php,
                                                                          Batch bt, NodeTransport tr) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    int l = 0;
    while (l + 1 < t.n && (int)blockIdx.y >= t.y0[l + 1]) ++l;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    Geom g = geom_off(t.g[l], bo_);
    BOp J = t.J[l];
    J.base = boff(J.base, bo_);
    V = boff(V, bo_);
    ne = boff(ne, bo_);
    np = boff(np, bo_);
    if (php) ph = php[blockIdx.z];

    int j = blockIdx.x * kTX + threadIdx.x;
    int i = (blockIdx.y - t.y0[l]) * kLevTabTY + threadIdx.y;
    if (i > g.nr || j > g.nz) return;
    const int64_t si = pitch0 << t.shift[l], sj = int64_t(1) << t.shift[l];
    assemble_node(g, J, i, j, [si, sj](int a, int b) { return (int64_t)a * si + (int64_t)b * sj; }, V, ne, np,
                  nullptr, nullptr, nullptr, nullptr, ph, false, tr);
}

// The kernels whose results must agree bit for bit (one- and two-sweep
// launches, half-sweeps, the fused coarse sub-cycle, with or without the
// restriction in the smoothing launch) share the expressions below, with
// every product-sum written as an explicit fused multiply-add: the rounding
// then does not depend on how the compiler contracts each kernel's code.
template <class T>
__device__ inline T fmad(T a, T b, T c) {
    return fma(a, b, c);
}
// acc + wi (wdn r[-1] + r[0] + wup r[+1]): one fine row's share of the
// restriction (the transpose of the z-weighted bilinear prolongation).
template <class T>
__device__ inline T restrict_add(T acc, T wi, T wdn, T wup, T rm, T r0, T rp) {
    return fmad(wi, fmad(wup, rp, fmad(wdn, rm, r0)), acc);
}

// Sum over the four neighbours of B_nb x_nb for the three rows; coef(q)
// returns the node's Jacobian entry of plane q (from memory or from a row
// held in registers: one expression for both, so every kernel rounds the
// same way), xnb(t, c) field c of neighbour t (0: i-1, 1: i+1, 2: j-1,
// 3: j+1).
template <class T, class Coef, class XNb>
inline __device__ void nb_sum_gen(Coef coef, const bool (&has)[4], XNb xnb, T &se, T &sp, T &sv) {
    const int dirs[4] = {0, 2, 3, 4};
    se = sp = sv = T(0);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (!has[t]) continue;
        int d = dirs[t];
        T v = xnb(t, 2);
        se = fmad(coef(kEE + d), xnb(t, 0), fmad(coef(kEV + d), v, se));
        sp = fmad(coef(kPP + d), xnb(t, 1), fmad(coef(kPV + d), v, sp));
        sv = fmad(coef(kVV + d), v, sv);
    }
}
// Adds the centre block times the node's own values to the neighbour sums.
template <class T, class Coef>
inline __device__ void centre_add(Coef coef, T xe, T xp, T xv, T &se, T &sp, T &sv) {
    se = fmad(coef(kEE + 1), xe, fmad(coef(kEV + 1), xv, se));
    sp = fmad(coef(kPP + 1), xp, fmad(coef(kPV + 1), xv, sp));
    sv = fmad(coef(kVV + 1), xv, fmad(coef(kVe), xe, fmad(coef(kVp), xp, sv)));
}
template <class T, class XNb>
inline __device__ void nb_sum_of(const BOpT<T> &J, int64_t p, const bool (&has)[4], XNb xnb, T &se, T &sp, T &sv) {
    nb_sum_gen<T>([&](int q) { return J.pl(q)[p]; }, has, xnb, se, sp, sv);
}

template <class T>
inline __device__ void nb_sum(const Geom &g, const BOpT<T> &J, const T *x, int64_t plane, int i, int64_t p,
                              T &se, T &sp, T &sv) {
    const int64_t nbp[4] = {p - g.pitch, p + g.pitch, p - 1, p + 1};
    const bool has[4] = {i > 0, i < g.nr, true, true};
    nb_sum_of(J, p, has, [&](int t, int c) { return x[nbp[t] + c * plane]; }, se, sp, sv);
}

// x plus the bilinear prolongation (z-distance weights) of one coarse field
// c at fine node (i, j) of an unknown row.
template <class T>
inline __device__ T prolong_add(T x, const Geom &gf, const Geom &gc, const T *c, int i, int j) {
    int I0 = i >> 1, I1 = (i + 1) >> 1;
    T v0, v1;
    if ((j & 1) == 0) {
        v0 = c[at(gc, I0, j >> 1)];
        v1 = c[at(gc, I1, j >> 1)];
    } else {
        int J_ = j >> 1;
        T wl = gf.wl[J_], wu = T(1) - wl;
        v0 = fmad(wl, c[at(gc, I0, J_)], wu * c[at(gc, I0, J_ + 1)]);
        v1 = fmad(wl, c[at(gc, I1, J_)], wu * c[at(gc, I1, J_ + 1)]);
    }
    return (i & 1) ? fmad(T(0.5), v0 + v1, x) : x + v0;
}

template <class T>
inline __device__ void prolong3_node(const Geom &gf, T *xf, int64_t pf, const Geom &gc, const T *xc,
                                     int64_t pc, int i, int j) {
    int64_t p = at(gf, i, j);
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        xf[p + f * pf] = prolong_add(xf[p + f * pf], gf, gc, xc + f * pc, i, j);
    }
}

// The Jacobian row block and right-hand side of one node, held in registers.
template <class T>
struct NodeRow {
    T ee[5], eV[5], pp[5], pV[5], VV[5], Ve, Vp, fe, fp, fv;
    // centre-block factors that do not depend on the iterate: 1/ee, 1/pp,
    // the couplings scaled by them, and 1 / (Schur complement of the
    // potential), formed once per loaded row
    T ie, ip, a, b, is;
    // entry of Jacobian plane q (q a compile-time constant after unrolling)
    __device__ T coef(int q) const {
        return q < kEV ? ee[q] : q < kPP ? eV[q - kEV] : q < kPV ? pp[q - kPP] : q < kVV ? pV[q - kPV]
               : q < kVe ? VV[q - kVV] : q == kVe ? Ve : Vp;
    }
};
template <class T>
inline __device__ void load_row(const BOpT<T> &J, const T *f, int64_t p, NodeRow<T> &R) {
#pragma unroll
    for (int d = 0; d < 5; ++d) {
        R.ee[d] = J.pl(kEE + d)[p];
        R.eV[d] = J.pl(kEV + d)[p];
        R.pp[d] = J.pl(kPP + d)[p];
        R.pV[d] = J.pl(kPV + d)[p];
        R.VV[d] = J.pl(kVV + d)[p];
    }
    R.Ve = J.pl(kVe)[p];
    R.Vp = J.pl(kVp)[p];
    R.fe = f[p];
    R.fp = f[p + J.plane];
    R.fv = f[p + 2 * J.plane];
}
template <class T>
inline __device__ void factor_row(NodeRow<T> &R) {
    R.ie = T(1) / R.ee[1];
    R.ip = T(1) / R.pp[1];
    R.a = R.Ve * R.ie;
    R.b = R.Vp * R.ip;
    R.is = T(1) / fmad(-R.b, R.pV[1], fmad(-R.a, R.eV[1], R.VV[1]));
}
// Collective Gauss-Seidel update of one node: the neighbour sums of the
// three rows, then the 3x3 centre block [[ee,0,eV],[0,pp,pV],[Ve,Vp,VV]]
// solved exactly for (n_e, n_p, V), reduced to the potential first, with
// the factors of factor_row.
template <class T, class XNb>
inline __device__ void solve_row(const NodeRow<T> &R, const bool (&has)[4], XNb xnb, T &oe, T &op, T &ov) {
    T se, sp, sv;
    nb_sum_gen<T>([&](int q) { return R.coef(q); }, has, xnb, se, sp, sv);
    T re = R.fe - se, rp = R.fp - sp, rv = R.fv - sv;
    ov = fmad(-R.b, rp, fmad(-R.a, re, rv)) * R.is;
    oe = fmad(-R.eV[1], ov, re) * R.ie;
    op = fmad(-R.pV[1], ov, rp) * R.ip;
}

template <class T>
inline __device__ void block_gs_node(const Geom &g, const BOpT<T> &J, const T *f, T *x, int i, int j) {
    const int64_t p = at(g, i, j), plane = J.plane;
    NodeRow<T> R;
    load_row(J, f, p, R);
    factor_row(R);
    const int64_t nbp[4] = {p - g.pitch, p + g.pitch, p - 1, p + 1};
    const bool has[4] = {i > 0, i < g.nr, true, true};
    T oe, op, ov;
    solve_row(R, has, [&](int t, int c) { return x[nbp[t] + c * plane]; }, oe, op, ov);
    x[p] = oe;
    x[p + plane] = op;
    x[p + 2 * plane] = ov;
}

// Red-black half-sweep: every unknown node with (i+j)%2 == colour.  Nodes of
// one colour only read nodes of the other colour.
template <class T>
__global__ void k_block_rbgs(Geom g, BOpT<T> J, const T *__restrict__ f, T *__restrict__ x, int colour, Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    g = geom_off(g, bo_);
    J.base = boff(J.base, bo_);
    f = boff(f, bo_);
    x = boff(x, bo_);

    int j = blockIdx.x * kTX + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > g.nr || j < 1 || j >= g.nz || ((i + j) & 1) != colour) return;
    block_gs_node(g, J, f, x, i, j);
}

// Block zebra z-line half-sweep: every axial line i of parity `colour`
// (one thread per line) solves its 3x3-block tridiagonal system along z,
//   L_j x_{j-1} + C_j x_j + U_j x_{j+1} = f_j - (couplings to lines i -+ 1),
// with the other parity's current values, by block forward elimination and
// back substitution (block Thomas): P_j = D_j^-1 U_j and y_j = D_j^-1 (g_j -
// L_j y_{j-1}) with D_j = C_j - L_j P_{j-1} go to tmp (12 planes: P row-
// major, then y), then x_j = y_j - P_j x_{j+1}.  The electrode rows hold
// zero corrections, so the first and last unknowns have no outer coupling.
// The coefficients of node j+1 are loaded while node j is eliminated.
template <class T>
struct ZlRow {
    T c[kFe];     // Jacobian planes 0 .. kVp of the node
    T g[3];       // f minus the couplings to the neighbouring lines
};
template <class T>
inline __device__ void zl_load(const Geom &g, const BOpT<T> &J, const T *f, const T *x, int i, int j, ZlRow<T> &R) {
    const int64_t p = at(g, i, j), plane = J.plane;
#pragma unroll
    for (int q = 0; q < kFe; ++q) R.c[q] = J.pl(q)[p];
    T ge = f[p], gp = f[p + plane], gv = f[p + 2 * plane];
    const int dirs[2] = {0, 2};
    const bool has[2] = {i > 0, i < g.nr};
    const int64_t nb[2] = {p - g.pitch, p + g.pitch};
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        if (!has[t]) continue;
        const int d = dirs[t];
        const T xe = x[nb[t]], xp = x[nb[t] + plane], xv = x[nb[t] + 2 * plane];
        ge = fmad(-R.c[kEE + d], xe, fmad(-R.c[kEV + d], xv, ge));
        gp = fmad(-R.c[kPP + d], xp, fmad(-R.c[kPV + d], xv, gp));
        gv = fmad(-R.c[kVV + d], xv, gv);
    }
    R.g[0] = ge;
    R.g[1] = gp;
    R.g[2] = gv;
}
template <class T>
__global__ __launch_bounds__(64) void k_block_zline(Geom g, BOpT<T> J, const T *__restrict__ f, T *__restrict__ x,
                                                    T *__restrict__ tmp, int colour, Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    g = geom_off(g, bo_);
    J.base = boff(J.base, bo_);
    f = boff(f, bo_);
    x = boff(x, bo_);
    tmp = boff(tmp, bo_);
    const int i = 2 * (blockIdx.x * blockDim.x + threadIdx.x) + colour;
    if (i > g.nr) return;
    const int64_t plane = J.plane;
    const int n = g.nz - 1;  // unknowns j = 1 .. n
    T P[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, y[3] = {0, 0, 0};
    ZlRow<T> cur, nxt;
    zl_load(g, J, f, x, i, 1, cur);
    for (int j = 1; j <= n; ++j) {
        if (j < n) zl_load(g, J, f, x, i, j + 1, nxt);
        const T *c = cur.c;
        // D = C - L P_{j-1}, r = g - L y_{j-1}  (L = [[ee3,0,eV3],[0,pp3,pV3],[0,0,VV3]])
        T D[9] = {c[kEE + 1], T(0), c[kEV + 1], T(0), c[kPP + 1], c[kPV + 1], c[kVe], c[kVp], c[kVV + 1]};
        T r0 = cur.g[0], r1 = cur.g[1], r2 = cur.g[2];
        if (j > 1) {
            const T le = c[kEE + 3], lev = c[kEV + 3], lp = c[kPP + 3], lpv = c[kPV + 3], lv = c[kVV + 3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                D[k] = fmad(-le, P[k], fmad(-lev, P[6 + k], D[k]));
                D[3 + k] = fmad(-lp, P[3 + k], fmad(-lpv, P[6 + k], D[3 + k]));
                D[6 + k] = fmad(-lv, P[6 + k], D[6 + k]);
            }
            r0 = fmad(-le, y[0], fmad(-lev, y[2], r0));
            r1 = fmad(-lp, y[1], fmad(-lpv, y[2], r1));
            r2 = fmad(-lv, y[2], r2);
        }
        // D^-1 by the adjugate
        const T a00 = fmad(D[4], D[8], -D[5] * D[7]), a01 = fmad(D[2], D[7], -D[1] * D[8]),
                a02 = fmad(D[1], D[5], -D[2] * D[4]);
        const T a10 = fmad(D[5], D[6], -D[3] * D[8]), a11 = fmad(D[0], D[8], -D[2] * D[6]),
                a12 = fmad(D[2], D[3], -D[0] * D[5]);
        const T a20 = fmad(D[3], D[7], -D[4] * D[6]), a21 = fmad(D[1], D[6], -D[0] * D[7]),
                a22 = fmad(D[0], D[4], -D[1] * D[3]);
        const T id = T(1) / fmad(D[0], a00, fmad(D[1], a10, D[2] * a20));
        const T Di[9] = {a00 * id, a01 * id, a02 * id, a10 * id, a11 * id, a12 * id, a20 * id, a21 * id, a22 * id};
        // y_j = D^-1 r; P_j = D^-1 U (U = [[ee4,0,eV4],[0,pp4,pV4],[0,0,VV4]]; none for the last unknown)
#pragma unroll
        for (int k = 0; k < 3; ++k) y[k] = fmad(Di[3 * k], r0, fmad(Di[3 * k + 1], r1, Di[3 * k + 2] * r2));
        const bool last = j == n;
        const T ue = last ? T(0) : c[kEE + 4], uev = last ? T(0) : c[kEV + 4], up = last ? T(0) : c[kPP + 4],
                upv = last ? T(0) : c[kPV + 4], uv = last ? T(0) : c[kVV + 4];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            P[3 * k] = Di[3 * k] * ue;
            P[3 * k + 1] = Di[3 * k + 1] * up;
            P[3 * k + 2] = fmad(Di[3 * k], uev, fmad(Di[3 * k + 1], upv, Di[3 * k + 2] * uv));
        }
        const int64_t p = at(g, i, j);
#pragma unroll
        for (int k = 0; k < 9; ++k) tmp[p + k * plane] = P[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) tmp[p + (9 + k) * plane] = y[k];
        cur = nxt;
    }
    // back substitution from the last unknown (x_n = y_n, held in y)
    T xe = y[0], xp = y[1], xv = y[2];
    int64_t p = at(g, i, n);
    x[p] = xe;
    x[p + plane] = xp;
    x[p + 2 * plane] = xv;
    for (int j = n - 1; j >= 1; --j) {
        p = at(g, i, j);
        T Pj[9], yj[3];
#pragma unroll
        for (int k = 0; k < 9; ++k) Pj[k] = tmp[p + k * plane];
#pragma unroll
        for (int k = 0; k < 3; ++k) yj[k] = tmp[p + (9 + k) * plane];
        const T ne = fmad(-Pj[0], xe, fmad(-Pj[1], xp, fmad(-Pj[2], xv, yj[0])));
        const T np = fmad(-Pj[3], xe, fmad(-Pj[4], xp, fmad(-Pj[5], xv, yj[1])));
        const T nv = fmad(-Pj[6], xe, fmad(-Pj[7], xp, fmad(-Pj[8], xv, yj[2])));
        xe = ne;
        xp = np;
        xv = nv;
        x[p] = xe;
        x[p + plane] = xp;
        x[p + 2 * plane] = xv;
    }
}

// Tile of a sweep workgroup.  The hardware deals workgroups to the eight
// XCDs round-robin by linear index b (XCD = b mod 8); with g.xcd the tile of
// workgroup b is t = start(b mod 8) + b / 8, so every XCD works through one
// contiguous run of tiles in row-major order and neighbouring tiles, whose
// rings overlap, read each other's Jacobian lines from the same L2.  A
// permutation of the tiles: the arithmetic is unchanged.
__device__ inline void sweep_tile(const Geom &g, int &tx, int &ty) {
    if (!g.xcd) {
        tx = blockIdx.x;
        ty = blockIdx.y;
        return;
    }
    const int nx = gridDim.x, n = gridDim.x * gridDim.y;
    const int b = blockIdx.y * nx + blockIdx.x;
    const int k = b & 7, q = n >> 3, r = n & 7;
    const int t = k * q + (k < r ? k : r) + (b >> 3);
    tx = t % nx;
    ty = t / nx;
}

// One full collective red-black sweep (colour 0, then colour 1) from the
// input to xout (xin and xout distinct, electrode rows zero).  The input is
// xin, or zero (zin != 0, xin not read), or xin plus the bilinear
// prolongation of the coarse correction xc (xc != nullptr: the coarse-grid
// correction applied on the fly, never stored).
//
// A workgroup owns a kSW x kSH tile (z by r) and kSR more thread rows for
// the ring.  Phase 0 stages the input over the tile and a 2-node ring in LDS
// while every thread loads its node's Jacobian row block into registers
// (tile threads: their own node; ring threads: one colour-0 node of the
// 1-node ring, owned by a neighbouring workgroup).  Phase 1 updates the
// colour-0 nodes of tile and ring into LDS, phase 2 the tile's colour-1
// nodes.  Every value equals what two half-sweep launches compute, with one
// launch and one pass over the Jacobian; the ring costs (kSW + kSH) /
// (kSW kSH / 2) extra colour-0 updates.
constexpr int kSW = 32;
template <int SH>
struct SweepTile {
    static constexpr int kSH = SH;                                // tile rows
    static constexpr int kSR = (2 * kSW + 2 * SH + kSW - 1) / kSW;  // ring thread rows
};
template <class T, int SH>
__global__ __launch_bounds__(kSW *(SH + SweepTile<SH>::kSR)) void k_block_rb_sweep(
    Geom g, BOpT<T> J, const T *__restrict__ f, const T *__restrict__ xin, T *__restrict__ xout, int zin, Geom gc,
    const T *__restrict__ xc, int64_t pc, Batch bt) {
    constexpr int kSH = SH, kSR = SweepTile<SH>::kSR;
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    g = geom_off(g, bo_);
    J.base = boff(J.base, bo_);
    f = boff(f, bo_);
    xin = boff(xin, bo_);
    xout = boff(xout, bo_);
    if (xc) {
        gc = geom_off(gc, bo_);
        xc = boff(xc, bo_);
    }

    constexpr int W = kSW + 2, W2 = kSW + 4;
    __shared__ T lx[3][(kSH + 2) * W];
    __shared__ T lin[3][(kSH + 4) * W2];
    int tx, ty;
    sweep_tile(g, tx, ty);
    const int i0 = ty * kSH, j0 = tx * kSW;
    const int64_t plane = J.plane;
    const int ti = threadIdx.y, tj = threadIdx.x;
    const int tid = ti * kSW + tj;
    // the node this thread updates in phase 1 or 2
    int ni, nj;
    if (ti < kSH) {
        ni = i0 + ti;
        nj = j0 + tj;
    } else {
        const int k = (ti - kSH) * kSW + tj;
        if (k < kSW) {
            ni = i0 - 1;
            nj = j0 + k;
        } else if (k < 2 * kSW) {
            ni = i0 + kSH;
            nj = j0 + k - kSW;
        } else if (k < 2 * kSW + kSH) {
            ni = i0 + k - 2 * kSW;
            nj = j0 - 1;
        } else if (k < 2 * kSW + 2 * kSH) {
            ni = i0 + k - 2 * kSW - kSH;
            nj = j0 + kSW;
        } else {
            ni = -1;  // spare ring thread
            nj = 0;
        }
    }
    const bool valid = ni >= 0 && ni <= g.nr && nj >= 1 && nj < g.nz;
    const bool red = ((ni + nj) & 1) == 0;
    const bool tile = ti < kSH;
    const int64_t p = at(g, ni, nj);
    NodeRow<T> R;
    // the Jacobian row loads are issued before the window's, so that both
    // latencies overlap
    if (valid && (tile || red)) load_row(J, f, p, R);
    // phase 0: input over the window rows i0-2 .. i0+kSH+1, columns j0-2 .. j0+kSW+1
    for (int t = tid; t < (kSH + 4) * W2; t += kSW * (kSH + kSR)) {
        const int ii = i0 - 2 + t / W2, jj = j0 - 2 + t % W2;
        if (ii < 0 || ii > g.nr || jj < 0 || jj > g.nz) continue;
        const int64_t q = at(g, ii, jj);
        const bool un = jj >= 1 && jj < g.nz;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T v = zin ? T(0) : xin[q + c * plane];
            if (xc && un) v = prolong_add(v, g, gc, xc + c * pc, ii, jj);
            lin[c][t] = v;
        }
    }
    if (valid && (tile || red)) factor_row(R);
    __syncthreads();
    auto in_at = [&](int ii, int jj, int c) { return lin[c][(ii - i0 + 2) * W2 + (jj - j0 + 2)]; };
    const bool has[4] = {ni > 0, ni < g.nr, true, true};
    const int dni[4] = {-1, 1, 0, 0}, dnj[4] = {0, 0, -1, 1};
    if (valid && red) {
        T oe, op, ov;
        solve_row(R, has, [&](int t, int c) { return in_at(ni + dni[t], nj + dnj[t], c); }, oe, op, ov);
        const int l = (ni - i0 + 1) * W + (nj - j0 + 1);
        lx[0][l] = oe;
        lx[1][l] = op;
        lx[2][l] = ov;
        if (tile) {
            xout[p] = oe;
            xout[p + plane] = op;
            xout[p + 2 * plane] = ov;
        }
    }
    __syncthreads();
    if (!tile || !valid || red) return;
    // electrode neighbours (j - 1 == 0 or j + 1 == nz) are not updated: input value
    const bool fixed[4] = {false, false, nj - 1 == 0, nj + 1 == g.nz};
    T oe, op, ov;
    solve_row(R, has,
              [&](int t, int c) {
                  const int ii = ni + dni[t], jj = nj + dnj[t];
                  return fixed[t] ? in_at(ii, jj, c) : lx[c][(ii - i0 + 1) * W + (jj - j0 + 1)];
              },
              oe, op, ov);
    xout[p] = oe;
    xout[p + plane] = op;
    xout[p + 2 * plane] = ov;
}

// r = f - B x (apply == 0) or r = B x (apply == 1) at one node, 3 fields,
// 0 on the electrode rows.
template <class T>
inline __device__ void block_apply_node(const Geom &g, const BOpT<T> &J, const T *x, int i, int64_t p, T &se, T &sp,
                                        T &sv) {
    const int64_t plane = J.plane;
    nb_sum(g, J, x, plane, i, p, se, sp, sv);
    T xe = x[p], xp = x[p + plane], xv = x[p + 2 * plane];
    centre_add<T>([&](int q) { return J.pl(q)[p]; }, xe, xp, xv, se, sp, sv);
}

template <class T>
inline __device__ void block_residual_node(const Geom &g, const BOpT<T> &J, const T *f, const T *x,
                                           T *r, int apply, int i, int j) {
    int64_t p = at(g, i, j), plane = J.plane;
    if (j == 0 || j == g.nz) {
        r[p] = r[p + plane] = r[p + 2 * plane] = T(0);
        return;
    }
    T se, sp, sv;
    block_apply_node(g, J, x, i, p, se, sp, sv);
    if (apply) {
        r[p] = se;
        r[p + plane] = sp;
        r[p + 2 * plane] = sv;
    } else {
        r[p] = f[p] - se;
        r[p + plane] = f[p + plane] - sp;
        r[p + 2 * plane] = f[p + 2 * plane] - sv;
    }
}

// Two full collective red-black sweeps in one launch, xin -> xout (distinct
// buffers, electrode rows zero), input as for k_block_rb_sweep.  Each
// workgroup owns a kSW x SH tile T and keeps the window T+(4+E) (every node
// within 4+E rows / columns of T) in LDS, updated in place:
//   A: colour 0 on T+(3+E) (first sweep), B: colour 1 on T+(2+E),
//   C: colour 0 on T+(1+E) (second sweep), D: colour 1 on T+E,
// so each phase reads only values the previous phases made current.  Each
// thread holds the Jacobian rows of one colour-0 node of T+(3+E) and one
// colour-1 node of T+(2+E) in registers; the arithmetic of every update is
// that of the per-node block solve, so the result equals four half-sweeps
// bit for bit, with one launch and one pass over the Jacobian.
// With kRestrict (E = 2: the sweeps end current on T+2) the launch also
// forms the residual f - B x on T+1 from the rows in registers and restricts
// it to the coarse nodes (I, J) with (2I, 2J) in T (fc, coarse geometry gc,
// plane pc): bitwise what k_block_residual_restrict computes from xout.
// (Without it, gc / xc / pc are the optional prolongation-on-read input.)
template <int SH, bool kRestrict = false>
struct Sweep2Tile {
    static constexpr int kE = kRestrict ? 2 : 0;
    static constexpr int kR3 = SH + 2 * (3 + kE), kC3 = (kSW + 2 * (3 + kE)) / 2;  // colour-0 nodes of T+3+E
    static constexpr int kR2 = SH + 2 * (2 + kE), kC2 = (kSW + 2 * (2 + kE)) / 2;  // colour-1 nodes of T+2+E
    static constexpr int kN = (kR3 * kC3 > kR2 * kC2) ? kR3 * kC3 : kR2 * kC2;
    static constexpr int kThreads = (kN + 63) / 64 * 64;
    static constexpr int kWR = SH + 2 * (4 + kE), kWC = kSW + 2 * (4 + kE);  // window T+4+E
    static constexpr int kRR = kRestrict ? SH + 2 : 1, kRC = kRestrict ? kSW + 2 : 1;  // residual on T+1
};
template <class T, int SH, bool kRestrict>
__global__ __launch_bounds__((Sweep2Tile<SH, kRestrict>::kThreads)) void k_block_rb_sweep2(
    Geom g, BOpT<T> J, const T *__restrict__ f, const T *__restrict__ xin, T *__restrict__ xout, int zin, Geom gc,
    const T *__restrict__ xc, int64_t pc, T *__restrict__ fc, Batch bt) {
    using Tl = Sweep2Tile<SH, kRestrict>;
    constexpr int kWR = Tl::kWR, kWC = Tl::kWC, kE = Tl::kE, kM = 4 + kE;
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    g = geom_off(g, bo_);
    J.base = boff(J.base, bo_);
    f = boff(f, bo_);
    xin = boff(xin, bo_);
    xout = boff(xout, bo_);
    if (xc || kRestrict) gc = geom_off(gc, bo_);
    if (xc) xc = boff(xc, bo_);
    if (kRestrict) fc = boff(fc, bo_);

    __shared__ T w[3][kWR * kWC];
    __shared__ T lr[3][Tl::kRR * Tl::kRC];
    int tx, ty;
    sweep_tile(g, tx, ty);
    const int i0 = ty * SH, j0 = tx * kSW;
    const int64_t plane = J.plane;
    const int tid = threadIdx.x;
    // this thread's colour-0 node of T+3+E (a) and colour-1 node of T+2+E (b)
    int ai = -1, aj = 0, bi = -1, bj = 0;
    if (tid < Tl::kR3 * Tl::kC3) {
        const int r = tid / Tl::kC3, k = tid % Tl::kC3;
        ai = i0 - (3 + kE) + r;
        aj = j0 - (3 + kE) + 2 * k + ((i0 + j0 + r) & 1);
    }
    if (tid < Tl::kR2 * Tl::kC2) {
        const int r = tid / Tl::kC2, k = tid % Tl::kC2;
        bi = i0 - (2 + kE) + r;
        bj = j0 - (2 + kE) + 2 * k + ((i0 + j0 + r + 1) & 1);
    }
    const bool va = ai >= 0 && ai <= g.nr && aj >= 1 && aj < g.nz;
    const bool vb = bi >= 0 && bi <= g.nr && bj >= 1 && bj < g.nz;
    const int64_t pa = at(g, ai, aj), pb = at(g, bi, bj);
    NodeRow<T> Ra, Rb;
    if (va) load_row(J, f, pa, Ra);
    if (vb) load_row(J, f, pb, Rb);
    // (row loads first: the window loads below overlap their latency)
    for (int t = tid; t < kWR * kWC; t += Tl::kThreads) {
        const int ii = i0 - kM + t / kWC, jj = j0 - kM + t % kWC;
        if (ii < 0 || ii > g.nr || jj < 0 || jj > g.nz) continue;
        const int64_t q = at(g, ii, jj);
        const bool un = jj >= 1 && jj < g.nz;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            T v = zin ? T(0) : xin[q + c * plane];
            if (xc && un) v = prolong_add(v, g, gc, xc + c * pc, ii, jj);
            w[c][t] = v;
        }
    }
    if constexpr (kRestrict)
        for (int t = tid; t < Tl::kRR * Tl::kRC; t += Tl::kThreads) lr[0][t] = lr[1][t] = lr[2][t] = T(0);
    if (va) factor_row(Ra);
    if (vb) factor_row(Rb);
    const int dni[4] = {-1, 1, 0, 0}, dnj[4] = {0, 0, -1, 1};
    auto widx = [&](int ii, int jj) { return (ii - i0 + kM) * kWC + (jj - j0 + kM); };
    auto update = [&](const NodeRow<T> &R, int ni, int nj, bool write) {
        const bool has[4] = {ni > 0, ni < g.nr, true, true};
        T oe, op, ov;
        solve_row(R, has, [&](int t, int c) { return w[c][widx(ni + dni[t], nj + dnj[t])]; }, oe, op, ov);
        const int l = widx(ni, nj);
        w[0][l] = oe;
        w[1][l] = op;
        w[2][l] = ov;
        if (write) {
            const int64_t q = at(g, ni, nj);
            xout[q] = oe;
            xout[q + plane] = op;
            xout[q + 2 * plane] = ov;
        }
    };
    auto in_ring = [&](int ni, int nj, int d) {
        return ni >= i0 - d && ni < i0 + SH + d && nj >= j0 - d && nj < j0 + kSW + d;
    };
    __syncthreads();
    if (va) update(Ra, ai, aj, false);  // A
    __syncthreads();
    if (vb) update(Rb, bi, bj, false);  // B
    __syncthreads();
    if (va && in_ring(ai, aj, 1 + kE)) update(Ra, ai, aj, in_ring(ai, aj, 0));  // C
    __syncthreads();
    if (vb && in_ring(bi, bj, kE)) update(Rb, bi, bj, in_ring(bi, bj, 0));  // D
    if constexpr (kRestrict) {
        __syncthreads();
        // residual on T+1 (x current on T+2), the expressions of block_apply_node
        auto resid = [&](const NodeRow<T> &R, int ni, int nj) {
            const bool has[4] = {ni > 0, ni < g.nr, true, true};
            T se, sp, sv;
            nb_sum_gen<T>([&](int q) { return R.coef(q); }, has,
                          [&](int t, int c) { return w[c][widx(ni + dni[t], nj + dnj[t])]; }, se, sp, sv);
            const int l = widx(ni, nj);
            centre_add<T>([&](int q) { return R.coef(q); }, w[0][l], w[1][l], w[2][l], se, sp, sv);
            const int m = (ni - i0 + 1) * Tl::kRC + (nj - j0 + 1);
            lr[0][m] = R.fe - se;
            lr[1][m] = R.fp - sp;
            lr[2][m] = R.fv - sv;
        };
        if (va && in_ring(ai, aj, 1)) resid(Ra, ai, aj);
        if (vb && in_ring(bi, bj, 1)) resid(Rb, bi, bj);
        __syncthreads();
        // full weighting onto the coarse nodes of T, as k_block_residual_restrict
        constexpr int kCI = SH / 2, kCJ = kSW / 2;
        for (int t = tid; t < kCI * kCJ; t += Tl::kThreads) {
            const int I = i0 / 2 + t / kCJ, J_ = j0 / 2 + t % kCJ;
            if (I > gc.nr || J_ > gc.nz) continue;
            const int64_t q = at(gc, I, J_);
            if (J_ == 0 || J_ == gc.nz) {
                fc[q] = fc[q + pc] = fc[q + 2 * pc] = T(0);
                continue;
            }
            T wdn = T(1) - g.wl[J_ - 1], wup = g.wl[J_];
            T acc[3] = {0, 0, 0};
            for (int di = -1; di <= 1; ++di) {
                int i = 2 * I + di;
                if (i < 0 || i > g.nr) continue;
                T wi = (di == 0) ? T(1) : T(0.5);
                const int l = (i - i0 + 1) * Tl::kRC + (2 * J_ - j0 + 1);
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    acc[c] = restrict_add(acc[c], wi, wdn, wup, lr[c][l - 1], lr[c][l], lr[c][l + 1]);
            }
            fc[q] = acc[0];
            fc[q + pc] = acc[1];
            fc[q + 2 * pc] = acc[2];
        }
    }
}

template <class T>
__global__ void k_block_residual(Geom g, BOpT<T> J, const T *__restrict__ f, const T *__restrict__ x,
                                 T *__restrict__ r, int apply, Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    g = geom_off(g, bo_);
    J.base = boff(J.base, bo_);
    f = boff(f, bo_);
    x = boff(x, bo_);
    r = boff(r, bo_);

    int j = blockIdx.x * kTX + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > g.nr || j > g.nz) return;
    block_residual_node(g, J, f, x, r, apply, i, j);
}

// Three-field restriction (P^T of the bilinear prolongation), same weights
// as the scalar path, at coarse node (I, J_).
template <class T>
inline __device__ void restrict3_node(const Geom &gf, const T *rf, int64_t pf, const Geom &gc, T *fc,
                                      int64_t pc, int I, int J_) {
    int64_t q = at(gc, I, J_);
    if (J_ == 0 || J_ == gc.nz) {
        fc[q] = fc[q + pc] = fc[q + 2 * pc] = T(0);
        return;
    }
    T wdn = T(1) - gf.wl[J_ - 1], wup = gf.wl[J_];
    T acc[3] = {0, 0, 0};
    for (int di = -1; di <= 1; ++di) {
        int i = 2 * I + di;
        if (i < 0 || i > gf.nr) continue;
        T wi = (di == 0) ? T(1) : T(0.5);
        int64_t p = at(gf, i, 2 * J_);
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const T *r = rf + f * pf;
            acc[f] = restrict_add(acc[f], wi, wdn, wup, r[p - 1], r[p], r[p + 1]);
        }
    }
    fc[q] = acc[0];
    fc[q + pc] = acc[1];
    fc[q + 2 * pc] = acc[2];
}

template <class T>
__global__ void k_restrict3(Geom gf, const T *__restrict__ rf, int64_t pf, Geom gc, T *__restrict__ fc,
                            int64_t pc, Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    gf = geom_off(gf, bo_);
    gc = geom_off(gc, bo_);
    rf = boff(rf, bo_);
    fc = boff(fc, bo_);

    int J_ = blockIdx.x * kTX + threadIdx.x;
    int I = blockIdx.y * blockDim.y + threadIdx.y;
    if (I > gc.nr || J_ > gc.nz) return;
    restrict3_node(gf, rf, pf, gc, fc, pc, I, J_);
}

// Residual and restriction in one launch: a workgroup owns a kCW x kCH
// tile of coarse nodes, forms the fine residual r = f - B x over the fine
// window those nodes restrict from (2 kCH + 1 rows, 2 kCW + 1 columns) in
// LDS, then restricts it.  Bitwise the values of k_block_residual followed
// by k_restrict3; the fine residual itself is not stored.
constexpr int kCW = 32, kCH = 4;  // fine window 9 x 65: one node per thread of a 64 x 10 workgroup
static_assert((2 * kCW + 1) * (2 * kCH + 1) <= 64 * 10, "one fine node per thread");
template <class T>
__global__ __launch_bounds__(1024) void k_block_residual_restrict(Geom gf, BOpT<T> J, const T *__restrict__ f,
                                                                  const T *__restrict__ x, Geom gc,
                                                                  T *__restrict__ fc, int64_t pc, Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    gf = geom_off(gf, bo_);
    gc = geom_off(gc, bo_);
    J.base = boff(J.base, bo_);
    f = boff(f, bo_);
    x = boff(x, bo_);
    fc = boff(fc, bo_);

    constexpr int FW = 2 * kCW + 1, FH = 2 * kCH + 1;
    __shared__ T lr[3][FH * FW];
    const int I0 = blockIdx.y * kCH, J0 = blockIdx.x * kCW;
    const int fi0 = 2 * I0 - 1, fj0 = 2 * J0 - 1;
    const int tid = threadIdx.y * blockDim.x + threadIdx.x, nth = blockDim.x * blockDim.y;
    for (int t = tid; t < FH * FW; t += nth) {
        const int i = fi0 + t / FW, j = fj0 + t % FW;
        if (i < 0 || i > gf.nr || j < 0 || j > gf.nz) continue;
        if (j == 0 || j == gf.nz) {
            lr[0][t] = lr[1][t] = lr[2][t] = T(0);
            continue;
        }
        const int64_t p = at(gf, i, j);
        T se, sp, sv;
        block_apply_node(gf, J, x, i, p, se, sp, sv);
        lr[0][t] = f[p] - se;
        lr[1][t] = f[p + J.plane] - sp;
        lr[2][t] = f[p + 2 * J.plane] - sv;
    }
    __syncthreads();
    if (tid >= kCW * kCH) return;
    const int I = I0 + tid / kCW, J_ = J0 + tid % kCW;
    if (I > gc.nr || J_ > gc.nz) return;
    const int64_t q = at(gc, I, J_);
    if (J_ == 0 || J_ == gc.nz) {
        fc[q] = fc[q + pc] = fc[q + 2 * pc] = T(0);
        return;
    }
    T wdn = T(1) - gf.wl[J_ - 1], wup = gf.wl[J_];
    T acc[3] = {0, 0, 0};
    for (int di = -1; di <= 1; ++di) {
        int i = 2 * I + di;
        if (i < 0 || i > gf.nr) continue;
        T wi = (di == 0) ? T(1) : T(0.5);
        const int l = (i - fi0) * FW + (2 * J_ - fj0);
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] = restrict_add(acc[c], wi, wdn, wup, lr[c][l - 1], lr[c][l], lr[c][l + 1]);
    }
    fc[q] = acc[0];
    fc[q + pc] = acc[1];
    fc[q + 2 * pc] = acc[2];
}

// x += P xc on the unknown rows (bilinear, z-distance weights).
template <class T>
__global__ void k_prolong3(Geom gf, T *__restrict__ xf, int64_t pf, Geom gc, const T *__restrict__ xc,
                           int64_t pc, Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    gf = geom_off(gf, bo_);
    gc = geom_off(gc, bo_);
    xf = boff(xf, bo_);
    xc = boff(xc, bo_);

    int j = blockIdx.x * kTX + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > gf.nr || j < 1 || j >= gf.nz) return;
    prolong3_node(gf, xf, pf, gc, xc, pc, i, j);
}

// Coarsest grid: explicit inverse of the dense block matrix (Gauss-Jordan,
// partial pivoting, one workgroup); unknown (i, j, field) has index
// 3*(i*(nz-1) + j-1) + field.  Stored transposed.
__global__ __launch_bounds__(1024) void k_block_coarse_factor(Geom g, BOp J, double *__restrict__ M,
                                                              double *__restrict__ invT, Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    g = geom_off(g, bo_);
    J.base = boff(J.base, bo_);
    M = boff(M, bo_);
    invT = boff(invT, bo_);

    const int m = g.nz - 1;
    const int n = 3 * (g.nr + 1) * m;
    const int n2 = 2 * n;
    for (int64_t t = threadIdx.x; t < (int64_t)n * n2; t += blockDim.x) M[t] = 0.0;
    __syncthreads();
    for (int node = threadIdx.x; node < (g.nr + 1) * m; node += blockDim.x) {
        int i = node / m, j = node % m + 1;
        int64_t p = at(g, i, j);
        int rowb = 3 * node;
        int nbnode[5] = {node - m, node, node + m, node - 1, node + 1};
        bool has[5] = {i > 0, true, i < g.nr, j > 1, j < m};
        for (int d = 0; d < 5; ++d) {
            if (!has[d]) continue;
            int colb = 3 * nbnode[d];
            M[(int64_t)(rowb + 0) * n2 + colb + 0] = J.pl(kEE + d)[p];
            M[(int64_t)(rowb + 0) * n2 + colb + 2] = J.pl(kEV + d)[p];
            M[(int64_t)(rowb + 1) * n2 + colb + 1] = J.pl(kPP + d)[p];
            M[(int64_t)(rowb + 1) * n2 + colb + 2] = J.pl(kPV + d)[p];
            M[(int64_t)(rowb + 2) * n2 + colb + 2] = J.pl(kVV + d)[p];
        }
        M[(int64_t)(rowb + 2) * n2 + rowb + 0] = J.pl(kVe)[p];
        M[(int64_t)(rowb + 2) * n2 + rowb + 1] = J.pl(kVp)[p];
        for (int f = 0; f < 3; ++f) M[(int64_t)(rowb + f) * n2 + n + rowb + f] = 1.0;
    }
    __syncthreads();
    __shared__ int piv;
    __shared__ double fcol[3 * kMaxCoarseUnknowns];
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
        for (int64_t t = threadIdx.x; t < (int64_t)n * n2; t += blockDim.x) {
            int rr = (int)(t / n2), cc = (int)(t % n2);
            if (rr == col) continue;
            double fct = fcol[rr];
            if (fct != 0.0) M[(int64_t)rr * n2 + cc] -= fct * M[(int64_t)col * n2 + cc];
        }
        __syncthreads();
    }
    for (int64_t t = threadIdx.x; t < (int64_t)n * n; t += blockDim.x) {
        int row = (int)(t / n), k = (int)(t % n);
        invT[(int64_t)k * n + row] = M[(int64_t)row * n2 + n + k];
    }
}

// Same factorisation with the augmented matrix resident in LDS (n <= 63).
constexpr int kLdsGJ = 63;
constexpr int kFactorThreads = 1024;  // workgroup of the LDS Gauss-Jordan factorisation
__global__ __launch_bounds__(kFactorThreads) void k_block_coarse_factor_lds(Geom g, BOp J, double *__restrict__ invT,
                                                                  Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    g = geom_off(g, bo_);
    J.base = boff(J.base, bo_);
    invT = boff(invT, bo_);

    const int m = g.nz - 1;
    const int n = 3 * (g.nr + 1) * m;
    const int n2 = 2 * n;
    // two copies of the augmented matrix: column step k reads one, writes the other
    __shared__ double Mb[2][kLdsGJ * 2 * kLdsGJ];
    double *M = Mb[0];
    for (int t = threadIdx.x; t < n * n2; t += blockDim.x) M[t] = 0.0;
    __syncthreads();
    for (int node = threadIdx.x; node < (g.nr + 1) * m; node += blockDim.x) {
        int i = node / m, j = node % m + 1;
        int64_t p = at(g, i, j);
        int rowb = 3 * node;
        int nbnode[5] = {node - m, node, node + m, node - 1, node + 1};
        bool has[5] = {i > 0, true, i < g.nr, j > 1, j < m};
        for (int d = 0; d < 5; ++d) {
            if (!has[d]) continue;
            int colb = 3 * nbnode[d];
            M[(rowb + 0) * n2 + colb + 0] = J.pl(kEE + d)[p];
            M[(rowb + 0) * n2 + colb + 2] = J.pl(kEV + d)[p];
            M[(rowb + 1) * n2 + colb + 1] = J.pl(kPP + d)[p];
            M[(rowb + 1) * n2 + colb + 2] = J.pl(kPV + d)[p];
            M[(rowb + 2) * n2 + colb + 2] = J.pl(kVV + d)[p];
        }
        M[(rowb + 2) * n2 + rowb + 0] = J.pl(kVe)[p];
        M[(rowb + 2) * n2 + rowb + 1] = J.pl(kVp)[p];
        for (int f = 0; f < 3; ++f) M[(rowb + f) * n2 + n + rowb + f] = 1.0;
    }
    __syncthreads();
    // Gauss-Jordan with partial pivoting, one barrier per column: every
    // element of the next copy in one pass (scaled pivot row, exchanged row,
    // other rows eliminated against the scaled pivot row), each thread's
    // elements loaded before any is stored; meanwhile wavefront 0 forms the
    // next column's new values in its lanes (one row each, n <= 64) and finds
    // that column's pivot (largest magnitude, first row on ties) from them,
    // so no separate search phase follows.  The pivot indices alternate
    // between two slots.
    __shared__ int pivs[2];
    pivot_search_wave0(Mb[0], n2, 0, n, &pivs[0]);
    __syncthreads();
    // element (rr, cc) of the next copy, the same expression on both paths
    auto gj_elem = [&](const double *A, int rr, int cc, int col, int pv, double pinv, double fpv) {
        const double prc = A[pv * n2 + cc] * pinv;
        if (rr == col) return prc;
        const double src = (rr == pv) ? A[col * n2 + cc] : A[rr * n2 + cc];
        const double fct = (rr == pv) ? fpv : A[rr * n2 + col];
        return (fct != 0.0) ? fmad(-fct, prc, src) : src;
    };
    constexpr int kPer = (kLdsGJ * 2 * kLdsGJ + kFactorThreads - 1) / kFactorThreads;
    const int total = n * n2;
    int cur = 0;
    for (int col = 0; col < n; ++col) {
        const double *A = Mb[cur];
        double *B = Mb[cur ^ 1];
        const int pv = pivs[col & 1];
        const double pinv = 1.0 / A[pv * n2 + col];
        const double fpv = A[col * n2 + col];
        double v[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int t = threadIdx.x + k * kFactorThreads;
            if (t >= total) break;
            const int rr = t / n2, cc = t - rr * n2;
            v[k] = gj_elem(A, rr, cc, col, pv, pinv, fpv);
        }
        if (threadIdx.x < 64 && col + 1 < n) {
            const int r = threadIdx.x;
            int best = n;
            double bv = -1.0;
            if (r > col && r < n) {
                bv = fabs(gj_elem(A, r, col + 1, col, pv, pinv, fpv));
                best = r;
            }
            for (int off = 32; off >= 1; off >>= 1) {
                const double ov = __shfl_xor(bv, off);
                const int ob = __shfl_xor(best, off);
                if (ov > bv || (ov == bv && ob < best)) {
                    bv = ov;
                    best = ob;
                }
            }
            if (r == 0) pivs[(col + 1) & 1] = best < n ? best : col + 1;
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const int t = threadIdx.x + k * kFactorThreads;
            if (t >= total) break;
            B[t] = v[k];
        }
        __syncthreads();
        cur ^= 1;
    }
    M = Mb[cur];
    for (int t = threadIdx.x; t < n * n; t += blockDim.x) {
        int row = t / n, k = t % n;
        invT[(int64_t)k * n + row] = M[row * n2 + n + k];
    }
}

// x = A^{-1} f on the coarsest grid by one workgroup of 1024 threads (rhs
// staged in `rhs`, at least 3 * nodes values of LDS; `red` 16 x 64 values of
// LDS).  Rows go in blocks of 64, one per lane; the 16 wavefronts split the
// columns (wavefront w takes k = w, w + 16, ...) and the partial sums are
// added in wavefront order.  use_pre (n <= 64 only): pre holds this thread's
// matrix entries, k = w + 16 u for u < kCsPre, already loaded.
constexpr int kCsParts = 16;
constexpr int kCsPre = 4;  // kCsParts * kCsPre >= 64
template <class T>
inline __device__ void block_coarse_solve_wg(const Geom &g, int64_t plane, const T *f, const T *invT, T *x, T *rhs,
                                             T (*red)[64], bool use_pre, const T (&pre)[kCsPre]) {
    const int m = g.nz - 1;
    const int nn = (g.nr + 1) * m;
    const int n = 3 * nn;
    for (int node = threadIdx.x; node < nn; node += blockDim.x) {
        int i = node / m, j = node % m + 1;
        int64_t p = at(g, i, j);
        rhs[3 * node + 0] = f[p];
        rhs[3 * node + 1] = f[p + plane];
        rhs[3 * node + 2] = f[p + 2 * plane];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, part = threadIdx.x >> 6;
    for (int rb = 0; rb < n; rb += 64) {
        const int row = rb + lane;
        T acc = T(0);
        if (row < n) {
            if (use_pre) {
#pragma unroll
                for (int u = 0; u < kCsPre; ++u) {
                    const int k = part + kCsParts * u;
                    if (k < n) acc += pre[u] * rhs[k];
                }
            } else {
                for (int k = part; k < n; k += kCsParts) acc += invT[(int64_t)k * n + row] * rhs[k];
            }
        }
        red[part][lane] = acc;
        __syncthreads();
        if (threadIdx.x < 64 && row < n) {
            T sum = T(0);
            for (int q = 0; q < kCsParts; ++q) sum += red[q][lane];
            const int node = row / 3, fl = row % 3;
            const int i = node / m, j = node % m + 1;
            x[at(g, i, j) + fl * plane] = sum;
        }
        __syncthreads();
    }
}

template <class T>
__global__ __launch_bounds__(1024) void k_block_coarse_solve(Geom g, BOpT<T> J, const T *__restrict__ f,
                                                             const T *__restrict__ invT,
                                                             T *__restrict__ x, Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    g = geom_off(g, bo_);
    J.base = boff(J.base, bo_);
    f = boff(f, bo_);
    invT = boff(invT, bo_);
    x = boff(x, bo_);

    __shared__ T rhs[3 * kMaxCoarseUnknowns];
    __shared__ T red[kCsParts][64];
    const T none[kCsPre] = {};
    block_coarse_solve_wg(g, J.plane, f, invT, x, rhs, red, false, none);
}

// ---------------------------------------------------------------------------
// The coarse end of the block V-cycle in one workgroup: levels 0..n-1 of
// `F` (the last is the coarsest) are small enough that per-level launches
// would cost more than the work, so one workgroup runs their smoothing,
// residual, restriction, coarse solve and prolongation with barriers in
// between, node by node exactly as the per-level kernels do.
// ---------------------------------------------------------------------------
// Where the sub-cycle keeps its levels.  Global: the levels' own workspace.
// LDS: every level's Jacobian planes, correction and residual, and the top
// level's right-hand side, copied into LDS in a compact layout (pitch nz+1)
// when they fit, so that the barrier phases read no global memory; the top
// level's correction is written back at the end.
constexpr int kSubPool = 15360;  // LDS elements of the staged levels
constexpr int kStaged = kFe;     // matrix planes 0 .. kFe-1 (the rhs planes kFe.. come last)
static_assert(kFe == kBPlanes - 3, "the three rhs planes are the last ones");
template <class T, bool kLds>
struct SubMem;
template <class T>
struct SubMem<T, false> {
    const FusedLevelsT<T> &F;
    int64_t bo;
    __device__ Geom geom(int q) const { return geom_off(F.g[q], bo); }
    __device__ BOpT<T> jac(int q) const { return BOpT<T>{boff(F.J[q], bo), F.plane[q]}; }
    __device__ T *x(int q) const { return boff(F.x[q], bo); }
    __device__ T *r(int q) const { return boff(F.r[q], bo); }
    __device__ const T *f0() const { return boff(F.f0, bo); }
    __device__ int64_t xplane(int q) const { return F.plane[q]; }
};
template <class T>
struct SubMem<T, true> {
    const FusedLevelsT<T> &F;
    int64_t bo;
    T *pool;
    __device__ int nodes(int q) const { return (F.g[q].nr + 1) * (F.g[q].nz + 1); }
    __device__ int off(int q) const {
        int o = 0;
        for (int t = 0; t < q; ++t) o += (kBPlanes + 6) * nodes(t);
        return o;
    }
    __device__ Geom geom(int q) const {
        Geom g = geom_off(F.g[q], bo);
        g.pitch = g.nz + 1;
        return g;
    }
    __device__ BOpT<T> jac(int q) const { return BOpT<T>{pool + off(q), nodes(q)}; }
    __device__ T *x(int q) const { return pool + off(q) + kBPlanes * nodes(q); }
    __device__ T *r(int q) const { return pool + off(q) + (kBPlanes + 3) * nodes(q); }
    __device__ const T *f0() const { return pool + off(F.n); }
    __device__ int64_t xplane(int q) const { return nodes(q); }
    // Compact copies of every level's Jacobian planes and of the top level's
    // right-hand side into LDS, and zero corrections on every level.  Segment
    // q < n is level q's kStaged matrix planes (a level's right-hand-side
    // planes are written by the restriction before they are read, and the
    // top level uses f0), segment n the 3 planes of f0; value e of a segment
    // is row R = e / (nz + 1) (R = plane * (nr + 1) + i, which starts R *
    // pitch values into the array since planes are (nr + 1) * pitch apart),
    // column e % (nz + 1).  Each segment gets its own run of ceil(size / kB)
    // consecutive threads (at most 969 for a full pool), each of which loads
    // at most kB values of it, so every load of the staging is issued before
    // the first store waits.
    __device__ void stage_all() const {
        const int n = F.n;
        constexpr int kB = 16;
        static_assert(kSubPool / kB + kMaxFused + 1 <= 1024, "one run of threads per segment");
        int q = -1, first = 0, cnt = 0;
        for (int t = 0, start = 0; t <= n; ++t) {
            const int c = ((t < n ? kStaged : 3) * nodes(t < n ? t : 0) + kB - 1) / kB;
            if (q < 0 && (int)threadIdx.x < start + c) {
                q = t;
                first = start;
                cnt = c;
            }
            start += c;
        }
        if (q >= 0) {
            const int qq = q < n ? q : 0;
            const int w = F.g[qq].nz + 1, size = (q < n ? kStaged : 3) * (F.g[qq].nr + 1) * w;
            const uint32_t mg = F.wmagic[qq];
            const int64_t pitch = F.g[qq].pitch;
            const T *src = boff(q < n ? F.J[q] : F.f0, bo);
            T *dst = pool + (q < n ? off(q) : off(n));
            const int lt = threadIdx.x - first;
            T v[kB];
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                const int e = lt + u * cnt;
                if (e < size) {
                    const int R = (int)__umulhi((uint32_t)e, mg);
                    v[u] = src[(int64_t)R * pitch + (e - R * w)];
                }
            }
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                const int e = lt + u * cnt;
                if (e < size) dst[e] = v[u];
            }
        }
        for (int q = 0; q < n; ++q) {
            T *xq = x(q);
            for (int t = threadIdx.x; t < 3 * nodes(q); t += blockDim.x) xq[t] = T(0);
        }
    }
};

// nsweeps collective red-black sweeps of one level inside the sub-cycle's
// workgroup.  When every node of the level has a thread of its own, that
// thread loads its Jacobian row and factors once and keeps them in
// registers over all the half-sweeps (the arithmetic of block_gs_node);
// otherwise block_gs_node per node and half-sweep.
template <class T>
inline __device__ void subcycle_smooth(const Geom &g, const BOpT<T> &J, const T *f, T *x, int nsweeps) {
    const int nodes = (g.nr + 1) * (g.nz + 1), nt = blockDim.x;
    if (nodes <= nt) {
        const int t = threadIdx.x, i = t / (g.nz + 1), j = t % (g.nz + 1);
        const bool mine = t < nodes && j >= 1 && j < g.nz;
        const int64_t p = mine ? at(g, i, j) : 0, plane = J.plane;
        NodeRow<T> R;
        if (mine) {
            load_row(J, f, p, R);
            factor_row(R);
        }
        const int64_t nbp[4] = {p - g.pitch, p + g.pitch, p - 1, p + 1};
        const bool has[4] = {i > 0, i < g.nr, true, true};
        for (int s = 0; s < nsweeps; ++s)
            for (int col = 0; col < 2; ++col) {
                if (mine && ((i + j) & 1) == col) {
                    T oe, op, ov;
                    solve_row(R, has, [&](int k, int c) { return x[nbp[k] + c * plane]; }, oe, op, ov);
                    x[p] = oe;
                    x[p + plane] = op;
                    x[p + 2 * plane] = ov;
                }
                __syncthreads();
            }
        return;
    }
    for (int s = 0; s < nsweeps; ++s)
        for (int col = 0; col < 2; ++col) {
            for (int t = threadIdx.x; t < nodes; t += nt) {
                const int i = t / (g.nz + 1), j = t % (g.nz + 1);
                if (j >= 1 && j < g.nz && ((i + j) & 1) == col) block_gs_node(g, J, f, x, i, j);
            }
            __syncthreads();
        }
}

// The coarse end of the block V-cycle in one workgroup: levels 0..n-1 of
// `F` (the last is the coarsest) are small enough that per-level launches
// would cost more than the work, so one workgroup runs their smoothing,
// residual, restriction, coarse solve and prolongation with barriers in
// between, node by node exactly as the per-level kernels do.
template <class T, bool kLds>
__global__ __launch_bounds__(1024) void k_block_subcycle(FusedLevelsT<T> F, Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    __shared__ T pool[kLds ? kSubPool : 1];
    SubMem<T, kLds> M{F, bo_};
    // the coarsest inverse's entries this thread multiplies, loaded first
    // (n <= 64) so that their latency hides behind the staging and the
    // finer levels
    const T *invT = boff(F.invT, bo_);
    const Geom gl = geom_off(F.g[F.n - 1], bo_);
    const int nco = 3 * (gl.nr + 1) * (gl.nz - 1);
    T pre[kCsPre];
    {
        const int lane = threadIdx.x & 63, part = threadIdx.x >> 6;
#pragma unroll
        for (int u = 0; u < kCsPre; ++u) {
            const int k = part + kCsParts * u;
            pre[u] = (nco <= 64 && k < nco && lane < nco) ? invT[(int64_t)k * nco + lane] : T(0);
        }
    }
    if constexpr (kLds) {
        M.pool = pool;
        M.stage_all();
    } else {
        for (int q = 0; q < F.n; ++q) {
            const Geom g = geom_off(F.g[q], bo_);
            T *xq = M.x(q);
            const int nodes = (g.nr + 1) * (g.nz + 1);
            for (int t = threadIdx.x; t < nodes; t += blockDim.x) {
                int64_t p = at(g, t / (g.nz + 1), t % (g.nz + 1));
                xq[p] = xq[p + F.plane[q]] = xq[p + 2 * F.plane[q]] = T(0);
            }
        }
    }
    __syncthreads();
    auto geom = [&](int q) { return M.geom(q); };
    auto jac = [&](int q) { return M.jac(q); };
    auto xof = [&](int q) { return M.x(q); };
    auto rof = [&](int q) { return M.r(q); };
    const T *f0 = M.f0();

    __shared__ T rhs[3 * kMaxFusedCoarse];
    __shared__ T red[kCsParts][64];
    const int n = F.n;
    const int nt = blockDim.x;
    for (int q = 0; q < n - 1; ++q) {
        const Geom g = geom(q);
        const BOpT<T> J = jac(q);
        const T *f = (q == 0) ? f0 : J.pl(kFe);
        T *x = xof(q);
        T *r = rof(q);
        const int nodes = (g.nr + 1) * (g.nz + 1);
        // every level's correction starts from zero (set while staging)
        subcycle_smooth(g, J, f, x, F.nu1);
        for (int t = threadIdx.x; t < nodes; t += nt) {
            int i = t / (g.nz + 1), j = t % (g.nz + 1);
            block_residual_node(g, J, f, x, r, 0, i, j);
        }
        __syncthreads();
        const Geom gc = geom(q + 1);
        const BOpT<T> Jc = jac(q + 1);
        const int cnodes = (gc.nr + 1) * (gc.nz + 1);
        for (int t = threadIdx.x; t < cnodes; t += nt) {
            int I = t / (gc.nz + 1), J_ = t % (gc.nz + 1);
            restrict3_node(g, r, J.plane, gc, Jc.pl(kFe), Jc.plane, I, J_);
        }
        __syncthreads();
    }
    {
        const int q = n - 1;
        const BOpT<T> J = jac(q);
        const T *f = (q == 0) ? f0 : J.pl(kFe);
        // (the coarsest correction's electrode rows were zeroed while staging)
        block_coarse_solve_wg(geom(q), J.plane, f, invT, xof(q), rhs, red, nco <= 64, pre);
        __syncthreads();
    }
    for (int q = n - 2; q >= 0; --q) {
        const Geom g = geom(q);
        const BOpT<T> J = jac(q);
        const T *f = (q == 0) ? f0 : J.pl(kFe);
        T *x = xof(q);
        const Geom gc = geom(q + 1);
        const T *xc = xof(q + 1);
        const int nodes = (g.nr + 1) * (g.nz + 1);
        for (int t = threadIdx.x; t < nodes; t += nt) {
            int i = t / (g.nz + 1), j = t % (g.nz + 1);
            if (j >= 1 && j < g.nz) prolong3_node(g, x, J.plane, gc, xc, M.xplane(q + 1), i, j);
        }
        __syncthreads();
        subcycle_smooth(g, J, f, x, F.nu2);
    }
    if constexpr (kLds) {
        __syncthreads();
        const Geom gg = geom_off(F.g[0], bo_);
        T *dst = boff(F.x[0], bo_);
        const T *src = xof(0);
        const int w = gg.nz + 1, nn = (gg.nr + 1) * w;
        for (int t = threadIdx.x; t < 3 * nn; t += blockDim.x) {
            const int k = t / nn, node = t % nn;
            dst[k * F.plane[0] + (int64_t)(node / w) * gg.pitch + node % w] = src[k * (int64_t)nn + node];
        }
    }
}

// ---- FGMRES BLAS-1 (weighted inner product) ----
// <u, v>_W = sum over unknown nodes and fields of u v (c_f / vol)^2, with
// c_f = 1 for the densities and 1/k for the Poisson rows.

// One pass of classical Gram-Schmidt: w = B z (if z: the operator applied
// to the new preconditioned direction), or w -= sum_v h_sub[v] basis_v (if
// h_sub), at every unknown node, then the per-workgroup partial sums of the
// weighted dot products of (the updated) w with basis_0..basis_{nv-1}, or
// with w itself (self_norm).  The grid-wide sums are formed by a following
// launch (k_sum_cols, or the next chained pass) in a fixed order.
// Projections h_v = sum over the nblk workgroup partials (partial b of
// column v at part[b * nv + v]) in a fixed order: lane l adds the partials b
// = l, l + 64, ... in turn, then the 64 lane sums are combined by an xor
// butterfly and lane 0's total is taken (the same bits in every workgroup).
// One wavefront per column; the result goes to LDS hs[v], and workgroup
// (0, 0) also stores it to out (device) and out_host (pinned host memory).
// The loads of a lane's partials are issued together (kChainLoads per pass:
// one pass for the grids that chain their passes), then added in order.
constexpr int kChainLoads = 8;
constexpr int kCgsRegs = 8, kCgsRegs2 = 16;  // basis vectors a Gram-Schmidt pass keeps in registers
inline __device__ void reduce_projections(const double *__restrict__ part, int nblk, int nv, double *hs,
                                          double *out, double *out_host) {
    for (int v = threadIdx.y; v < nv; v += blockDim.y) {
        double a = 0.0;
        for (int b0 = threadIdx.x; b0 < nblk; b0 += kTX * kChainLoads) {
            double q[kChainLoads];
#pragma unroll
            for (int u = 0; u < kChainLoads; ++u) {
                const int b = b0 + u * kTX;
                q[u] = b < nblk ? part[(int64_t)b * nv + v] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kChainLoads; ++u)
                if (b0 + u * kTX < nblk) a += q[u];
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
        a = __shfl(a, 0);
        if (threadIdx.x == 0) {
            hs[v] = a;
            if (blockIdx.x == 0 && blockIdx.y == 0) {
                if (out) out[v] = a;
                if (out_host) out_host[v] = a;
            }
        }
    }
    __syncthreads();
}

// Squared norm of u - V h for u with (u, u) = ww and projections h = V^T u
// onto an orthonormal V (Pythagoras), the subtraction in a fixed order.
inline __device__ double lagged_nu2(const double *h, int nv, double ww) {
    double n2 = ww;
    for (int v = 0; v < nv; ++v) n2 = fmad(-h[v], h[v], n2);
    return n2;
}

// NV > 0: at most NV basis vectors (nv <= NV); a node's basis values are
// loaded once into registers, before the previous pass's projections are
// summed (their loads overlap), and serve both the update and the dot
// products (NV = 16 only for workgroups of at most 256 threads, whose
// register budget holds them).  NV = 0: any nv, the basis read as it is
// used.  All forms do the same arithmetic (explicit fused multiply-adds in
// the same order).
template <int NV>
__global__ __launch_bounds__(NV > 8 ? 256 : 1024) void k_cgs_pass(Geom g, double *__restrict__ w,
                                                                  const double *__restrict__ basis,
                                                   int64_t vstride, int nv, int64_t plane, double3 cw,
                                                   const double *__restrict__ h_sub, int self_norm, BOp Jop,
                                                   const double *__restrict__ z, double *__restrict__ partials,
                                                   const double *__restrict__ h_part, int h_nblk,
                                                   double *__restrict__ h_out, double *__restrict__ h_host,
                                                   CgsLag lag, Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    g = geom_off(g, bo_);
    w = boff(w, bo_);
    basis = boff(basis, bo_);
    h_sub = boff(h_sub, bo_);
    partials = boff(partials, bo_);
    z = boff(z, bo_);
    Jop.base = boff(Jop.base, bo_);
    lag.fin_h = boff(lag.fin_h, bo_);
    lag.fin_nu2 = boff(lag.fin_nu2, bo_);
    lag.fin_out = boff(lag.fin_out, bo_);
    lag.next = boff(lag.next, bo_);

    const int j = blockIdx.x * kTX + threadIdx.x;
    const int i = blockIdx.y * blockDim.y + threadIdx.y;
    __shared__ double sh[kMaxTY][kMaxKrylov + 1];
    __shared__ double hs[kMaxKrylov + 1];
    __shared__ double hf[kMaxKrylov + 1];
    __shared__ double inv_nu;
    const bool ok = i <= g.nr && j >= 1 && j < g.nz;
    const int64_t p = ok ? at(g, i, j) : 0;
    const int kf = nv - 1;  // the basis slot finalised by this pass (lag.fin_h)
    // basis values of this node (register form)
    double bv[NV > 0 ? NV : 1][3];
    const bool upd = h_part || h_sub;
    if constexpr (NV > 0) {
        if (ok && (upd || !self_norm)) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
                if (v < nv) {
                    const double *bb = basis + v * vstride + p;
                    bv[v][0] = bb[0];
                    bv[v][1] = bb[plane];
                    bv[v][2] = bb[2 * plane];
                }
        }
    }
    // Deferred second projection and normalisation of basis slot kf: it
    // holds u = w' of the previous Arnoldi step (one projection removed);
    // v = (u - sum_{v<kf} hf_v b_v) / nu with nu^2 = (u, u) - |hf|^2.  The
    // node's finalised values replace slot kf in memory and in the dot
    // products below (vf; slot kf is not read again).
    double vf[3] = {0.0, 0.0, 0.0};
    const bool fin = lag.fin_h || lag.fin_part;
    if (fin) {
        const int t = threadIdx.y * kTX + threadIdx.x;
        if (lag.fin_part) {
            // the previous second pass's partials: kf projections and (u, u)
            reduce_projections(boff(lag.fin_part, bo_), lag.fin_nblk, kf + 1, hf, nullptr, nullptr);
            if (t == 0) {
                const double n2 = lagged_nu2(hf, kf, hf[kf]);
                inv_nu = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
            }
        } else {
            for (int v = t; v < kf; v += kTX * blockDim.y) hf[v] = lag.fin_h[v];
            if (t == 0) {
                const double n2 = *lag.fin_nu2;
                inv_nu = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
            }
        }
        __syncthreads();
        if (ok) {
            double u[3];
            if constexpr (NV > 0) {
                // register indices stay compile-time constants
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    if (v == kf)
#pragma unroll
                        for (int f = 0; f < 3; ++f) u[f] = bv[v][f];
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    if (v < kf)
#pragma unroll
                        for (int f = 0; f < 3; ++f) u[f] = fmad(-hf[v], bv[v][f], u[f]);
            } else {
                for (int f = 0; f < 3; ++f) u[f] = basis[kf * vstride + p + f * plane];
                for (int v = 0; v < kf; ++v)
                    for (int f = 0; f < 3; ++f) u[f] = fmad(-hf[v], basis[v * vstride + p + f * plane], u[f]);
            }
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                vf[f] = u[f] * inv_nu;
                lag.fin_out[p + f * plane] = vf[f];
            }
            if constexpr (NV > 0) {
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    if (v == kf)
#pragma unroll
                        for (int f = 0; f < 3; ++f) bv[v][f] = vf[f];
            }
        }
    }
    if (h_part) {
        // the previous pass's projections, formed here instead of by a launch of their own
        reduce_projections(boff(h_part, bo_), h_nblk, nv, hs, boff(h_out, bo_), h_host);
        h_sub = hs;
    }
    double wf[3] = {0.0, 0.0, 0.0};
    if (z && i <= g.nr && (j == 0 || j == g.nz)) {
        const int64_t pb = at(g, i, j);
        w[pb] = w[pb + plane] = w[pb + 2 * plane] = 0.0;
    }
    if (ok && z) {
        block_apply_node(g, Jop, z, i, p, wf[0], wf[1], wf[2]);
        w[p] = wf[0];
        w[p + plane] = wf[1];
        w[p + 2 * plane] = wf[2];
    } else if (ok) {
        for (int f = 0; f < 3; ++f) wf[f] = w[p + f * plane];
        if (h_sub) {
            if constexpr (NV > 0) {
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    if (v < nv && h_sub[v] != 0.0)
                        for (int f = 0; f < 3; ++f) wf[f] = fmad(-h_sub[v], bv[v][f], wf[f]);
            } else {
                for (int v = 0; v < nv; ++v)
                    if (h_sub[v] != 0.0)
                        for (int f = 0; f < 3; ++f) wf[f] = fmad(-h_sub[v], basis[v * vstride + p + f * plane], wf[f]);
            }
            double *dst = lag.next ? lag.next : w;
            for (int f = 0; f < 3; ++f) dst[p + f * plane] = wf[f];
        }
    }
    if (lag.next && i <= g.nr && (j == 0 || j == g.nz)) {
        const int64_t pb = at(g, i, j);
        lag.next[pb] = lag.next[pb + plane] = lag.next[pb + 2 * plane] = 0.0;
    }
    const double iv = ok ? 1.0 / (g.wr[i] * g.dzc[j]) : 0.0;
    const double we = wf[0] * cw.x * cw.x * iv * iv;
    const double wp = wf[1] * cw.y * cw.y * iv * iv;
    const double wv = wf[2] * cw.z * cw.z * iv * iv;
    auto dot3 = [&](double b0, double b1, double b2) { return fmad(wv, b2, fmad(wp, b1, we * b0)); };
    auto wave_sum = [](double s) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        return s;
    };
    const int nd = self_norm ? 1 : nv + (lag.with_norm ? 1 : 0);
    if (self_norm) {
        const double s = wave_sum(ok ? dot3(wf[0], wf[1], wf[2]) : 0.0);
        if (threadIdx.x == 0) sh[threadIdx.y][0] = s;
    } else {
        if constexpr (NV > 0) {
            double sv[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) sv[v] = (ok && v < nv) ? dot3(bv[v][0], bv[v][1], bv[v][2]) : 0.0;
#pragma unroll
            for (int v = 0; v < NV; ++v)
                if (v < nv) {
                    const double s = wave_sum(sv[v]);
                    if (threadIdx.x == 0) sh[threadIdx.y][v] = s;
                }
        } else {
            for (int v = 0; v < nv; ++v) {
                double d = 0.0;
                if (ok) {
                    if (fin && v == kf) {
                        d = dot3(vf[0], vf[1], vf[2]);
                    } else {
                        const double *b = basis + v * vstride;
                        d = dot3(b[p], b[p + plane], b[p + 2 * plane]);
                    }
                }
                const double s = wave_sum(d);
                if (threadIdx.x == 0) sh[threadIdx.y][v] = s;
            }
        }
        if (lag.with_norm) {
            const double s = wave_sum(ok ? dot3(wf[0], wf[1], wf[2]) : 0.0);
            if (threadIdx.x == 0) sh[threadIdx.y][nv] = s;
        }
    }
    __syncthreads();
    const int blk = blockIdx.y * gridDim.x + blockIdx.x;
    const int t = threadIdx.y * kTX + threadIdx.x;
    if (t < nd) {
        double s = 0.0;
        for (int y = 0; y < (int)blockDim.y; ++y) s += sh[y][t];
        partials[(int64_t)blk * nd + t] = s;
        if (lag.part_host) lag.part_host[(int64_t)blk * nd + t] = s;
    }
}

// nu^2 = ww - sum_v h_v^2 for the unchained passes: h (nv values) and ww
// (at h[nv]) from k_sum_cols; one thread per problem.
__global__ void k_lagged_nu2(double *__restrict__ h, int nv, double *__restrict__ out, double *__restrict__ out_host,
                             Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    h = boff(h, bo_);
    out = boff(out, bo_);
    if (threadIdx.x != 0) return;
    const double n2 = lagged_nu2(h, nv, h[nv]);
    *out = n2;
    if (out_host) *out_host = n2;
}

// out[c] = sum over blocks of partials[b*ncomp + c], fixed order (one
// workgroup per component).
__global__ __launch_bounds__(256) void k_sum_cols(const double *__restrict__ part, int nblocks, int ncomp,
                                                   double *__restrict__ out, Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    part = boff(part, bo_);
    out = boff(out, bo_);

    int c = blockIdx.x;
    __shared__ double sh[256];
    double acc = sum_strided(part, nblocks, threadIdx.x, 256, ncomp, c);
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = sh[0];
}

// w = alpha * (w - sum_v h[v] basis_v)   (alpha = 1, or 1/h_next on demand)
__global__ void k_axpy_multi(Geom g, double *__restrict__ w, const double *__restrict__ basis, int64_t vstride,
                             int nv, int64_t plane, const double *__restrict__ h, double sign, Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    g = geom_off(g, bo_);
    w = boff(w, bo_);
    basis = boff(basis, bo_);
    h = boff(h, bo_);

    int j = blockIdx.x * kTX + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > g.nr || j < 1 || j >= g.nz) return;
    int64_t p = at(g, i, j);
    for (int f = 0; f < 3; ++f) {
        int64_t q = p + f * plane;
        double acc = w[q];
        for (int v = 0; v < nv; ++v)
            if (h[v] != 0.0) acc += sign * h[v] * basis[v * vstride + q];
        w[q] = acc;
    }
}

// dst = src * (1 / sqrt(*nrm2))
__global__ void k_scale_by_norm(Geom g, const double *__restrict__ src, double *__restrict__ dst, int64_t plane,
                                const double *__restrict__ nrm2, Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    g = geom_off(g, bo_);
    src = boff(src, bo_);
    dst = boff(dst, bo_);
    nrm2 = boff(nrm2, bo_);

    int j = blockIdx.x * kTX + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    if (i > g.nr || j > g.nz) return;
    int64_t p = at(g, i, j);
    double s = 1.0 / sqrt(*nrm2);
    bool un = j >= 1 && j < g.nz;
    for (int f = 0; f < 3; ++f) dst[p + f * plane] = un ? src[p + f * plane] * s : 0.0;
}

// Newton update u += du on the unknown nodes, with per-block sums of
// |du_f| and |u_f| (l1) and the minima of the densities.
__global__ __launch_bounds__(1024) void k_newton_update(Geom g, double *__restrict__ V, double *__restrict__ ne,
                                                        double *__restrict__ np, const double *__restrict__ du,
                                                        int64_t plane, double *__restrict__ partials, Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    g = geom_off(g, bo_);
    V = boff(V, bo_);
    ne = boff(ne, bo_);
    np = boff(np, bo_);
    du = boff(du, bo_);
    partials = boff(partials, bo_);

    int j = blockIdx.x * kTX + threadIdx.x;
    int i = blockIdx.y * blockDim.y + threadIdx.y;
    double s[8] = {0, 0, 0, 0, 0, 0, 1e300, 1e300};
    if (i <= g.nr && j >= 1 && j < g.nz) {
        int64_t p = at(g, i, j);
        double de = du[p], dp = du[p + plane], dv = du[p + 2 * plane];
        double a = ne[p] + de, b = np[p] + dp, c = V[p] + dv;
        ne[p] = a;
        np[p] = b;
        V[p] = c;
        s[0] = fabs(de);
        s[1] = fabs(a);
        s[2] = fabs(dp);
        s[3] = fabs(b);
        s[4] = fabs(dv);
        s[5] = fabs(c);
        s[6] = a;
        s[7] = b;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int k = 0; k < 6; ++k) s[k] += __shfl_xor(s[k], off);
        s[6] = fmin(s[6], __shfl_xor(s[6], off));
        s[7] = fmin(s[7], __shfl_xor(s[7], off));
    }
    __shared__ double sh[kMaxTY][8];
    if (threadIdx.x == 0)
        for (int k = 0; k < 8; ++k) sh[threadIdx.y][k] = s[k];
    __syncthreads();
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        double o[8] = {0, 0, 0, 0, 0, 0, 1e300, 1e300};
        for (int y = 0; y < (int)blockDim.y; ++y) {
            for (int k = 0; k < 6; ++k) o[k] += sh[y][k];
            o[6] = fmin(o[6], sh[y][6]);
            o[7] = fmin(o[7], sh[y][7]);
        }
        int blk = blockIdx.y * gridDim.x + blockIdx.x;
        for (int k = 0; k < 8; ++k) partials[(int64_t)blk * 8 + k] = o[k];
    }
}

__global__ __launch_bounds__(256) void k_reduce_newton(const double *__restrict__ part, int nblocks,
                                                        double *__restrict__ out, Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    part = boff(part, bo_);
    out = boff(out, bo_);

    __shared__ double sh[8][256];
    double o[8] = {0, 0, 0, 0, 0, 0, 1e300, 1e300};
    for (int b = threadIdx.x; b < nblocks; b += 256) {
        for (int k = 0; k < 6; ++k) o[k] += part[(int64_t)b * 8 + k];
        o[6] = fmin(o[6], part[(int64_t)b * 8 + 6]);
        o[7] = fmin(o[7], part[(int64_t)b * 8 + 7]);
    }
    for (int k = 0; k < 8; ++k) sh[k][threadIdx.x] = o[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int k = 0; k < 6; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
            sh[6][threadIdx.x] = fmin(sh[6][threadIdx.x], sh[6][threadIdx.x + w]);
            sh[7][threadIdx.x] = fmin(sh[7][threadIdx.x], sh[7][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 8) out[threadIdx.x] = sh[threadIdx.x][0];
}

}  // namespace

static dim3 gz(dim3 g, const Batch &bt) { return dim3(g.x, g.y, bt.n); }

void launch_newton_assemble(const Geom &g, const BOp &J, const double *V, const double *ne, const double *np,
                            const double *nek, const double *npk, const double *Se, const double *Sp,
                            const NewtonPhys &ph, bool with_rhs, hipStream_t s, const NewtonPhys *php,
                            const Batch &bt, const NodeTransport &tr) {
    k_newton_assemble<<<gz(grid2d(g), bt), blk2d(g), 0, s>>>(g, J, V, ne, np, nek, npk, Se, Sp, ph, with_rhs ? 1 : 0,
                                                         php, bt, tr);
}
template <class T>
void launch_block_zline(const Geom &g, const BOpT<T> &J, const T *f, T *x, T *tmp, int colour, hipStream_t s,
                        const Batch &bt) {
    const int lines = (g.nr + 2 - colour) / 2;  // i = colour, colour + 2, ... <= nr
    k_block_zline<T><<<dim3((lines + 63) / 64, 1, bt.n), 64, 0, s>>>(g, J, f, x, tmp, colour, bt);
}
template <class T>
void launch_block_rbgs(const Geom &g, const BOpT<T> &J, const T *f, T *x, int colour, hipStream_t s, const Batch &bt) {
    k_block_rbgs<T><<<gz(grid2d(g), bt), blk2d(g), 0, s>>>(g, J, f, x, colour, bt);
}
template <class T>
void launch_block_rb_sweep(const Geom &g, const BOpT<T> &J, const T *f, const T *xin, T *xout, bool zin,
                           const Geom *gc, const T *xc, int64_t pc, hipStream_t s, const Batch &bt) {
    const Geom &gcc = gc ? *gc : g;
    if (g.sh == 8) {
        using Tl = SweepTile<8>;
        dim3 grid((g.nz + 1 + kSW - 1) / kSW, (g.nr + 1 + Tl::kSH - 1) / Tl::kSH);
        k_block_rb_sweep<T, 8><<<gz(grid, bt), dim3(kSW, Tl::kSH + Tl::kSR), 0, s>>>(g, J, f, xin, xout, zin ? 1 : 0,
                                                                                    gcc, xc, pc, bt);
    } else {
        using Tl = SweepTile<16>;
        dim3 grid((g.nz + 1 + kSW - 1) / kSW, (g.nr + 1 + Tl::kSH - 1) / Tl::kSH);
        k_block_rb_sweep<T, 16><<<gz(grid, bt), dim3(kSW, Tl::kSH + Tl::kSR), 0, s>>>(g, J, f, xin, xout,
                                                                                      zin ? 1 : 0, gcc, xc, pc, bt);
    }
}
template <class T>
void launch_block_rb_sweep2(const Geom &g, const BOpT<T> &J, const T *f, const T *xin, T *xout, bool zin,
                            const Geom *gc, const T *xc, int64_t pc, hipStream_t s, const Batch &bt) {
    const Geom &gcc = gc ? *gc : g;
    if (g.sh2 == 4) {
        dim3 grid((g.nz + 1 + kSW - 1) / kSW, (g.nr + 1 + 4 - 1) / 4);
        k_block_rb_sweep2<T, 4, false><<<gz(grid, bt), Sweep2Tile<4>::kThreads, 0, s>>>(
            g, J, f, xin, xout, zin ? 1 : 0, gcc, xc, pc, nullptr, bt);
        return;
    }
    dim3 grid((g.nz + 1 + kSW - 1) / kSW, (g.nr + 1 + 8 - 1) / 8);
    k_block_rb_sweep2<T, 8, false><<<gz(grid, bt), Sweep2Tile<8>::kThreads, 0, s>>>(g, J, f, xin, xout, zin ? 1 : 0,
                                                                                  gcc, xc, pc, nullptr, bt);
}
template <class T>
void launch_block_rb_sweep2_restrict(const Geom &g, const BOpT<T> &J, const T *f, const T *xin, T *xout, bool zin,
                                     const Geom &gc, T *fc, int64_t pc, hipStream_t s, const Batch &bt) {
    if (g.sh2 == 4) {
        dim3 grid((g.nz + 1 + kSW - 1) / kSW, (g.nr + 1 + 4 - 1) / 4);
        k_block_rb_sweep2<T, 4, true><<<gz(grid, bt), Sweep2Tile<4, true>::kThreads, 0, s>>>(
            g, J, f, xin, xout, zin ? 1 : 0, gc, nullptr, pc, fc, bt);
        return;
    }
    dim3 grid((g.nz + 1 + kSW - 1) / kSW, (g.nr + 1 + 8 - 1) / 8);
    k_block_rb_sweep2<T, 8, true><<<gz(grid, bt), Sweep2Tile<8, true>::kThreads, 0, s>>>(
        g, J, f, xin, xout, zin ? 1 : 0, gc, nullptr, pc, fc, bt);
}
template <class T>
void launch_block_residual(const Geom &g, const BOpT<T> &J, const T *f, const T *x, T *r, bool apply,
                           hipStream_t s, const Batch &bt) {
    k_block_residual<T><<<gz(grid2d(g), bt), blk2d(g), 0, s>>>(g, J, f, x, r, apply ? 1 : 0, bt);
}
template <class T>
void launch_restrict3(const Geom &gf, const T *rf, int64_t pf, const Geom &gc, T *fc, int64_t pc, hipStream_t s,
                      const Batch &bt) {
    k_restrict3<T><<<gz(grid2d(gc), bt), blk2d(gc), 0, s>>>(gf, rf, pf, gc, fc, pc, bt);
}
template <class T>
void launch_residual_restrict(const Geom &gf, const BOpT<T> &J, const T *f, const T *x, const Geom &gc, T *fc,
                              int64_t pc, hipStream_t s, const Batch &bt) {
    dim3 grid((gc.nz + 1 + kCW - 1) / kCW, (gc.nr + 1 + kCH - 1) / kCH);
    k_block_residual_restrict<T><<<gz(grid, bt), dim3(64, 10), 0, s>>>(gf, J, f, x, gc, fc, pc, bt);
}
template <class T>
void launch_prolong3(const Geom &gf, T *xf, int64_t pf, const Geom &gc, const T *xc, int64_t pc, hipStream_t s,
                     const Batch &bt) {
    k_prolong3<T><<<gz(grid2d(gf), bt), blk2d(gf), 0, s>>>(gf, xf, pf, gc, xc, pc, bt);
}
void launch_block_coarse_factor(const Geom &g, const BOp &J, double *scratch, double *invT, hipStream_t s,
                                const Batch &bt) {
    int n = 3 * (g.nr + 1) * (g.nz - 1);
    if (n <= kLdsGJ)
        k_block_coarse_factor_lds<<<dim3(1, 1, bt.n), kFactorThreads, 0, s>>>(g, J, invT, bt);
    else
        k_block_coarse_factor<<<dim3(1, 1, bt.n), 1024, 0, s>>>(g, J, scratch, invT, bt);
}
template <class T>
void launch_block_coarse_solve(const Geom &g, const BOpT<T> &J, const T *f, const T *invT, T *x, hipStream_t s,
                               const Batch &bt) {
    k_block_coarse_solve<T><<<dim3(1, 1, bt.n), 1024, 0, s>>>(g, J, f, invT, x, bt);
}
template <class T>
void launch_block_subcycle(const FusedLevelsT<T> &F, hipStream_t s, const Batch &bt) {
    int64_t need = 0;
    for (int q = 0; q < F.n; ++q) need += (int64_t)(kBPlanes + 6) * (F.g[q].nr + 1) * (F.g[q].nz + 1);
    need += 3 * (int64_t)(F.g[0].nr + 1) * (F.g[0].nz + 1);
    // the LDS copy reads rows of planes (nr + 1) * pitch apart; row index
    // e / (nz + 1) by a multiply-high with ceil(2^32 / (nz + 1)) (exact for
    // e (nz + 1) < 2^32)
    bool rows_ok = true;
    FusedLevelsT<T> G = F;
    for (int q = 0; q < F.n; ++q) {
        const uint64_t w = (uint64_t)F.g[q].nz + 1;
        rows_ok = rows_ok && F.plane[q] == (int64_t)(F.g[q].nr + 1) * F.g[q].pitch && w * kSubPool < (1ull << 32);
        G.wmagic[q] = (uint32_t)(((1ull << 32) + w - 1) / w);
    }
    if (need <= kSubPool && rows_ok)
        k_block_subcycle<T, true><<<dim3(1, 1, bt.n), 1024, 0, s>>>(G, bt);
    else
        k_block_subcycle<T, false><<<dim3(1, 1, bt.n), 1024, 0, s>>>(F, bt);
}
int block_vec_blocks(const Geom &g) {
    dim3 gr = grid2d(g);
    return (int)(gr.x * gr.y);
}
// The Gram-Schmidt pass form for nv basis vectors and the launch's workgroup size.
decltype(&k_cgs_pass<0>) cgs_kernel(const Geom &g, int nv) {
    if (nv <= kCgsRegs) return k_cgs_pass<kCgsRegs>;
    if (nv <= kCgsRegs2 && kTX * g.ty <= 256) return k_cgs_pass<kCgsRegs2>;
    return k_cgs_pass<0>;
}
void launch_cgs_pass(const Geom &g, double *w, const double *basis, int64_t vstride, int nv, int64_t plane,
                     double3 cw, const double *h_sub, bool self_norm, double *partials, double *out, hipStream_t s,
                     const Batch &bt, const BOp *J, const double *z, const CgsLag &lag) {
    dim3 gr = grid2d(g);
    auto k = cgs_kernel(g, nv);
    k<<<gz(gr, bt), blk2d(g), 0, s>>>(g, w, basis, vstride, nv, plane, cw, h_sub, self_norm ? 1 : 0,
                                      J ? *J : BOp{nullptr, 0}, z, partials, nullptr, 0, nullptr, nullptr, lag, bt);
    if (out) {
        int nd = self_norm ? 1 : nv + (lag.with_norm ? 1 : 0);
        k_sum_cols<<<dim3(nd, 1, bt.n), 256, 0, s>>>(partials, (int)(gr.x * gr.y), nd, out, bt);
    }
}
void launch_lagged_nu2(double *h, int nv, double *out, double *out_host, hipStream_t s, const Batch &bt) {
    k_lagged_nu2<<<dim3(1, 1, bt.n), 64, 0, s>>>(h, nv, out, out_host, bt);
}
void launch_cgs_pass_chained(const Geom &g, double *w, const double *basis, int64_t vstride, int nv, int64_t plane,
                             double3 cw, bool self_norm, const double *h_part, double *h_out, double *h_host,
                             double *partials, hipStream_t s, const Batch &bt, const CgsLag &lag) {
    dim3 gr = grid2d(g);
    auto k = cgs_kernel(g, nv);
    k<<<gz(gr, bt), blk2d(g), 0, s>>>(g, w, basis, vstride, nv, plane, cw, nullptr, self_norm ? 1 : 0,
                                      BOp{nullptr, 0}, nullptr, partials, h_part, (int)(gr.x * gr.y), h_out, h_host,
                                      lag, bt);
}
void launch_axpy_multi(const Geom &g, double *w, const double *basis, int64_t vstride, int nv, int64_t plane,
                       const double *h, double sign, hipStream_t s, const Batch &bt) {
    k_axpy_multi<<<gz(grid2d(g), bt), blk2d(g), 0, s>>>(g, w, basis, vstride, nv, plane, h, sign, bt);
}
void launch_scale_by_norm(const Geom &g, const double *src, double *dst, int64_t plane, const double *nrm2,
                          hipStream_t s, const Batch &bt) {
    k_scale_by_norm<<<gz(grid2d(g), bt), blk2d(g), 0, s>>>(g, src, dst, plane, nrm2, bt);
}
void launch_newton_update(const Geom &g, double *V, double *ne, double *np, const double *du, int64_t plane,
                          double *partials, double *out, hipStream_t s, const Batch &bt) {
    dim3 gr = grid2d(g);
    k_newton_update<<<gz(gr, bt), blk2d(g), 0, s>>>(g, V, ne, np, du, plane, partials, bt);
    k_reduce_newton<<<dim3(1, 1, bt.n), 256, 0, s>>>(partials, (int)(gr.x * gr.y), out, bt);
}

// FP32 copy of the block Jacobian: every plane rounded, except the diagonal
// entries of the three five-point blocks (ee, pp, VV), which are rebuilt from
// their exact FP64 column excess minus the rounded neighbour entries of the
// same column (see k_op_to_f32 for the reason).
namespace {
// FP32 copy of one node's planes.  The diagonal centre entries are
// re-rounded so that each FP32 row keeps the FP64 row's excess of the
// centre over the neighbour couplings of its own field.
inline __device__ void block_to_f32_node(const Geom &g, const BOp &J, const BOpT<float> &J32, int i, int j) {
    int64_t p = at(g, i, j);
    for (int k = 0; k < kBPlanes; ++k) J32.pl(k)[p] = (float)J.pl(k)[p];
    if (j == 0 || j == g.nz) return;
    const int kinds[3] = {kEE, kPP, kVV};
    for (int t = 0; t < 3; ++t) {
        const int K = kinds[t];
        double ex = J.pl(K + 1)[p], r32 = 0.0;
        if (i > 0) {
            double v = J.pl(K + 2)[p - g.pitch];
            ex += v;
            r32 += (double)(float)v;
        }
        if (i < g.nr) {
            double v = J.pl(K + 0)[p + g.pitch];
            ex += v;
            r32 += (double)(float)v;
        }
        if (j > 1) {
            double v = J.pl(K + 4)[p - 1];
            ex += v;
            r32 += (double)(float)v;
        }
        if (j < g.nz - 1) {
            double v = J.pl(K + 3)[p + 1];
            ex += v;
            r32 += (double)(float)v;
        }
        J32.pl(K + 1)[p] = (float)(ex - r32);
    }
}

__global__ __launch_bounds__(kTX *kLevTabTY) void k_block_to_f32_levels(LevTab t, Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    int l = 0;
    while (l + 1 < t.n && (int)blockIdx.y >= t.y0[l + 1]) ++l;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    Geom g = geom_off(t.g[l], bo_);
    BOp J = t.J[l];
    J.base = boff(J.base, bo_);
    BOpT<float> J32 = t.J32[l];
    J32.base = boff(J32.base, bo_);

    int j = blockIdx.x * kTX + threadIdx.x;
    int i = (blockIdx.y - t.y0[l]) * kLevTabTY + threadIdx.y;
    if (i > g.nr || j > g.nz) return;
    block_to_f32_node(g, J, J32, i, j);
}

// Row-block starts of every level of the table; returns the launch grid.
dim3 levtab_grid(LevTab &t, const Batch &bt) {
    int y = 0, x = 0;
    for (int k = 0; k < t.n; ++k) {
        t.y0[k] = y;
        y += (t.g[k].nr + 1 + kLevTabTY - 1) / kLevTabTY;
        int bx = (t.g[k].nz + 1 + kTX - 1) / kTX;
        x = bx > x ? bx : x;
    }
    t.y0[t.n] = y;
    return dim3(x, y, bt.n);
}
}  // namespace

void launch_block_to_f32_levels(LevTab t, hipStream_t s, const Batch &bt) {
    dim3 grid = levtab_grid(t, bt);
    k_block_to_f32_levels<<<grid, dim3(kTX, kLevTabTY), 0, s>>>(t, bt);
}
void launch_newton_assemble_coarse(LevTab t, const double *V, const double *ne, const double *np, int64_t pitch0,
                                   const NewtonPhys &ph, hipStream_t s, const NewtonPhys *php, const Batch &bt,
                                   const NodeTransport &tr) {
    dim3 grid = levtab_grid(t, bt);
    k_newton_assemble_coarse<<<grid, dim3(kTX, kLevTabTY), 0, s>>>(t, V, ne, np, pitch0, ph, php, bt, tr);
}

// planes -> FP32 copies (n planes of `plane` elements)
__global__ void k_planes_to_f32(const double *__restrict__ src, float *__restrict__ dst, int64_t n, Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    src = boff(src, bo_);
    dst = boff(dst, bo_);

    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; t < n; t += stride) dst[t] = (float)src[t];
}
__global__ void k_planes_to_f64(const float *__restrict__ src, double *__restrict__ dst, int64_t n, Batch bt) {
    if (bt.active && !bt.active[blockIdx.z]) return;
    const int64_t bo_ = (int64_t)blockIdx.z * bt.stride;
    src = boff(src, bo_);
    dst = boff(dst, bo_);

    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; t < n; t += stride) dst[t] = (double)src[t];
}
void launch_planes_to_f32(const double *src, float *dst, int64_t n, hipStream_t s, const Batch &bt) {
    int64_t b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    k_planes_to_f32<<<dim3((unsigned)b, 1, bt.n), 256, 0, s>>>(src, dst, n, bt);
}
void launch_planes_to_f64(const float *src, double *dst, int64_t n, hipStream_t s, const Batch &bt) {
    int64_t b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    k_planes_to_f64<<<dim3((unsigned)b, 1, bt.n), 256, 0, s>>>(src, dst, n, bt);
}

#define MGF_INST(T)                                                                                          \
    template void launch_block_rbgs<T>(const Geom &, const BOpT<T> &, const T *, T *, int, hipStream_t,      \
                                       const Batch &);                                                       \
    template void launch_block_rb_sweep<T>(const Geom &, const BOpT<T> &, const T *, const T *, T *, bool,   \
                                           const Geom *, const T *, int64_t, hipStream_t, const Batch &);     \
    template void launch_block_zline<T>(const Geom &, const BOpT<T> &, const T *, T *, T *, int, hipStream_t,  \
                                        const Batch &);                                                      \
    template void launch_block_rb_sweep2<T>(const Geom &, const BOpT<T> &, const T *, const T *, T *, bool,  \
                                            const Geom *, const T *, int64_t, hipStream_t, const Batch &);    \
    template void launch_block_rb_sweep2_restrict<T>(const Geom &, const BOpT<T> &, const T *, const T *, T *,  \
                                                     bool, const Geom &, T *, int64_t, hipStream_t,             \
                                                     const Batch &);                                            \
    template void launch_block_residual<T>(const Geom &, const BOpT<T> &, const T *, const T *, T *, bool,   \
                                           hipStream_t, const Batch &);                                      \
    template void launch_restrict3<T>(const Geom &, const T *, int64_t, const Geom &, T *, int64_t,          \
                                      hipStream_t, const Batch &);                                           \
    template void launch_residual_restrict<T>(const Geom &, const BOpT<T> &, const T *, const T *,          \
                                              const Geom &, T *, int64_t, hipStream_t, const Batch &);        \
    template void launch_prolong3<T>(const Geom &, T *, int64_t, const Geom &, const T *, int64_t,           \
                                     hipStream_t, const Batch &);                                            \
    template void launch_block_coarse_solve<T>(const Geom &, const BOpT<T> &, const T *, const T *, T *,     \
                                               hipStream_t, const Batch &);                                  \
    template void launch_block_subcycle<T>(const FusedLevelsT<T> &, hipStream_t, const Batch &);
MGF_INST(double)
MGF_INST(float)

}  // namespace mgf
