// Host side of the coupled Newton path (Sec. 2, Eq. 14): workspace layout,
// block V-cycle, restarted FGMRES (right preconditioned by one block
// V-cycle, weighted inner product), Newton iteration of one backward-Euler
// step, and the steady driver with the paper's time-step rule.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <new>
#include <vector>
#include <stdlib.h>

#include "mg_newton.h"

namespace mgf {

namespace {

int64_t plane_of(const Level &L) { return (int64_t)(L.g.nr + 1) * L.g.pitch; }

BOp bop(mg_ctx *c, int l) { return BOp{c->nw.lev[l].J, plane_of(c->lev[l])}; }

template <class T>
struct Prec;
template <>
struct Prec<double> {
    static BOpT<double> op(mg_ctx *c, int l) { return BOpT<double>{c->nw.lev[l].J, plane_of(c->lev[l])}; }
    static double *x(mg_ctx *c, int l) { return c->nw.lev[l].x; }
    static double *r(mg_ctx *c, int l) { return c->nw.lev[l].r; }
    static double *x2(mg_ctx *c, int l) { return c->nw.lev[l].x2; }
    static double *zt(mg_ctx *c, int l) { return c->nw.lev[l].zt; }
    static const double *inv(mg_ctx *c) { return c->nw.lev[c->nlev - 1].cinvT; }
};
template <>
struct Prec<float> {
    static BOpT<float> op(mg_ctx *c, int l) { return BOpT<float>{c->nw.lev[l].J32, plane_of(c->lev[l])}; }
    static float *x(mg_ctx *c, int l) { return c->nw.lev[l].x32; }
    static float *r(mg_ctx *c, int l) { return c->nw.lev[l].r32; }
    static float *x2(mg_ctx *c, int l) { return c->nw.lev[l].x2_32; }
    // the FP64 factor planes hold the FP32 ones (same plane stride in elements)
    static float *zt(mg_ctx *c, int l) { return reinterpret_cast<float *>(c->nw.lev[l].zt); }
    static const float *inv(mg_ctx *c) { return c->nw.lev[c->nlev - 1].cinvT32; }
};

// Field weights of the inner product: Poisson rows are scaled by 1/k so that
// all three equations are measured in density units.
double3 field_weights(const mg_physics *ph) {
    return make_double3(1.0, 1.0, ph->k > 0 ? 1.0 / ph->k : 1.0);
}

// nu collective red-black sweeps on level l: pairs of fused sweeps x -> x2 ->
// x, and two half-sweeps for an odd last one.  x_zero: x is zero on entry
// (the first fused sweep then does not read it).  xc (level l+1): the coarse
// correction still to be prolonged and added to x, which the first fused
// sweep does on the fly; the caller guarantees a fused sweep when x_zero or
// xc is set (fused_ok).
void join_factor(mg_ctx *c, hipStream_t s);

// Gram-Schmidt passes that form the previous pass's projections themselves
// pay on grids of at most chain_max_blocks workgroups (default 512;
// measured: 325 workgroups at 257x257 gain, several thousand at 1025x1025
// lose); single problems only, a batch's column sums cover all its problems
// in one launch.

template <class T>
bool fused_ok(mg_ctx *c, int nu) { return c->nw.rb_fused && nu >= 2; }
// Pairs of sweeps per launch on level l: every pre- and post-smoothing
// count even and the launch small enough to be latency-bound (nodes of all
// problems of a batch counted; larger launches are throughput-bound, where
// two one-sweep launches are faster).
bool sweep2_ok(const mg_ctx *c, int l) {
    const Geom &g = c->lev[l].g;
    return c->nw.rb_fused && (int64_t)(g.nr + 1) * (g.nz + 1) * c->bt.n <= c->nw.sweep2_max_nodes &&
           c->desc.nu1 >= 2 && c->desc.nu2 >= 2 && c->desc.nu1 % 2 == 0 && c->desc.nu2 % 2 == 0;
}
// Pre-smoothing alone in pairs (its last launch restricting the residual),
// post-smoothing one sweep per launch: levels above the two-sweep bound up
// to sweep2_pre_max_nodes, where the launch saved by the restriction pays
// for the slower two-sweep launch.
bool sweep2_pre_ok(const mg_ctx *c, int l) {
    const Geom &g = c->lev[l].g;
    return c->nw.rb_fused && c->nw.sweep2_restrict &&
           (int64_t)(g.nr + 1) * (g.nz + 1) * c->bt.n <= c->nw.sweep2_pre_max_nodes && c->desc.nu1 >= 2 &&
           c->desc.nu1 % 2 == 0 && c->desc.nu2 >= 2;
}

// Block zebra z-line smoothing selected (MG_SMOOTH_ZEBRA_BLOCK).
bool zebra_block(const mg_ctx *c) { return c->desc.smoother == MG_SMOOTH_ZEBRA_BLOCK; }

template <class T>
void block_smooth(mg_ctx *c, int l, const BOpT<T> &J, const T *f, T *x, int nu, bool x_zero, const T *xc,
                  hipStream_t s) {
    const Geom &g = c->lev[l].g;
    if (zebra_block(c)) {
        // nu zebra sweeps (even lines, then odd) on x, which holds the
        // iterate (written zero first when x_zero; a coarse correction xc is
        // added by its own launch)
        if (x_zero) launch_fill(x, 3 * plane_of(c->lev[l]), T(0), s, c->bt);
        if (xc) launch_prolong3<T>(g, x, plane_of(c->lev[l]), c->lev[l + 1].g, xc, plane_of(c->lev[l + 1]), s, c->bt);
        for (int k = 0; k < nu; ++k)
            for (int col = 0; col < 2; ++col) launch_block_zline<T>(g, J, f, x, Prec<T>::zt(c, l), col, s, c->bt);
        return;
    }
    int k = 0;
    if (fused_ok<T>(c, nu)) {
        T *x2 = Prec<T>::x2(c, l);
        const Geom *gc = xc ? &c->lev[l + 1].g : nullptr;
        const int64_t pc = xc ? plane_of(c->lev[l + 1]) : 0;
        for (; k + 2 <= nu; k += 2) {
            const bool first = k == 0;
            launch_block_rb_sweep<T>(g, J, f, x, x2, x_zero && first, first ? gc : nullptr, first ? xc : nullptr,
                                     pc, s, c->bt);
            launch_block_rb_sweep<T>(g, J, f, x2, x, false, nullptr, nullptr, 0, s, c->bt);
        }
    }
    for (; k < nu; ++k)
        for (int col = 0; col < 2; ++col) launch_block_rbgs<T>(g, J, f, x, col, s, c->bt);
}

// One block V(nu1, nu2) cycle for B x = f on level l from a zero initial
// guess; x is not read on entry (its electrode rows hold zeros).
template <class T>
void block_vcycle(mg_ctx *c, int l, const T *f, T *x, hipStream_t s) {
    const Level &L = c->lev[l];
    BOpT<T> J = Prec<T>::op(c, l);
    const bool zb = zebra_block(c);
    if (l == 0 && c->nw.smoother_only) {
        // relaxation only: nu1 + nu2 sweeps from zero (collective red-black,
        // or block zebra)
        const int nu = c->desc.nu1 + c->desc.nu2;
        const bool zs = zb || fused_ok<T>(c, nu);
        if (!zs) launch_fill(x, 3 * plane_of(L), T(0), s, c->bt);
        block_smooth<T>(c, 0, J, f, x, nu, zs, nullptr, s);
        return;
    }
    // (the block zebra smoother runs on every level above the coarsest, by
    // per-level launches)
    if (!zb && c->nw.fuse && L.g.nr <= c->nw.fuse_max && L.g.nz <= c->nw.fuse_max && c->nlev - l <= kMaxFused) {
        FusedLevelsT<T> F;
        memset(&F, 0, sizeof F);
        F.n = c->nlev - l;
        F.nu1 = c->desc.nu1;
        F.nu2 = c->desc.nu2;
        for (int q = 0; q < F.n; ++q) {
            F.g[q] = c->lev[l + q].g;
            F.J[q] = Prec<T>::op(c, l + q).base;
            F.plane[q] = plane_of(c->lev[l + q]);
            F.x[q] = (q == 0) ? x : Prec<T>::x(c, l + q);
            F.r[q] = Prec<T>::r(c, l + q);
        }
        F.f0 = f;
        F.invT = Prec<T>::inv(c);
        join_factor(c, s);
        launch_block_subcycle<T>(F, s, c->bt);
        return;
    }
    if (l == c->nlev - 1) {
        join_factor(c, s);
        launch_block_coarse_solve<T>(L.g, J, f, Prec<T>::inv(c), x, s, c->bt);
        return;
    }
    const Level &C = c->lev[l + 1];
    BOpT<T> Jc = Prec<T>::op(c, l + 1);
    T *fc = Jc.pl(kFe);
    T *xc = Prec<T>::x(c, l + 1);
    if (!zb && sweep2_ok(c, l)) {
        // sweeps in pairs, alternating between x and x2: the first from a zero
        // guess, the first post-smoothing pair adding the prolonged correction
        // as it stages its input; the buffer order makes the last pair land in x
        T *x2 = Prec<T>::x2(c, l);
        const int n1 = c->desc.nu1 / 2, n2 = c->desc.nu2 / 2;
        T *mid = (n2 & 1) ? x2 : x;  // iterate between pre- and post-smoothing
        auto other = [&](T *b) { return b == x ? x2 : x; };
        T *cur = (n1 & 1) ? mid : other(mid);
        // the last pre-smoothing launch also forms the restricted residual
        // (unless switched off: then its own launch)
        const bool fuse_r = c->nw.sweep2_restrict;
        for (int k = 0; k < n1; ++k) {
            const T *in = k == 0 ? nullptr : cur;
            T *out = k == 0 ? cur : other(cur);
            if (k == n1 - 1 && fuse_r)
                launch_block_rb_sweep2_restrict<T>(L.g, J, f, in, out, k == 0, C.g, fc, plane_of(C), s, c->bt);
            else
                launch_block_rb_sweep2<T>(L.g, J, f, in, out, k == 0, nullptr, nullptr, 0, s, c->bt);
            cur = out;
        }
        if (!fuse_r) launch_residual_restrict<T>(L.g, J, f, cur, C.g, fc, plane_of(C), s, c->bt);
        block_vcycle<T>(c, l + 1, fc, xc, s);
        for (int k = 0; k < n2; ++k) {
            const bool first = k == 0;
            launch_block_rb_sweep2<T>(L.g, J, f, cur, other(cur), false, first ? &C.g : nullptr,
                                      first ? xc : nullptr, plane_of(C), s, c->bt);
            cur = other(cur);
        }
        return;
    }
    if (!zb && sweep2_pre_ok(c, l)) {
        // pre-smoothing in pairs landing in x (the first from a zero guess,
        // the last restricting the residual), post-smoothing one sweep per
        // launch from x (the first adding the prolonged correction)
        T *x2 = Prec<T>::x2(c, l);
        const int n1 = c->desc.nu1 / 2;
        T *cur = (n1 & 1) ? x : x2;
        for (int k = 0; k < n1; ++k) {
            const T *in = k == 0 ? nullptr : cur;
            T *out = k == 0 ? cur : (cur == x ? x2 : x);
            if (k == n1 - 1)
                launch_block_rb_sweep2_restrict<T>(L.g, J, f, in, out, k == 0, C.g, fc, plane_of(C), s, c->bt);
            else
                launch_block_rb_sweep2<T>(L.g, J, f, in, out, k == 0, nullptr, nullptr, 0, s, c->bt);
            cur = out;
        }
        block_vcycle<T>(c, l + 1, fc, xc, s);
        block_smooth<T>(c, l, J, f, x, c->desc.nu2, false, xc, s);
        return;
    }
    // without a fused first sweep the zero guess has to be written
    const bool zero_sweep = zb || fused_ok<T>(c, c->desc.nu1);
    if (!zero_sweep) launch_fill(x, 3 * plane_of(L), T(0), s, c->bt);
    block_smooth<T>(c, l, J, f, x, c->desc.nu1, zero_sweep, nullptr, s);
    if (c->nw.rb_fused) {
        launch_residual_restrict<T>(L.g, J, f, x, C.g, fc, plane_of(C), s, c->bt);
    } else {
        T *r = Prec<T>::r(c, l);
        launch_block_residual<T>(L.g, J, f, x, r, false, s, c->bt);
        launch_restrict3<T>(L.g, r, plane_of(L), C.g, fc, plane_of(C), s, c->bt);
    }
    block_vcycle<T>(c, l + 1, fc, xc, s);
    // the coarse-grid correction: added by the first post-smoothing sweep, or
    // by its own launch
    if (fused_ok<T>(c, c->desc.nu2)) {
        block_smooth<T>(c, l, J, f, x, c->desc.nu2, false, xc, s);
    } else {
        launch_prolong3<T>(L.g, x, plane_of(L), C.g, xc, plane_of(C), s, c->bt);
        block_smooth<T>(c, l, J, f, x, c->desc.nu2, false, nullptr, s);
    }
}

// Assemble the Jacobian on every level: level 0 at the current state with
// the Newton right-hand side; coarser levels at the injected state.
static_assert(kMaxLevTab >= kMaxLevels, "one level-table launch covers the hierarchy");

void assemble_all(mg_ctx *c, const mg_physics *ph, const mg_state *st, double dt_inv) {
    hipStream_t s = c->stream;
    NewtonPhys np_;
    np_.qe = ph->mu_e / ph->D_e;   // -s mu/D with s = -1
    np_.qp = -ph->mu_p / ph->D_p;  // s = +1
    np_.De = ph->D_e;
    np_.Dp = ph->D_p;
    np_.k = ph->k;
    np_.dt_inv = dt_inv;
    const double *snap = c->nw.snap;
    int64_t p0 = plane_of(c->lev[0]);
    NodeTransport tr;
    tr.mue = st->mue;
    tr.De = st->De;
    tr.mup = st->mup;
    tr.Dp = st->Dp;
    launch_newton_assemble(c->lev[0].g, bop(c, 0), st->V, st->ne, st->np, snap + p0, snap + 2 * p0, st->Se,
                           st->Sp, np_, true, s, static_cast<const NewtonPhys *>(c->php_dev), c->bt, tr);
    if (c->nlev > 1) {
        // every coarser level at once, each at the finest state injected to it
        LevTab t;
        t.n = c->nlev - 1;
        for (int l = 1; l < c->nlev; ++l) {
            t.shift[l - 1] = l;
            t.g[l - 1] = c->lev[l].g;
            t.J[l - 1] = bop(c, l);
        }
        launch_newton_assemble_coarse(t, st->V, st->ne, st->np, c->lev[0].g.pitch, np_, s,
                                      static_cast<const NewtonPhys *>(c->php_dev), c->bt, tr);
    }
    if (c->nw.prec32) {
        // FP32 copies of every level's Jacobian (the coarsest inverse's copy
        // follows its factorisation, coarse_factor)
        LevTab t;
        t.n = c->nlev;
        for (int l = 0; l < c->nlev; ++l) {
            t.shift[l] = l;
            t.g[l] = c->lev[l].g;
            t.J[l] = bop(c, l);
            t.J32[l] = BOpT<float>{c->nw.lev[l].J32, plane_of(c->lev[l])};
        }
        launch_block_to_f32_levels(t, s, c->bt);
    }
}

// Explicit inverse of the coarsest Jacobian (and its FP32 copy) on stream s.
void coarse_factor(mg_ctx *c, hipStream_t s) {
    const Level &Lc = c->lev[c->nlev - 1];
    launch_block_coarse_factor(Lc.g, bop(c, c->nlev - 1), c->nw.scratch, c->nw.lev[c->nlev - 1].cinvT, s, c->bt);
    if (c->nw.prec32) {
        int64_t n = 3 * (int64_t)(Lc.g.nr + 1) * (Lc.g.nz - 1);
        launch_planes_to_f32(c->nw.lev[c->nlev - 1].cinvT, c->nw.lev[c->nlev - 1].cinvT32, n * n, s, c->bt);
    }
}

// Stream s waits for the coarsest factorisation if it is still a pending
// branch (the first V-cycle after a fork reaches the coarse end).
void join_factor(mg_ctx *c, hipStream_t s) {
    if (!c->nw.join_pending) return;
    (void)hipStreamWaitEvent(s, c->nw.evf[1], 0);
    c->nw.join_pending = false;
}

// Givens-rotation least squares of the Arnoldi relation (host, small).
struct Arnoldi {
    int m;
    double H[kMaxKrylov + 1][kMaxKrylov];
    double cs[kMaxKrylov], sn[kMaxKrylov], g[kMaxKrylov + 1];
    void start(double beta) {
        memset(g, 0, sizeof g);
        g[0] = beta;
    }
    // column k is in H[0..k+1][k]; returns the residual-norm estimate
    double add(int k) {
        for (int i = 0; i < k; ++i) {
            double a = H[i][k], b = H[i + 1][k];
            H[i][k] = cs[i] * a + sn[i] * b;
            H[i + 1][k] = -sn[i] * a + cs[i] * b;
        }
        double a = H[k][k], b = H[k + 1][k];
        double r = hypot(a, b);
        cs[k] = r > 0 ? a / r : 1.0;
        sn[k] = r > 0 ? b / r : 0.0;
        H[k][k] = r;
        H[k + 1][k] = 0.0;
        g[k + 1] = -sn[k] * g[k];
        g[k] = cs[k] * g[k];
        return fabs(g[k + 1]);
    }
    void solve(int k, double *y) {  // upper triangular H[0..k-1][0..k-1] y = g
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int t = i + 1; t < k; ++t) s -= H[i][t] * y[t];
            y[i] = s / H[i][i];
        }
    }
};

// A batch context (any number of problems, one included) reads its Arnoldi
// columns from the batch readback buffer.
bool is_batch(const mg_ctx *c) { return c->bpinned != nullptr; }

// Whether the Arnoldi step chains its Gram-Schmidt passes (a single-problem
// context, a grid of few workgroups): then the host sums the second pass's
// partials.
bool chained_cgs(const mg_ctx *c) {
    const int nb = block_vec_blocks(c->lev[0].g);
    return !is_batch(c) && nb <= c->nw.chain_max_blocks && nb <= kChainCap;
}

// Column v of the nblk x nd workgroup partials, summed as the kernels'
// chained reduction sums it: 64 running sums (partial b into sum b mod 64,
// in increasing b), then pairwise at distances 32, 16, ..., 1; the sum that
// ends in slot 0.
double host_column_sum(const double *part, int nblk, int nd, int v) {
    double a[64];
    for (int l = 0; l < 64; ++l) a[l] = 0.0;
    for (int b = 0; b < nblk; ++b) a[b & 63] += part[(int64_t)b * nd + v];
    for (int off = 32; off > 0; off >>= 1) {
        double t[64];
        for (int l = 0; l < 64; ++l) t[l] = a[l] + a[l ^ off];
        for (int l = 0; l < 64; ++l) a[l] = t[l];
    }
    return a[0];
}

// Hessenberg subdiagonal from nu^2 = (w', w') - |h2|^2: a value rounded
// below zero (w' inside the basis to working precision) is a breakdown,
// zero; a non-finite one stays non-finite.
double subdiag(double nu2) { return nu2 < 0.0 ? 0.0 : sqrt(nu2); }

// Copy `count` device doubles at `dev` of every problem of the batch to
// host[p * count ...] (one strided copy).
void readback(mg_ctx *c, double *host, const double *dev, int count, hipStream_t s) {
    if (c->bt.n <= 1)
        (void)hipMemcpyAsync(host, dev, count * sizeof(double), hipMemcpyDeviceToHost, s);
    else
        (void)hipMemcpy2DAsync(host, count * sizeof(double), dev, (size_t)c->bt.stride, count * sizeof(double),
                               (size_t)c->bt.n, hipMemcpyDeviceToHost, s);
}

// One Arnoldi step k.  Basis slot k holds u_k: v_0 for k = 0, otherwise the
// vector w' of step k-1, from which one projection has been removed.
//   z_k = M u_k (block V-cycle; flexible GMRES admits any z_k, J Z = V H is
//         what the least-squares update needs);
//   pass 1: slot k := v_k = (u_k - V_{<k} h2) / nu_k, the second projection
//           and the normalisation deferred from step k-1; w = J z_k and
//           h1 = V_{<=k}^T w;
//   pass 2: w' = w - V h1 into slot k+1, partial sums of h2 = V^T w' and
//           (w', w');
//   their sums and nu_{k+1}^2 = (w', w') - |h2|^2 (Pythagoras: v_{k+1}
//           would be (w' - V h2) / nu_{k+1}).
// The Hessenberg column is h1 + h2 with subdiagonal nu_{k+1}, the column two
// full classical Gram-Schmidt passes give, with one pass over the basis
// fewer per step, and two launches instead of four on chained grids (the
// sums of pass 2 are formed by the next step's pass 1 and by the host).
// h1 goes to the device scalars [0..k]; on large grids and for batches h2
// and nu^2 too ([m+1..m+1+k], [2m+2]).  A single problem's values go
// straight to one of two pinned slots (step k+1 can run while the host
// reads step k): h1 and, on chained grids, pass 2's partials, otherwise
// h2 and nu^2; a batch's are copied afterwards.
void arnoldi_step(mg_ctx *c, int k, double3 cw, hipStream_t s) {
    NewtonWork &W = c->nw;
    const Level &L0 = c->lev[0];
    const Geom &g = L0.g;
    int64_t p0 = plane_of(L0), vs = 3 * p0;
    BOp J = bop(c, 0);
    const int m = W.m;
    double *dev = W.dev;
    double *uk = W.V + k * vs, *zk = W.Z + k * vs, *uk1 = W.V + (k + 1) * vs;
    if (k == 0) {
        // the coarsest factorisation (of the Jacobian assembled before this
        // solve) overlaps the fine-level part of the first V-cycle
        (void)hipEventRecord(W.evf[0], s);
        (void)hipStreamWaitEvent(W.side, W.evf[0], 0);
        coarse_factor(c, W.side);
        (void)hipEventRecord(W.evf[1], W.side);
        W.join_pending = true;
    }
    if (W.prec32) {
        // preconditioner in FP32: z_k = M32 u_k (the Krylov space stays FP64)
        float *x32 = W.lev[0].x32;
        launch_planes_to_f32(uk, W.f32, vs, s, c->bt);
        block_vcycle<float>(c, 0, W.f32, x32, s);
        launch_planes_to_f64(x32, zk, vs, s, c->bt);
    } else {
        block_vcycle<double>(c, 0, uk, zk, s);
    }
    join_factor(c, s);  // (already joined by the V-cycle's coarse end)
    CgsLag fin;
    if (k > 0) {
        fin.fin_h = dev + m + 1;
        fin.fin_nu2 = dev + 2 * m + 2;
        fin.fin_out = uk;
    }
    CgsLag l2;
    l2.next = uk1;
    l2.with_norm = 1;
    // Every workgroup of a chained pass reads all partials of the previous
    // one: pass 2 those of pass 1, and pass 1 those of the previous step's
    // pass 2, which the host sums too from its pinned copy (the same order,
    // the same bits).  Large grids (many workgroups) and batches sum them in
    // launches of their own.
    double *P0 = W.partials, *P1 = W.partials2;
    if (chained_cgs(c)) {
        double *host = c->pinned_dev + kSlot * (k & 1);
        if (k > 0) {
            fin.fin_h = fin.fin_nu2 = nullptr;
            fin.fin_part = P1;
            fin.fin_nblk = block_vec_blocks(g);
        }
        l2.part_host = c->pinned_dev + 512 + kPartSlot * (k & 1);
        launch_cgs_pass(g, W.w, W.V, vs, k + 1, p0, cw, nullptr, false, P0, nullptr, s, c->bt, &J, zk, fin);
        launch_cgs_pass_chained(g, W.w, W.V, vs, k + 1, p0, cw, false, P0, dev, host, P1, s, c->bt, l2);
        return;
    }
    launch_cgs_pass(g, W.w, W.V, vs, k + 1, p0, cw, nullptr, false, P0, dev, s, c->bt, &J, zk, fin);
    launch_cgs_pass(g, W.w, W.V, vs, k + 1, p0, cw, dev, false, P0, dev + (m + 1), s, c->bt, nullptr, nullptr, l2);
    launch_lagged_nu2(dev + (m + 1), k + 1, dev + 2 * m + 2, nullptr, s, c->bt);
    readback(c, is_batch(c) ? c->bpinned : c->pinned + kSlot * (k & 1), dev, 2 * m + 3, s);
}

int run_arnoldi(mg_ctx *c, int k, double3 cw);

// Launch Arnoldi step k (run_arnoldi) and record the event that marks its
// readback.
int launch_step(mg_ctx *c, int k, double3 cw) {
    NewtonWork &W = c->nw;
    if (!W.ev[0]) {
        HIP_OK(hipEventCreateWithFlags(&W.ev[0], hipEventDisableTiming));
        HIP_OK(hipEventCreateWithFlags(&W.ev[1], hipEventDisableTiming));
    }
    if (int e = run_arnoldi(c, k, cw)) return e;
    HIP_OK(hipEventRecord(W.ev[k & 1], c->stream));
    return MG_OK;
}

// Run Arnoldi step k on the context stream, from a captured graph when
// graphs are enabled (captured on a private stream at first use; a change
// of the inner-product weights recaptures).
int run_arnoldi(mg_ctx *c, int k, double3 cw) {
    NewtonWork &W = c->nw;
    if (!W.side) {  // created outside any capture
        HIP_OK(hipStreamCreateWithFlags(&W.side, hipStreamNonBlocking));
        HIP_OK(hipEventCreateWithFlags(&W.evf[0], hipEventDisableTiming));
        HIP_OK(hipEventCreateWithFlags(&W.evf[1], hipEventDisableTiming));
    }
    if (!W.use_graphs) {
        arnoldi_step(c, k, cw, c->stream);
        return MG_OK;
    }
    if (W.cw_cap[0] != cw.x || W.cw_cap[1] != cw.y || W.cw_cap[2] != cw.z) {
        for (int t = 0; t < 64; ++t)
            if (W.exec[t]) {
                (void)hipGraphExecDestroy(W.exec[t]);
                W.exec[t] = nullptr;
            }
        W.cw_cap[0] = cw.x;
        W.cw_cap[1] = cw.y;
        W.cw_cap[2] = cw.z;
    }
    if (!W.cap) HIP_OK(hipStreamCreateWithFlags(&W.cap, hipStreamNonBlocking));
    if (!W.exec[k]) {
        hipGraph_t graph = nullptr;
        HIP_OK(hipStreamBeginCapture(W.cap, hipStreamCaptureModeThreadLocal));
        arnoldi_step(c, k, cw, W.cap);
        HIP_OK(hipStreamEndCapture(W.cap, &graph));
        hipError_t e = hipGraphInstantiate(&W.exec[k], graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            W.exec[k] = nullptr;
            return fail(MG_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
        }
    }
    HIP_OK(hipGraphLaunch(W.exec[k], c->stream));
    return MG_OK;
}

// Solve J delta = b (b = the Newton right-hand side planes of level 0) to
// weighted relative residual rtol.  Returns the iteration count in *its.
// Step k+1 is launched before the host has read step k when the residual
// estimates predict that step k will not converge (or, for k = 0, when the
// previous solve needed more than one step): the GPU then never waits for
// the host's Givens update, at the price of a discarded step when the
// prediction fails.
int fgmres(mg_ctx *c, const mg_physics *ph, double rtol, int maxit, int *its, double *relres) {
    hipStream_t s = c->stream;
    NewtonWork &W = c->nw;
    const Level &L0 = c->lev[0];
    const Geom &g = L0.g;
    int64_t p0 = plane_of(L0), vs = 3 * p0;
    BOp J = bop(c, 0);
    const double *b = J.pl(kFe);
    double3 cw = field_weights(ph);
    double *dev = W.dev;  // [0..m] dots, [m+1..2m+1] second pass, [2m+2] norm^2, y at [3m+8..]
    const int m = W.m;
    double *ybuf = c->pinned + 2 * kSlot, *sbuf = c->pinned + 2 * kSlot + kMaxKrylov + 8;
    const bool chained = chained_cgs(c);
    const int nblk = block_vec_blocks(g);
    Arnoldi A;
    launch_fill(W.delta, vs, 0.0, s);
    // r0 = b; its norm goes to pinned memory and is read with the first
    // Arnoldi step's readback, so no host round trip precedes that step (a
    // zero or non-finite norm is acted on then)
    launch_cgs_pass(g, const_cast<double *>(b), b, vs, 1, p0, cw, nullptr, true, W.partials, dev, s);
    HIP_OK(hipMemcpyAsync(sbuf, dev, sizeof(double), hipMemcpyDeviceToHost, s));
    launch_scale_by_norm(g, b, W.V, p0, dev, s);
    *its = 0;
    *relres = 0.0;
    double beta0 = -1.0, beta = -1.0;
    int total = 0;
    const int prev = W.last_its;
    while (true) {
        if (beta0 >= 0) A.start(beta);
        int k = 0;
        double est = beta, est_prev = beta;
        bool next_launched = false;
        if (int e = launch_step(c, 0, cw)) return e;
        for (; k < m && total < maxit; ++k) {
            // speculative launch of step k+1
            bool more = k + 1 < m && total + 1 < maxit;
            if (more) {
                bool spec;
                if (k == 0)
                    spec = prev != 1;
                else {
                    double pred = est * (est / est_prev);
                    spec = pred > 1.5 * rtol * beta0;
                }
                next_launched = spec;
                if (spec)
                    if (int e = launch_step(c, k + 1, cw)) return e;
            } else {
                next_launched = false;
            }
            HIP_OK(hipEventSynchronize(W.ev[k & 1]));
            if (beta0 < 0) {
                // first step of the solve: the norm of r0 is in sbuf by now
                beta0 = beta = sqrt(sbuf[0]);
                if (!(beta0 > 0)) {
                    HIP_OK(hipStreamSynchronize(s));  // drain a speculative step
                    if (!isfinite(beta0)) return fail(MG_ENONFINITE, "Newton residual is not finite");
                    return MG_OK;  // b = 0: delta = 0
                }
                A.start(beta0);
                est = est_prev = beta0;
            }
            const double *host = c->pinned + kSlot * (k & 1);
            if (chained) {
                // second projections and (w', w') from the pinned partials of pass 2
                const double *pp = c->pinned + 512 + kPartSlot * (k & 1);
                double h2[kMaxKrylov + 1];
                for (int i = 0; i <= k + 1; ++i) h2[i] = host_column_sum(pp, nblk, k + 2, i);
                double nu2 = h2[k + 1];
                for (int i = 0; i <= k; ++i) nu2 = fma(-h2[i], h2[i], nu2);
                for (int i = 0; i <= k; ++i) A.H[i][k] = host[i] + h2[i];
                A.H[k + 1][k] = subdiag(nu2);
            } else {
                for (int i = 0; i <= k; ++i) A.H[i][k] = host[i] + host[m + 1 + i];
                A.H[k + 1][k] = subdiag(host[2 * m + 2]);
            }
            ++total;
            c->vcycles++;
            est_prev = est;
            est = A.add(k);
            if (!isfinite(est)) {
                HIP_OK(hipStreamSynchronize(s));
                return fail(MG_ENONFINITE, "FGMRES breakdown (non-finite)");
            }
            if (est <= rtol * beta0 || A.H[k][k] == 0.0) {
                ++k;
                break;
            }
            if (more && !next_launched)
                if (int e = launch_step(c, k + 1, cw)) return e;
        }
        double y[kMaxKrylov];
        A.solve(k, y);
        for (int i = 0; i < k; ++i) ybuf[i] = y[i];
        HIP_OK(hipMemcpyAsync(dev + 3 * m + 8, ybuf, k * sizeof(double), hipMemcpyHostToDevice, s));
        launch_axpy_multi(g, W.delta, W.Z, vs, k, p0, dev + 3 * m + 8, 1.0, s);
        *its = total;
        W.last_its = total;
        if (est <= rtol * beta0) {
            // converged by the recurrence's residual (that of the iterate in
            // exact arithmetic): no true-residual round trip; the caller's
            // next synchronisation covers the update
            *relres = est / beta0;
            return MG_OK;
        }
        // true residual for the restart / final check
        launch_block_residual<double>(g, J, b, W.delta, W.w, false, s);
        launch_cgs_pass(g, W.w, W.w, vs, 1, p0, cw, nullptr, true, W.partials, dev, s);
        HIP_OK(hipMemcpyAsync(sbuf, dev, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        beta = sqrt(sbuf[0]);
        *relres = beta / beta0;
        if (!isfinite(beta)) return fail(MG_ENONFINITE, "FGMRES residual is not finite");
        if (beta <= rtol * beta0 * 1.0000001) return MG_OK;
        if (total >= maxit)
            return fail(MG_ENOCONV, "FGMRES: relative residual %.3e after %d iterations", beta / beta0, total);
        launch_scale_by_norm(g, W.w, W.V, p0, dev, s);
    }
}

void copy_state(mg_ctx *c, const mg_state *st, double *dst) {
    const Level &L0 = c->lev[0];
    int64_t p0 = plane_of(L0);
    launch_copy_field(L0.g, st->V, dst, c->stream, c->bt);
    launch_copy_field(L0.g, st->ne, dst + p0, c->stream, c->bt);
    launch_copy_field(L0.g, st->np, dst + 2 * p0, c->stream, c->bt);
}

void restore_state(mg_ctx *c, const double *src, mg_state *st) {
    const Level &L0 = c->lev[0];
    int64_t p0 = plane_of(L0);
    launch_copy_field(L0.g, src, st->V, c->stream, c->bt);
    launch_copy_field(L0.g, src + p0, st->ne, c->stream, c->bt);
    launch_copy_field(L0.g, src + 2 * p0, st->np, c->stream, c->bt);
}

void launch_step_change(mg_ctx *c, const mg_state *st, double *out);

// Newton iterations of one BE step; the step's starting state is in W.snap.
// With `change`, every iteration also forms the step's relative density
// change against W.snap (launch_step_change) and reads it back with the
// Newton reduction; *change is set when the step converges.
int newton_iterate(mg_ctx *c, const mg_physics *ph, mg_state *st, double dt, const mg_schedule *sc,
                   mg_report *rep, bool *converged, double *change = nullptr) {
    hipStream_t s = c->stream;
    const Level &L0 = c->lev[0];
    int64_t p0 = plane_of(L0);
    double dt_inv = (dt > 0 && isfinite(dt)) ? 1.0 / dt : 0.0;
    *converged = false;
    int maxn = sc->max_newton > 0 ? sc->max_newton : 10;
    for (int it = 1; it <= maxn; ++it) {
        assemble_all(c, ph, st, dt_inv);
        int its = 0;
        double rr = 0;
        int e = fgmres(c, ph, sc->lin_rtol, sc->max_cycles > 0 ? sc->max_cycles : 200, &its, &rr);
        if (rep) {
            rep->final_relres = rr;
            rep->newton_its += 1;
            rep->vcycles += its;
        }
        if (e == MG_ENOCONV || e == MG_ENONFINITE) return MG_OK;  // step fails: caller rejects
        if (e) return e;
        launch_newton_update(L0.g, st->V, st->ne, st->np, c->nw.delta, p0, c->nw.partials, c->scal, s);
        if (change) launch_step_change(c, st, c->scal + 8);
        HIP_OK(hipMemcpyAsync(c->pinned, c->scal, (change ? 12 : 8) * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        const double *o = c->pinned;
        double re = o[0] / fmax(o[1], 1e-300), rp = o[2] / fmax(o[3], 1e-300), rv = o[4] / fmax(o[5], 1e-300);
        double mx = fmax(re, fmax(rp, rv));
        if (rep) rep->last_change = mx;  // size of the last Newton correction
        if (!isfinite(mx)) return MG_OK;
        if (mx > sc->reject_limit) return MG_OK;
        if (mx < sc->newton_tol) {
            // the converged densities must be non-negative to rounding
            double cnt = (double)(L0.g.nr + 1) * (L0.g.nz - 1);
            *converged = o[6] >= -1e-10 * o[1] / cnt && o[7] >= -1e-10 * o[3] / cnt;
            if (change) *change = fmax(sqrt(o[8] / fmax(o[9], 1e-300)), sqrt(o[10] / fmax(o[11], 1e-300)));
            return MG_OK;
        }
    }
    return MG_OK;
}

// ||n - n^k||_2^2 and ||n||_2^2 of both species against the snapshot, to
// out[0..3] (device).
void launch_step_change(mg_ctx *c, const mg_state *st, double *out) {
    const Level &L0 = c->lev[0];
    int64_t p0 = plane_of(L0);
    hipStream_t s = c->stream;
    int nb = 0;
    launch_diff_norms(L0.g, st->ne, c->nw.snap + p0, c->partials, &nb, s);
    launch_sum_partials(c->partials, nb, 2, out, s);
    launch_diff_norms(L0.g, st->np, c->nw.snap + 2 * p0, c->partials, &nb, s);
    launch_sum_partials(c->partials, nb, 2, out + 2, s);
}

}  // namespace

void carve_newton(mg_ctx *c, const mg_grid_desc *d, Carver &cv, int nl) {
    int m = d->krylov_m;
    if (c) c->nw.m = m;
    if (m <= 0) return;
    int64_t p0 = 0;
    for (int l = 0; l < nl; ++l) {
        int nr = d->nr >> l, nz = d->nz >> l;
        int64_t pitch = round_up(nz + 1, 16);
        int64_t pl = (int64_t)(nr + 1) * pitch;
        if (l == 0) p0 = pl;
        BLevel B;
        memset(&B, 0, sizeof B);
        B.J = cv.take<double>(kBPlanes * pl);
        B.x = cv.take<double>(3 * pl);
        B.x2 = cv.take<double>(3 * pl);
        B.r = cv.take<double>(3 * pl);
        if (d->smoother == MG_SMOOTH_ZEBRA_BLOCK) B.zt = cv.take<double>(12 * pl);
        bool p32 = d->prec == MG_FP32_IR;
        if (p32) {
            B.J32 = cv.take<float>(kBPlanes * pl);
            B.x32 = cv.take<float>(3 * pl);
            B.x2_32 = cv.take<float>(3 * pl);
            B.r32 = cv.take<float>(3 * pl);
        }
        if (l == nl - 1) {
            int64_t n = 3 * (int64_t)(nr + 1) * (nz - 1);
            B.cinvT = cv.take<double>(n * n);
            if (p32) B.cinvT32 = cv.take<float>(n * n);
            double *scr = cv.take<double>(n * 2 * n);
            if (c) c->nw.scratch = scr;
        }
        if (c) c->nw.lev[l] = B;
    }
    double *V = cv.take<double>((int64_t)(m + 1) * 3 * p0);
    double *Z = cv.take<double>((int64_t)m * 3 * p0);
    double *w = cv.take<double>(3 * p0);
    double *delta = cv.take<double>(3 * p0);
    double *snap = cv.take<double>(3 * p0);
    int nblk = ((d->nz + 1 + 63) / 64) * (d->nr + 1);  // one row per workgroup at most
    double *part = cv.take<double>((int64_t)nblk * (m + 2) + (int64_t)nblk * 8 + 64);
    double *part2 = cv.take<double>((int64_t)nblk * (m + 2) + 64);
    double *dev = cv.take<double>(4 * kMaxKrylov + 64);
    float *f32 = (d->prec == MG_FP32_IR) ? cv.take<float>(3 * p0) : nullptr;
    if (c) {
        c->nw.f32 = f32;
        c->nw.prec32 = d->prec == MG_FP32_IR;
        c->nw.V = V;
        c->nw.Z = Z;
        c->nw.w = w;
        c->nw.delta = delta;
        c->nw.snap = snap;
        c->nw.partials = part;
        c->nw.partials2 = part2;
        c->nw.dev = dev;
    }
}

int newton_implicit_step(mg_ctx *c, const mg_physics *ph, mg_state *st, double dt, const mg_schedule *sc,
                         mg_report *rep, bool *converged) {
    if (c->nw.m <= 0) return fail(MG_EINVAL, "context built with krylov_m = 0: no Newton workspace");
    const Level &L0 = c->lev[0];
    set_boundary(L0.g, st->V, st->ne, st->np, *ph, c->stream);
    copy_state(c, st, c->nw.snap);
    int e = newton_iterate(c, ph, st, dt, sc, rep, converged);
    if (e) return e;
    if (rep) rep->steps += 1;
    return MG_OK;
}

int newton_solve_steady(mg_ctx *c, const mg_physics *ph, mg_state *st, const mg_schedule *sc, mg_report *rep) {
    if (c->nw.m <= 0) return fail(MG_EINVAL, "context built with krylov_m = 0: no Newton workspace");
    auto t0 = std::chrono::steady_clock::now();
    mg_report local;
    memset(&local, 0, sizeof local);
    mg_report *R = rep ? rep : &local;
    memset(R, 0, sizeof *R);
    const Level &L0 = c->lev[0];
    set_boundary(L0.g, st->V, st->ne, st->np, *ph, c->stream);
    double dt = sc->dt0, dt_acc = 0.0, t = 0.0;
    int consecutive_rejects = 0;
    int status = MG_ENOCONV;
    while (R->steps < sc->max_steps) {
        copy_state(c, st, c->nw.snap);
        bool ok = false;
        double ch = 0;
        int e = newton_iterate(c, ph, st, dt, sc, R, &ok, &ch);
        if (e) return e;
        if (!ok) {
            restore_state(c, c->nw.snap, st);
            R->rejected++;
            if (++consecutive_rejects > 60) {
                status = fail(MG_EREJECT, "time step rejected %d times in a row (dt = %.3e)", consecutive_rejects, dt);
                break;
            }
            // retry with the last accepted step (Sec. 2), then halve
            dt = (dt_acc > 0 && dt > dt_acc) ? dt_acc : 0.5 * dt;
            continue;
        }
        consecutive_rejects = 0;
        R->steps++;
        t += dt;
        R->last_change = ch;  // relative density change of the step (Sec. 2 stop rule)
        if (!isfinite(ch)) {
            status = fail(MG_ENONFINITE, "density change is not finite");
            break;
        }
        dt_acc = dt;
        if (ch < sc->steady_tol) {
            status = MG_OK;
            break;
        }
        dt = fmin(sc->growth * dt, sc->dt_max);
    }
    R->t_end = t;
    R->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (status == MG_ENOCONV) fail(MG_ENOCONV, "not steady after %d steps (change %.3e)", R->steps, R->last_change);
    return status;
}


// ===========================================================================
// Batches of same-shape problems (one size class of a parameter sweep).
// Every problem owns an equal-stride region of the workspace (solver
// workspace + its five state fields); kernels index the problem by
// blockIdx.z and skip problems whose active flag is 0, so one launch
// advances the whole batch.  Time stepping, Newton and FGMRES run in
// lockstep with per-problem control on the host: each problem keeps its
// own dt, step count, Krylov recurrence and convergence decisions.
// ===========================================================================
namespace {

struct BatchRun {
    int n;
    std::vector<int> act;   // host copy of the active flags
};

// Upload the active flags through the next pinned slot.  The host waits for
// the copy that last used that slot (recorded event) before rewriting it.
int set_active(mg_ctx *c, const std::vector<int> &act) {
    int k = c->active_seq++ % kActiveSlots;
    if (c->active_ev_used[k]) HIP_OK(hipEventSynchronize(c->active_ev[k]));
    int *slot = c->active_host + (size_t)k * c->bt.n;
    for (int p = 0; p < c->bt.n; ++p) slot[p] = act[p];
    HIP_OK(hipMemcpyAsync((void *)c->bt.active, slot, c->bt.n * sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIP_OK(hipEventRecord(c->active_ev[k], c->stream));
    c->active_ev_used[k] = true;
    return MG_OK;
}

int any_of(const std::vector<int> &v) {
    for (int x : v)
        if (x) return 1;
    return 0;
}

// Upload y coefficients (k per problem, zero-padded to kmax) into each
// problem's device scalars at offset `off`.
int upload_per_problem(mg_ctx *c, const std::vector<double> &vals, int count, double *dev_at) {
    int n = c->bt.n;
    double *h = c->bpinned;
    for (int p = 0; p < n; ++p)
        for (int i = 0; i < count; ++i) h[p * count + i] = vals[(size_t)p * count + i];
    HIP_OK(hipMemcpy2DAsync(dev_at, (size_t)c->bt.stride, h, count * sizeof(double), count * sizeof(double),
                            (size_t)n, hipMemcpyHostToDevice, c->stream));
    return MG_OK;
}

// Lockstep FGMRES over the problems with act[p] = 1.  ok[p] = 1 when the
// problem's weighted relative residual reached rtol.
int fgmres_batch(mg_ctx *c, double3 cw, double rtol, int maxit, const std::vector<int> &act,
                 std::vector<int> &ok, std::vector<int> &its) {
    hipStream_t s = c->stream;
    NewtonWork &W = c->nw;
    const int n = c->bt.n, m = W.m;
    const Level &L0 = c->lev[0];
    const Geom &g = L0.g;
    int64_t p0 = plane_of(L0), vs = 3 * p0;
    BOp J = bop(c, 0);
    const double *b = J.pl(kFe);
    double *dev = W.dev;
    double *host = c->bpinned;
    std::vector<Arnoldi> A(n);
    std::vector<double> beta0(n, 0.0), beta(n, 0.0), est(n, 0.0);
    std::vector<int> live = act, kp(n, 0);
    ok.assign(n, 0);
    its.assign(n, 0);
    int e = set_active(c, live);
    if (e) return e;
    launch_fill(W.delta, vs, 0.0, s, c->bt);
    launch_cgs_pass(g, const_cast<double *>(b), b, vs, 1, p0, cw, nullptr, true, W.partials, dev, s, c->bt);
    readback(c, host, dev, 1, s);
    HIP_OK(hipStreamSynchronize(s));
    for (int p = 0; p < n; ++p) {
        if (!live[p]) continue;
        beta0[p] = beta[p] = sqrt(host[p]);
        if (!(beta0[p] > 0)) {  // zero right-hand side: delta = 0 is exact
            ok[p] = isfinite(beta0[p]) ? 1 : 0;
            live[p] = 0;
        }
    }
    if ((e = set_active(c, live))) return e;
    launch_scale_by_norm(g, b, W.V, p0, dev, s, c->bt);
    std::vector<int> cycle_act;
    while (any_of(live)) {
        for (int p = 0; p < n; ++p)
            if (live[p]) A[p].start(beta[p]);
        cycle_act = live;  // problems taking part in this restart cycle
        std::vector<int> iter = live;
        int kmax = 0;
        for (int k = 0; k < m && any_of(iter); ++k) {
            if ((e = set_active(c, iter))) return e;
            if ((e = run_arnoldi(c, k, cw))) return e;
            HIP_OK(hipStreamSynchronize(s));
            kmax = k + 1;
            for (int p = 0; p < n; ++p) {
                if (!iter[p]) continue;
                const double *hp = host + (size_t)p * (2 * m + 3);
                for (int i = 0; i <= k; ++i) A[p].H[i][k] = hp[i] + hp[m + 1 + i];
                A[p].H[k + 1][k] = subdiag(hp[2 * m + 2]);
                est[p] = A[p].add(k);
                kp[p] = k + 1;
                its[p]++;
                if (!isfinite(est[p]) || est[p] <= rtol * beta0[p] || A[p].H[k][k] == 0.0 || its[p] >= maxit)
                    iter[p] = 0;
            }
        }
        // delta += Z y for every problem of the cycle (y zero-padded to kmax)
        std::vector<double> Y((size_t)n * kmax, 0.0);
        for (int p = 0; p < n; ++p) {
            if (!cycle_act[p] || !isfinite(est[p])) continue;
            double y[kMaxKrylov];
            A[p].solve(kp[p], y);
            for (int i = 0; i < kp[p]; ++i) Y[(size_t)p * kmax + i] = y[i];
        }
        if ((e = set_active(c, cycle_act))) return e;
        if ((e = upload_per_problem(c, Y, kmax, dev + 3 * m + 8))) return e;
        launch_axpy_multi(g, W.delta, W.Z, vs, kmax, p0, dev + 3 * m + 8, 1.0, s, c->bt);
        launch_block_residual<double>(g, J, b, W.delta, W.w, false, s, c->bt);
        launch_cgs_pass(g, W.w, W.w, vs, 1, p0, cw, nullptr, true, W.partials, dev, s, c->bt);
        readback(c, host, dev, 1, s);
        HIP_OK(hipStreamSynchronize(s));
        std::vector<int> restart(n, 0);
        for (int p = 0; p < n; ++p) {
            if (!cycle_act[p]) continue;
            beta[p] = sqrt(host[p]);
            live[p] = 0;
            if (!isfinite(beta[p]) || !isfinite(est[p])) continue;  // ok stays 0
            if (beta[p] <= rtol * beta0[p] * 1.0000001 || est[p] <= rtol * beta0[p]) {
                ok[p] = 1;
                continue;
            }
            if (its[p] >= maxit) continue;
            restart[p] = 1;
            live[p] = 1;
        }
        if (any_of(restart)) {
            if ((e = set_active(c, restart))) return e;
            launch_scale_by_norm(g, W.w, W.V, p0, dev, s, c->bt);
        }
    }
    return MG_OK;
}

}  // namespace

int64_t batch_layout(const mg_grid_desc *d, int nprob, int64_t *ws_bytes, int64_t *state_off, int64_t *tail_off) {
    int64_t ws = carve_ctx(nullptr, d, nullptr);
    int64_t nf0 = (int64_t)(d->nr + 1) * level_pitch_of(d->nz) * 8;
    int64_t stride = round_up(ws + 5 * round_up(nf0, kAlign), kAlign);
    if (ws_bytes) *ws_bytes = ws;
    if (state_off) *state_off = ws;
    int64_t tail = stride * nprob;
    if (tail_off) *tail_off = tail;
    int64_t tail_bytes = round_up(nprob * (int64_t)sizeof(NewtonPhys), kAlign) + round_up(nprob * 6 * 8, kAlign) +
                         round_up(nprob * (int64_t)sizeof(int), kAlign);
    return tail + tail_bytes;
}

int batch_setup(const mg_grid_desc *d, int nprob, void *workspace, int64_t bytes, void *stream, mg_ctx **out) {
    int64_t wsb = 0, soff = 0, toff = 0;
    int64_t need = batch_layout(d, nprob, &wsb, &soff, &toff);
    if (bytes < need)
        return fail(MG_ENOMEM, "batch workspace has %lld bytes, needs %lld", (long long)bytes, (long long)need);
    mg_ctx *c = new (std::nothrow) mg_ctx();
    if (!c) return fail(MG_ENOMEM, "host allocation failed");
    c->desc = *d;
    c->zhost.assign(d->z_host, d->z_host + d->nz + 1);
    c->desc.z_host = c->zhost.data();
    c->stream = reinterpret_cast<hipStream_t>(stream);
    if (hipGetDevice(&c->device) != hipSuccess) c->device = 0;
    char *base = reinterpret_cast<char *>(workspace);
    carve_ctx(c, d, base);
    c->nw.fuse = getenv("MGF_NO_FUSE") == nullptr;
    c->nw.use_graphs = getenv("MGF_NO_GRAPHS") == nullptr;
    c->nw.smoother_only = getenv("MGF_SMOOTHER_ONLY") != nullptr;
    c->nw.rb_fused = getenv("MGF_HALF_SWEEPS") == nullptr;
    if (getenv("MGF_ONE_SWEEP")) c->nw.sweep2_max_nodes = 0;
    if (getenv("MGF_NO_SWEEP_RESTRICT")) c->nw.sweep2_restrict = false;
    if (const char *e = getenv("MGF_TWO_SWEEP_PRE_NODES")) c->nw.sweep2_pre_max_nodes = atoll(e);
    if (const char *e = getenv("MGF_TWO_SWEEP_NODES")) c->nw.sweep2_max_nodes = atoll(e);
    if (const char *e = getenv("MGF_CHAIN_MAX_BLOCKS")) c->nw.chain_max_blocks = atoi(e);
    if (const char *sr = getenv("MGF_SWEEP_ROWS"))
        for (int l = 0; l < c->nlev; ++l) c->lev[l].g.sh = atoi(sr) == 16 ? 16 : 8;
    if (const char *e = getenv("MGF_SWEEP2_ROWS"))
        for (int l = 0; l < c->nlev; ++l) c->lev[l].g.sh2 = atoi(e) == 4 ? 4 : 8;
    c->ws_base = base;
    c->ws_bytes = wsb;
    int64_t stride = toff / nprob;
    char *tail = base + toff;
    c->php_dev = tail;
    c->lohi_dev = reinterpret_cast<double *>(tail + round_up(nprob * (int64_t)sizeof(NewtonPhys), kAlign));
    int *act = reinterpret_cast<int *>(reinterpret_cast<char *>(c->lohi_dev) + round_up(nprob * 6 * 8, kAlign));
    c->bt.stride = stride;
    c->bt.active = act;
    c->bt.n = nprob;
    hipError_t e = hipHostMalloc((void **)&c->pinned, 512 * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&c->pinned_dev, c->pinned, 0);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&c->active_host, (size_t)kActiveSlots * nprob * sizeof(int), hipHostMallocDefault);
    for (int k = 0; k < kActiveSlots && e == hipSuccess; ++k)
        e = hipEventCreateWithFlags(&c->active_ev[k], hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&c->bpinned, (size_t)nprob * (2 * kMaxKrylov + 16) * sizeof(double),
                          hipHostMallocDefault);
    if (e == hipSuccess) e = hipMemsetAsync(workspace, 0, (size_t)need, c->stream);
    if (e != hipSuccess) {
        mg_destroy(c);
        return fail(MG_EHIP, "batch setup: %s", hipGetErrorString(e));
    }
    int st = upload_tables(c);
    if (st) {
        mg_destroy(c);
        return st;
    }
    // every problem gets the same grid tables: replicate problem 0's
    // workspace (tables + zeros) into the other regions
    for (int p = 1; p < nprob; ++p) {
        e = hipMemcpyAsync(base + p * stride, base, (size_t)wsb, hipMemcpyDeviceToDevice, c->stream);
        if (e != hipSuccess) {
            mg_destroy(c);
            return fail(MG_EHIP, "batch setup copy: %s", hipGetErrorString(e));
        }
    }
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        mg_destroy(c);
        return fail(MG_EHIP, "batch setup: %s", hipGetErrorString(e));
    }
    *out = c;
    return MG_OK;
}

int batch_state(mg_ctx *c, int p, mg_state *out) {
    if (p < 0 || p >= c->bt.n) return fail(MG_EINVAL, "problem %d outside 0..%d", p, c->bt.n - 1);
    int64_t nf0 = round_up((int64_t)(c->desc.nr + 1) * level_pitch_of(c->desc.nz) * 8, kAlign);
    char *r = c->ws_base + (int64_t)p * c->bt.stride + c->ws_bytes;
    out->V = reinterpret_cast<double *>(r);
    out->ne = reinterpret_cast<double *>(r + nf0);
    out->np = reinterpret_cast<double *>(r + 2 * nf0);
    out->Se = reinterpret_cast<const double *>(r + 3 * nf0);
    out->Sp = reinterpret_cast<const double *>(r + 4 * nf0);
    out->mue = out->De = out->mup = out->Dp = nullptr;  // batches use the constants
    return MG_OK;
}

int batch_solve_steady(mg_ctx *c, const mg_physics *phys, const mg_schedule *sc, mg_report *reps) {
    const int n = c->bt.n;
    hipStream_t s = c->stream;
    auto t0 = std::chrono::steady_clock::now();
    mg_state st;
    batch_state(c, 0, &st);
    const Level &L0 = c->lev[0];
    int64_t p0 = plane_of(L0);
    for (int p = 1; p < n; ++p)
        if (phys[p].k != phys[0].k) return fail(MG_EINVAL, "all problems of a batch need the same k");
    double3 cw = field_weights(&phys[0]);
    // the electrode kernel reads lohi[2p], lohi[2p+1]: pass per-field views
    std::vector<double> lohi_e(2 * n), lohi_p(2 * n), lohi_v(2 * n);
    for (int p = 0; p < n; ++p) {
        lohi_v[2 * p] = phys[p].V_bottom;
        lohi_v[2 * p + 1] = phys[p].V_top;
        lohi_e[2 * p] = phys[p].ne_bottom;
        lohi_e[2 * p + 1] = phys[p].ne_top;
        lohi_p[2 * p] = phys[p].np_bottom;
        lohi_p[2 * p + 1] = phys[p].np_top;
    }
    {
        double *h = c->bpinned;
        for (int q = 0; q < 2 * n; ++q) {
            h[q] = lohi_v[q];
            h[2 * n + q] = lohi_e[q];
            h[4 * n + q] = lohi_p[q];
        }
        HIP_OK(hipMemcpyAsync(c->lohi_dev, h, 6 * n * sizeof(double), hipMemcpyHostToDevice, s));
        std::vector<int> all(n, 1);
        int e0 = set_active(c, all);
        if (e0) return e0;
        launch_set_electrodes(L0.g, st.V, 0, 0, s, c->lohi_dev, c->bt);
        launch_set_electrodes(L0.g, st.ne, 0, 0, s, c->lohi_dev + 2 * n, c->bt);
        launch_set_electrodes(L0.g, st.np, 0, 0, s, c->lohi_dev + 4 * n, c->bt);
        launch_set_wall(L0.g, st.V, 0, 0, s, c->lohi_dev, c->bt);
        launch_set_wall(L0.g, st.ne, 0, 0, s, nullptr, c->bt);
        launch_set_wall(L0.g, st.np, 0, 0, s, nullptr, c->bt);
    }
    std::vector<double> dt(n, sc->dt0), dt_acc(n, 0.0), tt(n, 0.0), change(n, 0.0), relres(n, 0.0);
    std::vector<int> status(n, 0), steps(n, 0), rej(n, 0), newt(n, 0), fgm(n, 0), consec(n, 0);
    std::vector<NewtonPhys> hp(n);
    int maxn = sc->max_newton > 0 ? sc->max_newton : 10;
    int maxit = sc->max_cycles > 0 ? sc->max_cycles : 200;
    int rounds = 0;
    const bool progress = getenv("MGF_PROGRESS") != nullptr;
    while (true) {
        std::vector<int> run(n, 0);
        int nrun = 0;
        for (int p = 0; p < n; ++p) {
            run[p] = status[p] == 0 && steps[p] < sc->max_steps;
            nrun += run[p];
        }
        if (!nrun) break;
        ++rounds;
        if (progress && rounds % 50 == 0) {
            fprintf(stderr, "[mgfluid batch %dx%d] round %d: %d of %d problems still running\n", c->desc.nr + 1,
                    c->desc.nz + 1, rounds, nrun, n);
            fflush(stderr);
        }
        // per-problem physics with this round's dt
        for (int p = 0; p < n; ++p) {
            hp[p].qe = phys[p].mu_e / phys[p].D_e;
            hp[p].qp = -phys[p].mu_p / phys[p].D_p;
            hp[p].De = phys[p].D_e;
            hp[p].Dp = phys[p].D_p;
            hp[p].k = phys[p].k;
            hp[p].dt_inv = 1.0 / dt[p];
        }
        HIP_OK(hipMemcpyAsync(c->php_dev, hp.data(), n * sizeof(NewtonPhys), hipMemcpyHostToDevice, s));
        int e = set_active(c, run);
        if (e) return e;
        copy_state(c, &st, c->nw.snap);
        // Newton iterations in lockstep
        std::vector<int> nconv(n, 0), nfail(n, 0);
        for (int it = 1; it <= maxn; ++it) {
            std::vector<int> act(n, 0);
            for (int p = 0; p < n; ++p) act[p] = run[p] && !nconv[p] && !nfail[p];
            if (!any_of(act)) break;
            if ((e = set_active(c, act))) return e;
            mg_physics dummy = phys[0];
            assemble_all(c, &dummy, &st, 0.0);
            std::vector<int> ok, its;
            if ((e = fgmres_batch(c, cw, sc->lin_rtol, maxit, act, ok, its))) return e;
            std::vector<int> upd(n, 0);
            for (int p = 0; p < n; ++p) {
                if (!act[p]) continue;
                newt[p]++;
                fgm[p] += its[p];
                if (!ok[p])
                    nfail[p] = 1;
                else
                    upd[p] = 1;
            }
            if ((e = set_active(c, upd))) return e;
            launch_newton_update(L0.g, st.V, st.ne, st.np, c->nw.delta, p0, c->nw.partials, c->scal, s, c->bt);
            readback(c, c->bpinned, c->scal, 8, s);
            HIP_OK(hipStreamSynchronize(s));
            for (int p = 0; p < n; ++p) {
                if (!upd[p]) continue;
                const double *o = c->bpinned + 8 * p;
                double re = o[0] / fmax(o[1], 1e-300), rp = o[2] / fmax(o[3], 1e-300), rv = o[4] / fmax(o[5], 1e-300);
                double mx = fmax(re, fmax(rp, rv));
                if (!isfinite(mx) || mx > sc->reject_limit) {
                    nfail[p] = 1;
                } else if (mx < sc->newton_tol) {
                    double cnt = (double)(L0.g.nr + 1) * (L0.g.nz - 1);
                    if (o[6] >= -1e-10 * o[1] / cnt && o[7] >= -1e-10 * o[3] / cnt)
                        nconv[p] = 1;
                    else
                        nfail[p] = 1;
                }
            }
        }
        // accept or reject every running problem
        std::vector<int> acc(n, 0), rejd(n, 0);
        for (int p = 0; p < n; ++p) {
            if (!run[p]) continue;
            if (nconv[p])
                acc[p] = 1;
            else
                rejd[p] = 1;
        }
        if (any_of(rejd)) {
            if ((e = set_active(c, rejd))) return e;
            restore_state(c, c->nw.snap, &st);
        }
        if (any_of(acc)) {
            if ((e = set_active(c, acc))) return e;
            int nb = 0;
            launch_diff_norms(L0.g, st.ne, c->nw.snap + p0, c->partials, &nb, s, c->bt);
            launch_sum_partials(c->partials, nb, 2, c->scal, s, c->bt);
            launch_diff_norms(L0.g, st.np, c->nw.snap + 2 * p0, c->partials, &nb, s, c->bt);
            launch_sum_partials(c->partials, nb, 2, c->scal + 2, s, c->bt);
            readback(c, c->bpinned, c->scal, 4, s);
            HIP_OK(hipStreamSynchronize(s));
        }
        for (int p = 0; p < n; ++p) {
            if (rejd[p]) {
                rej[p]++;
                if (++consec[p] > 60) {
                    status[p] = MG_EREJECT;
                    continue;
                }
                dt[p] = (dt_acc[p] > 0 && dt[p] > dt_acc[p]) ? dt_acc[p] : 0.5 * dt[p];
            } else if (acc[p]) {
                consec[p] = 0;
                steps[p]++;
                tt[p] += dt[p];
                const double *o = c->bpinned + 4 * p;
                double ch = fmax(sqrt(o[0] / fmax(o[1], 1e-300)), sqrt(o[2] / fmax(o[3], 1e-300)));
                change[p] = ch;
                dt_acc[p] = dt[p];
                if (!isfinite(ch))
                    status[p] = MG_ENONFINITE;
                else if (ch < sc->steady_tol)
                    status[p] = 1;
                else
                    dt[p] = fmin(sc->growth * dt[p], sc->dt_max);
            }
        }
    }
    double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int worst = MG_OK;
    for (int p = 0; p < n; ++p) {
        if (reps) {
            reps[p].steps = steps[p];
            reps[p].rejected = rej[p];
            reps[p].vcycles = fgm[p];
            reps[p].newton_its = newt[p];
            reps[p].last_change = change[p];
            reps[p].final_relres = relres[p];
            reps[p].seconds = secs;
            reps[p].t_end = tt[p];
        }
        int code = status[p] == 1 ? MG_OK : (status[p] == 0 ? MG_ENOCONV : status[p]);
        if (code < worst) worst = code;
    }
    if (worst) fail(worst, "batch: some problems did not reach steady state");
    return worst;
}

void drop_graphs(mg_ctx *c) {
    for (int t = 0; t < 64; ++t)
        if (c->nw.exec[t]) {
            (void)hipGraphExecDestroy(c->nw.exec[t]);
            c->nw.exec[t] = nullptr;
        }
    for (int t = 0; t < 2; ++t) {
        if (c->nw.ev[t]) {
            (void)hipEventDestroy(c->nw.ev[t]);
            c->nw.ev[t] = nullptr;
        }
        if (c->nw.evf[t]) {
            (void)hipEventDestroy(c->nw.evf[t]);
            c->nw.evf[t] = nullptr;
        }
    }
    if (c->nw.side) {
        (void)hipStreamDestroy(c->nw.side);
        c->nw.side = nullptr;
    }
    c->nw.join_pending = false;
}

// Weighted norm of the steady residual F(u) (dt = infinity) at the state st
// (a diagnostic of how far a state is from steady).
int steady_residual(mg_ctx *c, const mg_physics *ph, const mg_state *st, double *out) {
    if (c->nw.m <= 0) return fail(MG_EINVAL, "no Newton workspace (krylov_m = 0)");
    hipStream_t s = c->stream;
    NewtonPhys np_;
    np_.qe = ph->mu_e / ph->D_e;
    np_.qp = -ph->mu_p / ph->D_p;
    np_.De = ph->D_e;
    np_.Dp = ph->D_p;
    np_.k = ph->k;
    np_.dt_inv = 0.0;
    const Level &L0 = c->lev[0];
    int64_t p0 = plane_of(L0);
    BOp J = bop(c, 0);
    NodeTransport tr;
    tr.mue = st->mue;
    tr.De = st->De;
    tr.mup = st->mup;
    tr.Dp = st->Dp;
    launch_newton_assemble(L0.g, J, st->V, st->ne, st->np, st->ne, st->np, st->Se, st->Sp, np_, true, s, nullptr,
                           Batch(), tr);
    launch_cgs_pass(L0.g, J.pl(kFe), J.pl(kFe), 3 * p0, 1, p0, field_weights(ph), nullptr, true, c->nw.partials,
                    c->nw.dev, s);
    HIP_OK(hipMemcpyAsync(c->pinned, c->nw.dev, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    *out = sqrt(c->pinned[0]);
    return MG_OK;
}

// One block V(nu1, nu2) cycle z = M r at the Newton Jacobian of the state
// st, every level assembled as for an implicit step of size dt (dt = inf:
// the steady Jacobian); the coarsest inverse on the context stream.
int newton_precond(mg_ctx *c, const mg_physics *ph, const mg_state *st, double dt, const double *r, double *z) {
    if (c->nw.m <= 0) return fail(MG_EINVAL, "no Newton workspace (krylov_m = 0)");
    if (c->bt.n > 1) return fail(MG_EINVAL, "a single-problem context is needed");
    hipStream_t s = c->stream;
    const double dt_inv = std::isfinite(dt) ? 1.0 / dt : 0.0;
    copy_state(c, st, c->nw.snap);
    assemble_all(c, ph, st, dt_inv);
    coarse_factor(c, s);
    const int64_t vs = 3 * plane_of(c->lev[0]);
    launch_fill(z, vs, 0.0, s);
    if (c->nw.prec32) {
        float *x32 = c->nw.lev[0].x32;
        launch_planes_to_f32(r, c->nw.f32, vs, s, c->bt);
        block_vcycle<float>(c, 0, c->nw.f32, x32, s);
        launch_planes_to_f64(x32, z, vs, s, c->bt);
    } else {
        block_vcycle<double>(c, 0, r, z, s);
    }
    HIP_OK(hipStreamSynchronize(s));
    return MG_OK;
}

int time_block_smoother(mg_ctx *c, int reps, int mode, int level, double *avg_ms) {
    if (c->nw.m <= 0) return fail(MG_EINVAL, "no Newton workspace (krylov_m = 0)");
    if (level < 0 || level >= c->nlev) return fail(MG_EINVAL, "bad level %d", level);
    const Level &L0 = c->lev[level];
    BOp J = bop(c, level);
    double *x = c->nw.lev[level].x, *x2 = c->nw.lev[level].x2;
    if (mode == 3 && level + 1 >= c->nlev) return fail(MG_EINVAL, "level %d has no coarser level", level);
    auto one = [&](int r) {
        if (mode == 3) {
            const Level &C = c->lev[level + 1];
            BOp Jc = bop(c, level + 1);
            launch_block_rb_sweep2_restrict<double>(L0.g, J, J.pl(kFe), (r & 1) ? x2 : x, (r & 1) ? x : x2, false,
                                                    C.g, Jc.pl(kFe), plane_of(C), c->stream);
        } else if (mode == 2)
            launch_block_rb_sweep2<double>(L0.g, J, J.pl(kFe), (r & 1) ? x2 : x, (r & 1) ? x : x2, false, nullptr,
                                           nullptr, 0, c->stream);
        else if (mode == 1)
            launch_block_rb_sweep<double>(L0.g, J, J.pl(kFe), (r & 1) ? x2 : x, (r & 1) ? x : x2, false, nullptr,
                                          nullptr, 0, c->stream);
        else
            launch_block_rbgs<double>(L0.g, J, J.pl(kFe), x, r & 1, c->stream);
    };
    hipEvent_t a, b;
    HIP_OK(hipEventCreate(&a));
    HIP_OK(hipEventCreate(&b));
    one(0);
    one(1);
    HIP_OK(hipEventRecord(a, c->stream));
    for (int r = 0; r < reps; ++r) one(r);
    HIP_OK(hipEventRecord(b, c->stream));
    HIP_OK(hipEventSynchronize(b));
    float ms = 0;
    HIP_OK(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *avg_ms = ms / reps;
    return MG_OK;
}

}  // namespace mgf
