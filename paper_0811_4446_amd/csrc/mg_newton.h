// Declarations of the coupled Newton (3x3-block) path.
#pragma once
#include "mg_internal.h"

namespace mgf {

constexpr int kMaxKrylov = 40;
// pinned host doubles per Arnoldi readback slot (2 m + 3 used); the context's
// 512 pinned doubles hold two slots, the least-squares solution and scalars
constexpr int kSlot = 128;
static_assert(2 * kSlot + 2 * kMaxKrylov + 16 <= 512, "pinned layout");
// After those 512 doubles: two slots of the second Gram-Schmidt pass's
// workgroup partials (chained grids of at most kChainCap workgroups, up to
// kMaxKrylov + 1 columns), which the host sums itself.
constexpr int kChainCap = 512;
constexpr int64_t kPartSlot = (int64_t)kChainCap * (kMaxKrylov + 1);
constexpr int64_t kPinnedDoubles = 512 + 2 * kPartSlot;
constexpr int kBPlanes = 30;
constexpr int kEE = 0, kEV = 5, kPP = 10, kPV = 15, kVV = 20, kVe = 25, kVp = 26, kFe = 27, kFp = 28, kFV = 29;

// Block operator: kBPlanes planes of (nr+1) x pitch values.
template <class T>
struct BOpT {
    T *base;
    int64_t plane;
    __host__ __device__ T *pl(int k) const { return base + (int64_t)k * plane; }
};
using BOp = BOpT<double>;

// Levels run by the single-workgroup coarse sub-cycle (last = coarsest).
constexpr int kMaxFused = 8;
constexpr int kMaxFusedCoarse = 1024;  // 3 x unknown nodes of the coarsest level
template <class T>
struct FusedLevelsT {
    int n, nu1, nu2;
    Geom g[kMaxFused];
    T *J[kMaxFused];
    int64_t plane[kMaxFused];
    T *x[kMaxFused];
    T *r[kMaxFused];
    const T *f0;
    const T *invT;
    uint32_t wmagic[kMaxFused];  // set by the launcher: ceil(2^32 / (nz + 1)) per level
};

struct NewtonPhys {
    double qe, qp;   // -s mu / D for electrons (s = -1) and ions (s = +1)
    double De, Dp, k, dt_inv;
};

// Several levels of the hierarchy in one launch of a 2D kernel: blocks of
// 64 x kLevTabTY threads; level k of the table owns the row blocks
// blockIdx.y in [y0[k], y0[k+1]) (filled by the launcher).
constexpr int kLevTabTY = 4;
constexpr int kMaxLevTab = 16;  // callers keep 1 <= n <= kMaxLevTab
struct LevTab {
    int n = 0;
    int y0[kMaxLevTab + 1];
    int shift[kMaxLevTab];  // levels below the finest grid
    Geom g[kMaxLevTab];
    BOp J[kMaxLevTab];
    BOpT<float> J32[kMaxLevTab];
};

void launch_newton_assemble(const Geom &g, const BOp &J, const double *V, const double *ne, const double *np,
                            const double *nek, const double *npk, const double *Se, const double *Sp,
                            const NewtonPhys &ph, bool with_rhs, hipStream_t s, const NewtonPhys *php = nullptr,
                            const Batch &bt = Batch(), const NodeTransport &tr = NodeTransport());
template <class T>
void launch_block_rbgs(const Geom &g, const BOpT<T> &J, const T *f, T *x, int colour, hipStream_t s,
                       const Batch &bt = Batch());
// Block zebra z-line half-sweep of the lines i = colour, colour + 2, ...;
// tmp: 12 planes of the level's plane size (elimination factors).
template <class T>
void launch_block_zline(const Geom &g, const BOpT<T> &J, const T *f, T *x, T *tmp, int colour, hipStream_t s,
                        const Batch &bt = Batch());
// One full red-black sweep xin -> xout; zin: input zero; gc/xc/pc: input is
// xin plus the prolongation of the coarse correction xc (level gc, plane pc).
template <class T>
void launch_block_rb_sweep(const Geom &g, const BOpT<T> &J, const T *f, const T *xin, T *xout, bool zin,
                           const Geom *gc, const T *xc, int64_t pc, hipStream_t s, const Batch &bt = Batch());
// Two full red-black sweeps xin -> xout in one launch (same input options).
template <class T>
void launch_block_rb_sweep2(const Geom &g, const BOpT<T> &J, const T *f, const T *xin, T *xout, bool zin,
                            const Geom *gc, const T *xc, int64_t pc, hipStream_t s, const Batch &bt = Batch());
// The same two sweeps, then the residual f - B xout restricted to the coarse
// right-hand side fc (level gc, plane pc) in the same launch.
template <class T>
void launch_block_rb_sweep2_restrict(const Geom &g, const BOpT<T> &J, const T *f, const T *xin, T *xout, bool zin,
                                     const Geom &gc, T *fc, int64_t pc, hipStream_t s, const Batch &bt = Batch());
template <class T>
void launch_block_residual(const Geom &g, const BOpT<T> &J, const T *f, const T *x, T *r, bool apply,
                           hipStream_t s, const Batch &bt = Batch());
template <class T>
void launch_restrict3(const Geom &gf, const T *rf, int64_t pf, const Geom &gc, T *fc, int64_t pc, hipStream_t s,
                      const Batch &bt = Batch());
// Coarse right-hand side fc = R (f - B x) in one launch (no fine residual stored).
template <class T>
void launch_residual_restrict(const Geom &gf, const BOpT<T> &J, const T *f, const T *x, const Geom &gc, T *fc,
                              int64_t pc, hipStream_t s, const Batch &bt = Batch());
template <class T>
void launch_prolong3(const Geom &gf, T *xf, int64_t pf, const Geom &gc, const T *xc, int64_t pc, hipStream_t s,
                     const Batch &bt = Batch());
// Jacobians of levels t.g[k] (no rhs) at the finest state injected to them
// (node (i, j) of level shift[k] reads the finest node (i, j) << shift[k]).
void launch_newton_assemble_coarse(LevTab t, const double *V, const double *ne, const double *np, int64_t pitch0,
                                   const NewtonPhys &ph, hipStream_t s, const NewtonPhys *php = nullptr,
                                   const Batch &bt = Batch(), const NodeTransport &tr = NodeTransport());
// FP32 copies t.J32[k] of every level's Jacobian t.J[k].
void launch_block_to_f32_levels(LevTab t, hipStream_t s, const Batch &bt = Batch());
void launch_block_coarse_factor(const Geom &g, const BOp &J, double *scratch, double *invT, hipStream_t s,
                                const Batch &bt = Batch());
template <class T>
void launch_block_coarse_solve(const Geom &g, const BOpT<T> &J, const T *f, const T *invT, T *x, hipStream_t s,
                               const Batch &bt = Batch());
int block_vec_blocks(const Geom &g);
template <class T>
void launch_block_subcycle(const FusedLevelsT<T> &F, hipStream_t s, const Batch &bt = Batch());
void launch_planes_to_f32(const double *src, float *dst, int64_t n, hipStream_t s, const Batch &bt = Batch());
void launch_planes_to_f64(const float *src, double *dst, int64_t n, hipStream_t s, const Batch &bt = Batch());
// Deferred (lagged) second projection of the Arnoldi vector.  fin_h: the
// pass first finalises basis slot nv-1, which holds u (one projection
// removed): slot = (u - sum_{v<nv-1} fin_h[v] basis_v) / sqrt(*fin_nu2)
// (written through fin_out, the same slot), and uses the result as basis
// vector nv-1.  next: the updated w is stored there (the next basis slot,
// zero on the electrode columns) instead of in w.  with_norm: the partial
// sums also hold (w, w) after the nv projections.
// fin_part (instead of fin_h, fin_nu2): the partials of the previous step's
// second pass (fin_nblk workgroups, nv columns: nv-1 projections and
// (u, u)), summed by every workgroup in the chained order.  part_host: the
// pass also stores its partials there (pinned host memory).
struct CgsLag {
    const double *fin_h = nullptr;
    const double *fin_nu2 = nullptr;
    const double *fin_part = nullptr;
    int fin_nblk = 0;
    double *fin_out = nullptr;
    double *next = nullptr;
    int with_norm = 0;
    double *part_host = nullptr;
};
// Gram-Schmidt pass: w = J z (if J and z) or w -= sum_v h_sub[v] basis_v
// (if h_sub), then the partial sums of the weighted (w, basis_v), v < nv,
// or of (w, w) when self_norm; with out != nullptr a second launch adds them
// into out[].
void launch_cgs_pass(const Geom &g, double *w, const double *basis, int64_t vstride, int nv, int64_t plane,
                     double3 cw, const double *h_sub, bool self_norm, double *partials, double *out, hipStream_t s,
                     const Batch &bt = Batch(), const BOp *J = nullptr, const double *z = nullptr,
                     const CgsLag &lag = CgsLag());
// nu^2 = h[nv] - sum_{v<nv} h[v]^2 (the k_sum_cols output of a with_norm
// pass) to out and, when given, to pinned out_host.
void launch_lagged_nu2(double *h, int nv, double *out, double *out_host, hipStream_t s, const Batch &bt = Batch());
// A Gram-Schmidt pass that first forms the projections h = V^T w of the
// previous pass from that pass's workgroup partials h_part (same launch
// grid; the result also to h_out and, when given, to pinned h_host), then
// w -= V h and its own partials (partials must not alias h_part).
void launch_cgs_pass_chained(const Geom &g, double *w, const double *basis, int64_t vstride, int nv, int64_t plane,
                             double3 cw, bool self_norm, const double *h_part, double *h_out, double *h_host,
                             double *partials, hipStream_t s, const Batch &bt = Batch(), const CgsLag &lag = CgsLag());
void launch_axpy_multi(const Geom &g, double *w, const double *basis, int64_t vstride, int nv, int64_t plane,
                       const double *h, double sign, hipStream_t s, const Batch &bt = Batch());
void launch_scale_by_norm(const Geom &g, const double *src, double *dst, int64_t plane, const double *nrm2,
                          hipStream_t s, const Batch &bt = Batch());
void launch_newton_update(const Geom &g, double *V, double *ne, double *np, const double *du, int64_t plane,
                          double *partials, double *out, hipStream_t s, const Batch &bt = Batch());

}  // namespace mgf
