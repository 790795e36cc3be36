// Internal declarations shared by the library's translation units.
// Device fields are row-major (nr+1) x pitch, z (index j) contiguous.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/mgfluid.h"

namespace mgf {

constexpr int kMaxLevels = 16;
constexpr int kMaxCoarseUnknowns = 1024;
constexpr int kMaxTY = 16;  // largest rows-per-workgroup of the 2D kernels

// Per-level grid tables and sizes, passed to kernels by value.
struct Geom {
    int nr, nz;
    int ty;             // radial rows per workgroup of the 2D kernels (tuning)
    int sh;             // radial rows of a red-black sweep tile: 8 (default) or 16
    int sh2;            // radial rows of a two-sweep tile: 8 (default) or 4
    int wall;           // 1: Dirichlet wall at r = R (rows i = nr are identity rows)
    int xcd;            // 1: sweep tiles in XCD-contiguous order (xcd_tile), 0: launch order
    int64_t pitch;
    double dr;
    const double *wr;   // radial width of node i (area of its z-faces), nr+1
    const double *fr;   // radius of face i+1/2, nr (fr[nr] = 0)
    const double *z;    // axial nodes, nz+1
    const double *dz;   // z[j+1]-z[j], nz
    const double *dzc;  // axial control width (dz[j-1]+dz[j])/2, nz+1 (0 at electrodes)
    const double *wl;   // prolongation weight of coarse node J for fine node 2J+1, nz/2
};

// Optional node values of the transport coefficients (null: constants).
struct NodeTransport {
    const double *mue = nullptr, *De = nullptr, *mup = nullptr, *Dp = nullptr;
};

// Five-point operator plus right-hand side, FV (integrated) form:
// a x[i-1][j] + b x[i][j] + c x[i+1][j] + d x[i][j-1] + e x[i][j+1] = f.
template <class T>
struct Op {
    T *a, *b, *c, *d, *e, *f;
};

struct Level {
    Geom g;
    Op<double> op[3];
    Op<float> op32[3];
    double *x, *r, *vinj;
    double *muinj, *Dinj;  // node transport injected to this level (scalar path)
    double *x2;        // partner of the level's field for one-launch sweeps
    float *x32, *r32, *x2_32;
    double *cinv[3];   // coarsest level only: transposed inverse, n x n
    float *cinv32[3];
    int ncoarse;       // unknowns on the coarsest level
};

// A batch of same-shape problems stored in equal-stride regions of one
// workspace: problem p's data is problem 0's address + p * stride bytes.
// Kernels take the problem index from blockIdx.z and skip inactive problems.
struct Batch {
    int64_t stride = 0;
    const int *active = nullptr;
    int n = 1;
};

template <class T>
__host__ __device__ inline T *boff(T *p, int64_t off) {
    return p ? reinterpret_cast<T *>(reinterpret_cast<char *>(p) + off) : p;
}
template <class T>
__host__ __device__ inline const T *boff(const T *p, int64_t off) {
    return p ? reinterpret_cast<const T *>(reinterpret_cast<const char *>(p) + off) : p;
}
__host__ __device__ inline Geom geom_off(Geom g, int64_t off) {
    g.wr = boff(g.wr, off);
    g.fr = boff(g.fr, off);
    g.z = boff(g.z, off);
    g.dz = boff(g.dz, off);
    g.dzc = boff(g.dzc, off);
    g.wl = boff(g.wl, off);
    return g;
}

#ifdef __HIPCC__
constexpr int kSumLoads = 8;
// sum of p[b * ld + c] over b = b0, b0 + step, ... < n, added in that order;
// the loads are issued kSumLoads at a time (a long grid's partials would
// otherwise be one dependent load per addition).
inline __device__ double sum_strided(const double *__restrict__ p, int n, int b0, int step, int64_t ld, int c) {
    double a = 0.0;
    for (int b = b0; b < n; b += step * kSumLoads) {
        double q[kSumLoads];
#pragma unroll
        for (int u = 0; u < kSumLoads; ++u) {
            const int bb = b + u * step;
            q[u] = bb < n ? p[(int64_t)bb * ld + c] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kSumLoads; ++u)
            if (b + u * step < n) a += q[u];
    }
    return a;
}

// Partial pivoting of the Gauss-Jordan factorisations: the first wavefront
// finds the row r in [col, n) with the largest |M[r][col]| (the first such
// row on ties, as a serial scan would) and stores it in *piv.  The caller
// synchronises the workgroup afterwards.
__device__ inline void pivot_search_wave0(const double *M, int64_t n2, int col, int n, int *piv) {
    if (threadIdx.x >= 64) return;
    int best = n;
    double bv = -1.0;
    for (int rr = col + (int)threadIdx.x; rr < n; rr += 64) {
        double v = fabs(M[(int64_t)rr * n2 + col]);
        if (v > bv) {
            bv = v;
            best = rr;
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        double ov = __shfl_xor(bv, off);
        int ob = __shfl_xor(best, off);
        if (ov > bv || (ov == bv && ob < best)) {
            bv = ov;
            best = ob;
        }
    }
    if (threadIdx.x == 0) *piv = best < n ? best : col;
}
#endif

// ---- kernel launchers (mg_kernels.hip) ----
void launch_poisson_assemble(const Geom &g, Op<double> op, const double *ne, const double *np,
                             double k, bool charge, double vlo, double vhi, hipStream_t s);
// mun, Dn: node transport (face = mean of its nodes; q = -sgn mu/D), or null (q, D)
void launch_sg_assemble(const Geom &g, Op<double> op, const double *V, const double *nk,
                        const double *S, double q, double D, double dt_inv, hipStream_t s,
                        const double *mun = nullptr, const double *Dn = nullptr, double sgn = 0.0);
void launch_inject(const Geom &gf, const double *vf, const Geom &gc, double *vc, hipStream_t s);
void launch_set_electrodes(const Geom &g, double *u, double lo, double hi, hipStream_t s,
                           const double *lohi = nullptr, const Batch &bt = Batch());
// With a Dirichlet wall (g.wall): row i = nr of u := lo + (hi - lo) (z_j - z_0)/(z_nz - z_0)
// (lohi: per-problem lo, hi); nothing otherwise.
void launch_set_wall(const Geom &g, double *u, double lo, double hi, hipStream_t s,
                     const double *lohi = nullptr, const Batch &bt = Batch());
// Particle flow out through cathode, anode and wall (3 device doubles).
void launch_boundary_flow(const Geom &g, const double *V, const double *n, double q, double D, double *out,
                          hipStream_t s, const double *mun = nullptr, const double *Dn = nullptr, double sgn = 0.0);
void launch_transport_table(const Geom &g, const double *V, const double *Et, const double *mut, const double *Dt,
                            int ntab, double *mu, double *D, hipStream_t s);
// Electrode rows and (with a wall) wall row of the three state fields.
void set_boundary(const Geom &g, double *V, double *ne, double *np, const mg_physics &ph, hipStream_t s);
void launch_fill(double *p, int64_t n, double v, hipStream_t s, const Batch &bt = Batch());
void launch_fill(float *p, int64_t n, float v, hipStream_t s, const Batch &bt = Batch());
template <class T>
void launch_rbgs(const Geom &g, Op<T> op, T *x, int colour, hipStream_t s);
template <class T>
void launch_zline(const Geom &g, Op<T> op, T *x, int parity, hipStream_t s);
// r = f - A x; if partials != nullptr also per-block sums of (r/vol)^2 and (b/vol)^2.
template <class TA, class TX, class TR>
void launch_residual(const Geom &g, Op<TA> op, const TX *f_override, const TX *x, TR *r,
                     double *partials, int *nblocks_out, hipStream_t s);
template <class T>
void launch_restrict(const Geom &gf, const T *rf, const Geom &gc, T *fc, hipStream_t s);
template <class T>
void launch_prolong(const Geom &gf, T *xf, const Geom &gc, const T *xc, hipStream_t s);
void launch_coarse_factor(const Geom &g, Op<double> op, double *scratch, double *invT, float *invT32,
                          hipStream_t s);
template <class T>
void launch_coarse_solve(const Geom &g, Op<T> op, const T *invT, T *x, hipStream_t s);
// One full red-black sweep xin -> xout (xout a whole field); zin: input zero;
// gc/xc: input is xin plus the prolongation of the coarse correction xc.
template <class T>
void launch_rb_sweep(const Geom &g, Op<T> op, const T *xin, T *xout, bool zin, const Geom *gc, const T *xc,
                     hipStream_t s);
// Coarse right-hand side fc = R (f - A x) in one launch.
template <class T>
void launch_residual_restrict_s(const Geom &gf, Op<T> op, const T *x, const Geom &gc, T *fc, hipStream_t s);
// Levels of the coarse end of the scalar V-cycle run by one workgroup.
constexpr int kMaxFusedS = 8;
template <class T>
struct FusedScalar {
    int n, nu1, nu2;
    Geom g[kMaxFusedS];
    Op<T> op[kMaxFusedS];
    const T *invT;
    T *x0;
};
// Returns false (nothing launched) when the levels do not fit in LDS.
template <class T>
bool launch_subcycle_s(const FusedScalar<T> &F, hipStream_t s);
void launch_sum_partials(const double *partials, int nblocks, int ncomp, double *out, hipStream_t s,
                         const Batch &bt = Batch());
void launch_diff_norms(const Geom &g, const double *a, const double *b, double *partials,
                       int *nblocks_out, hipStream_t s, const Batch &bt = Batch());
int residual_blocks(const Geom &g);
void launch_copy_field(const Geom &g, const double *src, double *dst, hipStream_t s, const Batch &bt = Batch());
void launch_to_f32(const Geom &g, const double *src, float *dst, hipStream_t s);
void launch_add_f32(const Geom &g, double *x, const float *e, hipStream_t s);
void launch_op_to_f32(const Geom &g, Op<double> op, Op<float> o32, hipStream_t s);
void launch_prolong_state(const Geom &gf, double *xf, const Geom &gc, const double *xc, hipStream_t s);

int fail(int code, const char *fmt, ...);

#define HIP_OK(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::mgf::fail(MG_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

constexpr int64_t kAlign = 256;
inline int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Bump allocator over the caller's workspace; with base == nullptr it only
// measures.
struct Carver {
    char *base;
    int64_t off = 0;
    template <class T>
    T *take(int64_t count) {
        off = round_up(off, kAlign);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * (int64_t)sizeof(T);
        return p;
    }
};

// Pinned staging slots of a batch's active flags (used in turn).
constexpr int kActiveSlots = 8;

// Per-level storage of the coupled (3x3-block) Newton path.
struct BLevel {
    double *J;      // kBPlanes planes
    double *x, *r;  // 3-field correction and residual
    double *x2;     // partner of x for the fused red-black sweep (zero electrode rows)
    double *cinvT;  // coarsest level: transposed inverse of the block matrix
    double *zt;     // block zebra smoother: 12 planes of line-elimination factors (else null)
    // FP32 copies for the mixed-precision preconditioner
    float *J32, *x32, *r32, *cinvT32, *x2_32;
};

struct NewtonWork {
    int m = 0;                 // FGMRES restart length (0: path disabled)
    BLevel lev[kMaxLevels];
    double *V = nullptr;       // Krylov basis, (m+1) 3-field vectors
    double *Z = nullptr;       // preconditioned directions, m vectors
    double *w = nullptr;       // work vector
    double *delta = nullptr;   // Newton correction
    double *snap = nullptr;    // state at the start of the step (V, ne, np)
    double *partials = nullptr;
    double *partials2 = nullptr;  // second buffer: a pass reads one while writing the other
    double *dev = nullptr;     // device scalars (dots, norms, y)
    double *scratch = nullptr; // coarsest factorisation workspace
    float *f32 = nullptr;      // FP32 right-hand side of the preconditioner (level 0)
    bool prec32 = false;       // block V-cycle in FP32 inside FP64 FGMRES
    // one captured graph per Arnoldi index k (block V-cycle, product,
    // orthogonalisation, readback), replayed on the context's stream
    hipStream_t cap = nullptr;
    hipGraphExec_t exec[64] = {};
    double cw_cap[3] = {0, 0, 0};
    bool use_graphs = true;
    // preconditioner reduced to nu1 + nu2 red-black sweeps on the finest grid
    // (no coarse correction): plain relaxation, measured against multigrid
    bool smoother_only = false;
    bool rb_fused = true;      // full red-black sweeps in one launch (else two half-sweeps)
    // two full sweeps per launch (nu1 and nu2 even) on levels of at most this
    // many nodes; larger levels launch one sweep at a time, which is faster
    // there (measured crossover between 129^2 and 257^2)
    int64_t sweep2_max_nodes = 129 * 129;
    bool sweep2_restrict = true;  // last pre-smoothing two-sweep launch also restricts the residual
    // pre-smoothing alone in pairs (restricting) on levels of at most this
    // many nodes (post-smoothing then one sweep per launch)
    int64_t sweep2_pre_max_nodes = 257 * 257;
    // largest launch grid (workgroups) whose Gram-Schmidt passes form the
    // previous pass's projections themselves (single problems only)
    int chain_max_blocks = 512;
    hipEvent_t ev[2] = {nullptr, nullptr};  // readback of Arnoldi steps k (even / odd)
    // the coarsest factorisation runs on `side` as a branch of Arnoldi step 0
    // (fork: evf[0] on the step's stream; join: evf[1], awaited before the
    // first use of the inverse)
    hipStream_t side = nullptr;
    hipEvent_t evf[2] = {nullptr, nullptr};
    bool join_pending = false;
    int last_its = 0;          // FGMRES iterations of the previous solve
    bool fuse = true;  // single-workgroup coarse sub-cycle
    int fuse_max = 16; // levels with nr, nz <= fuse_max run in it
};

}  // namespace mgf

struct mg_ctx {
    mg_grid_desc desc;
    std::vector<double> zhost;
    int nlev = 0;
    mgf::Level lev[mgf::kMaxLevels];
    hipStream_t stream = nullptr;
    int device = 0;              // HIP device current at setup (the context's work runs there)
    double *partials = nullptr;  // residual-kernel block sums
    double *scal = nullptr;      // device scalars
    double *coarse_scratch = nullptr;
    double *pinned = nullptr;    // host-pinned readback
    double *pinned_dev = nullptr;  // the same memory as kernels address it
    double *spare[4] = {nullptr, nullptr, nullptr, nullptr};
    bool assembled[3] = {false, false, false};
    int64_t vcycles = 0;
    mgf::NewtonWork nw;
    // batch of same-shape problems (n = 1: this context alone)
    mgf::Batch bt;
    void *php_dev = nullptr;      // device NewtonPhys[bt.n] in batch mode
    double *lohi_dev = nullptr;   // device electrode values, 6 per problem
    // pinned staging of the active flags: kActiveSlots slots of bt.n flags,
    // used in turn; a slot is rewritten only after the copy that last read
    // it has run (its event), so back-to-back uploads never race
    int *active_host = nullptr;
    hipEvent_t active_ev[mgf::kActiveSlots] = {};
    bool active_ev_used[mgf::kActiveSlots] = {};
    int active_seq = 0;
    double *bpinned = nullptr;    // pinned batch readback buffer
    char *ws_base = nullptr;
    int64_t ws_bytes = 0;         // bytes of one problem's solver workspace
};

namespace mgf {
// Newton path (mg_newton_host.hip)
void carve_newton(mg_ctx *c, const mg_grid_desc *d, Carver &cv, int nl);
int newton_implicit_step(mg_ctx *c, const mg_physics *ph, mg_state *st, double dt, const mg_schedule *sc,
                         mg_report *rep, bool *converged);
int newton_solve_steady(mg_ctx *c, const mg_physics *ph, mg_state *st, const mg_schedule *sc, mg_report *rep);
int newton_precond(mg_ctx *c, const mg_physics *ph, const mg_state *st, double dt, const double *r, double *z);
// mode 0: half-sweep, 1: one full sweep per launch, 2: two full sweeps per launch
int time_block_smoother(mg_ctx *c, int reps, int mode, int level, double *avg_ms);
void drop_graphs(mg_ctx *c);
int steady_residual(mg_ctx *c, const mg_physics *ph, const mg_state *st, double *out);
int64_t carve_ctx(mg_ctx *c, const mg_grid_desc *d, char *base);
int upload_tables(mg_ctx *c);
int validate_desc(const mg_grid_desc *d);
int64_t batch_layout(const mg_grid_desc *d, int nprob, int64_t *ws_bytes, int64_t *state_off, int64_t *tail_off);
int batch_setup(const mg_grid_desc *d, int nprob, void *workspace, int64_t bytes, void *stream, mg_ctx **out);
int batch_state(mg_ctx *c, int p, mg_state *out);
int batch_solve_steady(mg_ctx *c, const mg_physics *phys, const mg_schedule *sc, mg_report *reps);
int64_t level_pitch_of(int nz);
}  // namespace mgf
