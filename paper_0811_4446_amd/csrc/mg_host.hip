// Host side of the C ABI (include/mgfluid.h): grid hierarchy, workspace
// carving, assembly on all levels, V-cycle recursion, stop tests and the
// time-step drivers.  Every kernel goes to the context's stream.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <chrono>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "mg_internal.h"
#include "mg_newton.h"
#include "wn_net.h"

namespace {
constexpr int kMaxKrylovDesc = 40;
}

using namespace mgf;

namespace {
thread_local char g_err[512] = "";
}  // namespace

int mgf::fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

namespace {

int64_t level_pitch(int nz) { return round_up(nz + 1, 16); }

int count_levels(int nr, int nz, int coarsest) {
    if (nr < 2 || nz < 2 || coarsest < 2) return -1;
    int m = nr < nz ? nr : nz;
    if (m % coarsest) return -1;
    int q = m / coarsest, L = 0;
    while (q > 1) {
        if (q & 1) return -1;
        q >>= 1;
        ++L;
    }
    if (nr % (1 << L) || nz % (1 << L)) return -1;
    return L + 1;
}

int validate(const mg_grid_desc *d) {
    if (!d) return fail(MG_EINVAL, "null grid descriptor");
    if (d->abi_version != MG_ABI_VERSION)
        return fail(MG_EINVAL, "abi_version %d, library has %d", d->abi_version, MG_ABI_VERSION);
    if (!d->z_host) return fail(MG_EINVAL, "null z_host");
    if (!(d->R > 0) || !(d->d > 0)) return fail(MG_EINVAL, "R and d must be positive");
    if (d->smoother != MG_SMOOTH_RB && d->smoother != MG_SMOOTH_ZEBRA && d->smoother != MG_SMOOTH_ZEBRA_BLOCK)
        return fail(MG_EINVAL, "bad smoother %d", d->smoother);
    if (d->prec != MG_FP64 && d->prec != MG_FP32_IR) return fail(MG_EINVAL, "bad precision %d", d->prec);
    if (d->r_outer_bc != MG_WALL_ZERO_FLUX && d->r_outer_bc != MG_WALL_DIRICHLET)
        return fail(MG_EINVAL, "bad r_outer_bc %d", d->r_outer_bc);
    if (d->nu1 < 0 || d->nu2 < 0 || d->nu1 + d->nu2 < 1 || d->nu1 > 16 || d->nu2 > 16)
        return fail(MG_EINVAL, "bad smoothing counts %d, %d", d->nu1, d->nu2);
    int nl = count_levels(d->nr, d->nz, d->coarsest_n);
    if (nl < 1 || nl > kMaxLevels)
        return fail(MG_EINVAL, "grid %dx%d cannot be coarsened to %d by halving", d->nr, d->nz, d->coarsest_n);
    if (d->nz - 1 > 64 * 16) return fail(MG_EINVAL, "nz = %d exceeds the z-line limit 1025", d->nz);
    if (d->krylov_m < 0 || d->krylov_m > kMaxKrylovDesc)
        return fail(MG_EINVAL, "krylov_m = %d outside 0..%d", d->krylov_m, kMaxKrylovDesc);
    int nrc = d->nr >> (nl - 1), nzc = d->nz >> (nl - 1);
    if ((nrc + 1) * (nzc - 1) > kMaxCoarseUnknowns)
        return fail(MG_EINVAL, "coarsest grid has %d unknowns (limit %d)", (nrc + 1) * (nzc - 1),
                    kMaxCoarseUnknowns);
    const double *z = d->z_host;
    if (z[0] != 0.0 || z[d->nz] != d->d) return fail(MG_EINVAL, "z must start at 0 and end at d");
    for (int j = 0; j < d->nz; ++j)
        if (!(z[j + 1] > z[j])) return fail(MG_EINVAL, "z not strictly increasing at j = %d", j);
    return MG_OK;
}

}  // namespace

namespace {

// Lay out every workspace array; with ctx->... pointers filled when
// `base` is non-null.  Returns the byte count.
int64_t carve(mg_ctx *c, const mg_grid_desc *d, char *base) {
    Carver cv{base};
    int nl = count_levels(d->nr, d->nz, d->coarsest_n);
    bool ir = d->prec == MG_FP32_IR;
    for (int l = 0; l < nl; ++l) {
        int nr = d->nr >> l, nz = d->nz >> l;
        int64_t pitch = level_pitch(nz);
        int64_t nf = (int64_t)(nr + 1) * pitch;
        Level L;
        memset(&L, 0, sizeof L);
        L.g.nr = nr;
        L.g.nz = nz;
        L.g.ty = 4;
        L.g.sh = 8;
        L.g.sh2 = 8;
        L.g.wall = d->r_outer_bc == MG_WALL_DIRICHLET ? 1 : 0;
        L.g.xcd = getenv("MGF_NO_XCD_ORDER") ? 0 : 1;
        L.g.pitch = pitch;
        L.g.dr = d->R / nr;
        L.g.wr = cv.take<double>(nr + 1);
        L.g.fr = cv.take<double>(nr + 1);
        L.g.z = cv.take<double>(nz + 1);
        L.g.dz = cv.take<double>(nz);
        L.g.dzc = cv.take<double>(nz + 1);
        L.g.wl = cv.take<double>(nz / 2 + 1);
        for (int e = 0; e < 3; ++e) {
            Op<double> &o = L.op[e];
            o.a = cv.take<double>(nf);
            o.b = cv.take<double>(nf);
            o.c = cv.take<double>(nf);
            o.d = cv.take<double>(nf);
            o.e = cv.take<double>(nf);
            o.f = cv.take<double>(nf);
            if (ir) {
                Op<float> &p = L.op32[e];
                p.a = cv.take<float>(nf);
                p.b = cv.take<float>(nf);
                p.c = cv.take<float>(nf);
                p.d = cv.take<float>(nf);
                p.e = cv.take<float>(nf);
                p.f = cv.take<float>(nf);
            }
        }
        L.x = cv.take<double>(nf);
        L.x2 = cv.take<double>(nf);
        L.r = cv.take<double>(nf);
        L.vinj = cv.take<double>(nf);
        L.muinj = cv.take<double>(nf);
        L.Dinj = cv.take<double>(nf);
        if (ir) {
            L.x32 = cv.take<float>(nf);
            L.x2_32 = cv.take<float>(nf);
            L.r32 = cv.take<float>(nf);
        }
        if (l == nl - 1) {
            int n = (nr + 1) * (nz - 1);
            L.ncoarse = n;
            for (int e = 0; e < 3; ++e) {
                L.cinv[e] = cv.take<double>((int64_t)n * n);
                if (ir) L.cinv32[e] = cv.take<float>((int64_t)n * n);
            }
            double *scr = cv.take<double>((int64_t)n * 2 * n);
            if (c) c->coarse_scratch = scr;
        }
        if (c) c->lev[l] = L;
    }
    int64_t nf0 = (int64_t)(d->nr + 1) * level_pitch(d->nz);
    Geom g0;
    g0.nr = d->nr;
    g0.nz = d->nz;
    // sized for one radial row per workgroup (the smallest launch shape)
    int nblk = ((d->nz + 1 + 63) / 64) * (d->nr + 1);
    double *part = cv.take<double>(2 * (int64_t)nblk + 16);
    double *scal = cv.take<double>(64);
    double *sp[4];
    for (int t = 0; t < 4; ++t) sp[t] = cv.take<double>(nf0);
    if (c) {
        c->partials = part;
        c->scal = scal;
        for (int t = 0; t < 4; ++t) c->spare[t] = sp[t];
        c->nlev = nl;
    }
    carve_newton(c, d, cv, nl);
    return round_up(cv.off, kAlign);
}

// Grid tables of Sec. 2 for one level (host, FP64).
void level_tables(const mg_grid_desc *d, const double *zl, int nr, int nz, std::vector<double> &wr,
                  std::vector<double> &fr, std::vector<double> &dz, std::vector<double> &dzc,
                  std::vector<double> &wl) {
    double R = d->R, dr = R / nr;
    wr.assign(nr + 1, 0.0);
    fr.assign(nr + 1, 0.0);
    for (int i = 0; i <= nr; ++i) {
        if (i == 0)
            wr[i] = dr * dr / 8.0;
        else if (i == nr)
            wr[i] = 0.5 * dr * (R - 0.25 * dr);
        else
            wr[i] = (i * dr) * dr;
        if (i < nr) fr[i] = (i + 0.5) * dr;
    }
    dz.assign(nz, 0.0);
    for (int j = 0; j < nz; ++j) dz[j] = zl[j + 1] - zl[j];
    dzc.assign(nz + 1, 0.0);
    for (int j = 1; j < nz; ++j) dzc[j] = 0.5 * (zl[j + 1] - zl[j - 1]);
    wl.assign(nz / 2 + 1, 0.0);
    for (int J = 0; J < nz / 2; ++J) {
        double h0 = zl[2 * J + 1] - zl[2 * J];
        double h1 = zl[2 * J + 2] - zl[2 * J + 1];
        wl[J] = h1 / (h0 + h1);
    }
}

int check_ctx(const mg_ctx *c) {
    if (!c) return fail(MG_EINVAL, "null context");
    return MG_OK;
}

int check_eq(int eq) {
    if (eq < 0 || eq > 2) return fail(MG_EINVAL, "bad equation %d", eq);
    return MG_OK;
}

// ---- V-cycle --------------------------------------------------------------

template <class T>
Op<T> op_of(mg_ctx *c, int l, int eq);
template <>
Op<double> op_of<double>(mg_ctx *c, int l, int eq) { return c->lev[l].op[eq]; }
template <>
Op<float> op_of<float>(mg_ctx *c, int l, int eq) { return c->lev[l].op32[eq]; }

template <class T>
T *x_of(mg_ctx *c, int l);
template <>
double *x_of<double>(mg_ctx *c, int l) { return c->lev[l].x; }
template <>
float *x_of<float>(mg_ctx *c, int l) { return c->lev[l].x32; }

template <class T>
T *r_of(mg_ctx *c, int l);
template <>
double *r_of<double>(mg_ctx *c, int l) { return c->lev[l].r; }
template <>
float *r_of<float>(mg_ctx *c, int l) { return c->lev[l].r32; }

template <class T>
const T *cinv_of(mg_ctx *c, int eq);
template <>
const double *cinv_of<double>(mg_ctx *c, int eq) { return c->lev[c->nlev - 1].cinv[eq]; }
template <>
const float *cinv_of<float>(mg_ctx *c, int eq) { return c->lev[c->nlev - 1].cinv32[eq]; }

template <class T>
T *x2_of(mg_ctx *c, int l);
template <>
double *x2_of<double>(mg_ctx *c, int l) { return c->lev[l].x2; }
template <>
float *x2_of<float>(mg_ctx *c, int l) { return c->lev[l].x2_32; }

// Red-black sweeps in one launch each (with the fused residual-restriction,
// zero-guess first sweep, prolongation on read and the LDS coarse sub-cycle).
bool fused_rb(const mg_ctx *c) { return c->nw.rb_fused && c->desc.smoother == MG_SMOOTH_RB; }

// `sweeps` sweeps on level l: pairs of one-launch sweeps x -> x2 -> x, then
// half-sweeps (or zebra sweeps) for the rest.  x_zero: x is zero on entry and
// is not read; xc: the coarse correction (level l+1) still to be prolonged
// and added, which the first one-launch sweep does while staging its input.
// Callers set x_zero or xc only when fused_rb(c) and sweeps >= 2.
template <class T>
void smooth(mg_ctx *c, int l, int eq, T *x, int sweeps, bool x_zero = false, const T *xc = nullptr) {
    const Geom &g = c->lev[l].g;
    Op<T> op = op_of<T>(c, l, eq);
    int k = 0;
    if (fused_rb(c) && sweeps >= 2) {
        T *x2 = x2_of<T>(c, l);
        const Geom *gc = xc ? &c->lev[l + 1].g : nullptr;
        for (; k + 2 <= sweeps; k += 2) {
            const bool first = k == 0;
            launch_rb_sweep<T>(g, op, x, x2, x_zero && first, first ? gc : nullptr, first ? xc : nullptr,
                               c->stream);
            launch_rb_sweep<T>(g, op, x2, x, false, nullptr, nullptr, c->stream);
        }
    }
    for (; k < sweeps; ++k)
        for (int col = 0; col < 2; ++col) {
            if (c->desc.smoother == MG_SMOOTH_RB)
                launch_rbgs<T>(g, op, x, col, c->stream);
            else
                launch_zline<T>(g, op, x, col, c->stream);
        }
}

// Largest level (nr, nz) of the scalar coarse sub-cycle (LDS capacity).
constexpr int kFuseMaxS = 32;

// V(nu1, nu2) on level l for the field x (level l layout).  On levels l >= 1
// x is a correction that starts from zero (x is not read on entry).
template <class T>
void vcycle_level(mg_ctx *c, int l, int eq, T *x) {
    hipStream_t s = c->stream;
    const Level &L = c->lev[l];
    if (l == c->nlev - 1) {
        launch_coarse_solve<T>(L.g, op_of<T>(c, l, eq), cinv_of<T>(c, eq), x, s);
        return;
    }
    if (l >= 1 && fused_rb(c) && c->nw.fuse && c->nlev - l <= kMaxFusedS && L.g.nr <= kFuseMaxS &&
        L.g.nz <= kFuseMaxS) {
        FusedScalar<T> F;
        memset(&F, 0, sizeof F);
        F.n = c->nlev - l;
        F.nu1 = c->desc.nu1;
        F.nu2 = c->desc.nu2;
        for (int q = 0; q < F.n; ++q) {
            F.g[q] = c->lev[l + q].g;
            F.op[q] = op_of<T>(c, l + q, eq);
        }
        F.invT = cinv_of<T>(c, eq);
        F.x0 = x;
        if (launch_subcycle_s<T>(F, s)) return;
    }
    const bool zero_sweep = l >= 1 && fused_rb(c) && c->desc.nu1 >= 2;
    if (l >= 1 && !zero_sweep) launch_fill(x, (int64_t)(L.g.nr + 1) * L.g.pitch, T(0), s);
    smooth<T>(c, l, eq, x, c->desc.nu1, zero_sweep);
    const Level &C = c->lev[l + 1];
    Op<T> oc = op_of<T>(c, l + 1, eq);
    if (fused_rb(c)) {
        launch_residual_restrict_s<T>(L.g, op_of<T>(c, l, eq), x, C.g, oc.f, s);
    } else {
        T *r = r_of<T>(c, l);
        launch_residual<T, T, T>(L.g, op_of<T>(c, l, eq), nullptr, x, r, nullptr, nullptr, s);
        launch_restrict<T>(L.g, r, C.g, oc.f, s);
    }
    T *xc = x_of<T>(c, l + 1);
    vcycle_level<T>(c, l + 1, eq, xc);
    if (fused_rb(c) && c->desc.nu2 >= 2) {
        smooth<T>(c, l, eq, x, c->desc.nu2, false, xc);
    } else {
        launch_prolong<T>(L.g, x, C.g, xc, s);
        smooth<T>(c, l, eq, x, c->desc.nu2);
    }
}

// Strong-form relative residual of the FP64 system (synchronises).
int relres64(mg_ctx *c, int eq, const double *x, double *out) {
    const Level &L = c->lev[0];
    int nb = 0;
    launch_residual<double, double, double>(L.g, L.op[eq], nullptr, x, L.r, c->partials, &nb, c->stream);
    launch_sum_partials(c->partials, nb, 2, c->scal, c->stream);
    HIP_OK(hipMemcpyAsync(c->pinned, c->scal, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(hipStreamSynchronize(c->stream));
    double rr = c->pinned[0], bb = c->pinned[1];
    *out = (bb > 0.0) ? sqrt(rr / bb) : sqrt(rr);
    return MG_OK;
}

// One FP64 cycle, or one FP32 cycle applied as a defect correction.
int one_cycle(mg_ctx *c, int eq, double *x) {
    if (c->desc.prec == MG_FP64) {
        vcycle_level<double>(c, 0, eq, x);
    } else {
        const Level &L = c->lev[0];
        hipStream_t s = c->stream;
        // FP64 residual -> FP32 right-hand side of the correction equation
        launch_residual<double, double, float>(L.g, L.op[eq], nullptr, x, L.op32[eq].f, nullptr, nullptr, s);
        launch_fill(L.x32, (int64_t)(L.g.nr + 1) * L.g.pitch, 0.0f, s);
        vcycle_level<float>(c, 0, eq, L.x32);
        launch_add_f32(L.g, x, L.x32, s);
    }
    c->vcycles++;
    return MG_OK;
}

}  // namespace

int64_t mgf::carve_ctx(mg_ctx *c, const mg_grid_desc *d, char *base) { return carve(c, d, base); }
int mgf::validate_desc(const mg_grid_desc *d) { return validate(d); }
int64_t mgf::level_pitch_of(int nz) { return level_pitch(nz); }

// Grid tables of every level (Sec. 2) into the context's workspace.
int mgf::upload_tables(mg_ctx *c) {
    std::vector<double> zl, wr, fr, dz, dzc, wl;
    for (int l = 0; l < c->nlev; ++l) {
        Level &L = c->lev[l];
        zl.resize(L.g.nz + 1);
        for (int j = 0; j <= L.g.nz; ++j) zl[j] = c->zhost[(size_t)j << l];
        level_tables(&c->desc, zl.data(), L.g.nr, L.g.nz, wr, fr, dz, dzc, wl);
        HIP_OK(hipMemcpyAsync((void *)L.g.wr, wr.data(), wr.size() * 8, hipMemcpyHostToDevice, c->stream));
        HIP_OK(hipMemcpyAsync((void *)L.g.fr, fr.data(), fr.size() * 8, hipMemcpyHostToDevice, c->stream));
        HIP_OK(hipMemcpyAsync((void *)L.g.z, zl.data(), zl.size() * 8, hipMemcpyHostToDevice, c->stream));
        HIP_OK(hipMemcpyAsync((void *)L.g.dz, dz.data(), dz.size() * 8, hipMemcpyHostToDevice, c->stream));
        HIP_OK(hipMemcpyAsync((void *)L.g.dzc, dzc.data(), dzc.size() * 8, hipMemcpyHostToDevice, c->stream));
        HIP_OK(hipMemcpyAsync((void *)L.g.wl, wl.data(), wl.size() * 8, hipMemcpyHostToDevice, c->stream));
        // the host vectors are reused next level: wait for the copies
        HIP_OK(hipStreamSynchronize(c->stream));
    }
    return MG_OK;
}

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *mg_last_error(void) { return g_err; }

int mg_query(const mg_grid_desc *desc, int64_t *pitch_elems, int64_t *workspace_bytes) {
    int st = validate(desc);
    if (st) return st;
    if (pitch_elems) *pitch_elems = level_pitch(desc->nz);
    if (workspace_bytes) *workspace_bytes = carve(nullptr, desc, nullptr);
    return MG_OK;
}

int mg_setup(const mg_grid_desc *desc, void *workspace, int64_t workspace_bytes, void *stream,
             mg_ctx **out) {
    int st = validate(desc);
    if (st) return st;
    if (!out) return fail(MG_EINVAL, "null output pointer");
    if (!workspace) return fail(MG_EINVAL, "null workspace");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
        return fail(MG_EINVAL, "workspace must be %d-byte aligned", (int)kAlign);
    int64_t need = carve(nullptr, desc, nullptr);
    if (workspace_bytes < need)
        return fail(MG_ENOMEM, "workspace has %lld bytes, needs %lld", (long long)workspace_bytes,
                    (long long)need);
    mg_ctx *c = new (std::nothrow) mg_ctx();
    if (!c) return fail(MG_ENOMEM, "host allocation failed");
    c->desc = *desc;
    c->zhost.assign(desc->z_host, desc->z_host + desc->nz + 1);
    c->desc.z_host = c->zhost.data();
    c->stream = reinterpret_cast<hipStream_t>(stream);
    if (hipGetDevice(&c->device) != hipSuccess) c->device = 0;
    carve(c, desc, reinterpret_cast<char *>(workspace));
    // debugging switches: per-level launches instead of the fused coarse
    // sub-cycle, eager launches instead of captured graphs
    c->nw.fuse = getenv("MGF_NO_FUSE") == nullptr;
    c->nw.use_graphs = getenv("MGF_NO_GRAPHS") == nullptr;
    c->nw.smoother_only = getenv("MGF_SMOOTHER_ONLY") != nullptr;
    c->nw.rb_fused = getenv("MGF_HALF_SWEEPS") == nullptr;
    if (getenv("MGF_ONE_SWEEP")) c->nw.sweep2_max_nodes = 0;
    if (getenv("MGF_NO_SWEEP_RESTRICT")) c->nw.sweep2_restrict = false;
    if (const char *e = getenv("MGF_TWO_SWEEP_PRE_NODES")) c->nw.sweep2_pre_max_nodes = atoll(e);
    if (const char *e = getenv("MGF_TWO_SWEEP_NODES")) c->nw.sweep2_max_nodes = atoll(e);
    if (const char *e = getenv("MGF_CHAIN_MAX_BLOCKS")) c->nw.chain_max_blocks = atoi(e);
    if (const char *e = getenv("MGF_SWEEP_ROWS"))
        for (int l = 0; l < c->nlev; ++l) c->lev[l].g.sh = atoi(e) == 16 ? 16 : 8;
    if (const char *e = getenv("MGF_SWEEP2_ROWS"))
        for (int l = 0; l < c->nlev; ++l) c->lev[l].g.sh2 = atoi(e) == 4 ? 4 : 8;
    hipError_t e = hipHostMalloc((void **)&c->pinned, kPinnedDoubles * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&c->pinned_dev, c->pinned, 0);
    if (e != hipSuccess) {
        if (c->pinned) (void)hipHostFree(c->pinned);
        delete c;
        return fail(MG_EHIP, "hipHostMalloc: %s", hipGetErrorString(e));
    }
    e = hipMemsetAsync(workspace, 0, (size_t)need, c->stream);
    // level tables
    std::vector<double> zl, wr, fr, dz, dzc, wl;
    for (int l = 0; l < c->nlev && e == hipSuccess; ++l) {
        Level &L = c->lev[l];
        zl.resize(L.g.nz + 1);
        for (int j = 0; j <= L.g.nz; ++j) zl[j] = c->zhost[(size_t)j << l];
        level_tables(desc, zl.data(), L.g.nr, L.g.nz, wr, fr, dz, dzc, wl);
        e = hipMemcpyAsync((void *)L.g.wr, wr.data(), wr.size() * 8, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync((void *)L.g.fr, fr.data(), fr.size() * 8, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync((void *)L.g.z, zl.data(), zl.size() * 8, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync((void *)L.g.dz, dz.data(), dz.size() * 8, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync((void *)L.g.dzc, dzc.data(), dzc.size() * 8, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync((void *)L.g.wl, wl.data(), wl.size() * 8, hipMemcpyHostToDevice, c->stream);
        // the host vectors are reused next level: wait for the copies
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    if (e != hipSuccess) {
        (void)hipHostFree(c->pinned);
        delete c;
        return fail(MG_EHIP, "mg_setup: %s", hipGetErrorString(e));
    }
    *out = c;
    return MG_OK;
}

void mg_destroy(mg_ctx *ctx) {
    if (!ctx) return;
    // work still queued (a speculative Arnoldi step) may copy into pinned memory
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->active_host) (void)hipHostFree(ctx->active_host);
    for (hipEvent_t ev : ctx->active_ev)
        if (ev) (void)hipEventDestroy(ev);
    if (ctx->bpinned) (void)hipHostFree(ctx->bpinned);
    drop_graphs(ctx);
    if (ctx->nw.cap) (void)hipStreamDestroy(ctx->nw.cap);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
}

int mg_levels(const mg_ctx *ctx) { return ctx ? ctx->nlev : MG_EINVAL; }

int mg_level_shape(const mg_ctx *ctx, int level, int32_t *nr, int32_t *nz, int64_t *pitch) {
    if (int st = check_ctx(ctx)) return st;
    if (level < 0 || level >= ctx->nlev) return fail(MG_EINVAL, "bad level %d", level);
    const Geom &g = ctx->lev[level].g;
    if (nr) *nr = g.nr;
    if (nz) *nz = g.nz;
    if (pitch) *pitch = g.pitch;
    return MG_OK;
}

int sg_assemble(mg_ctx *c, int eq, const mg_physics *ph, const mg_state *st, double dt) {
    if (int e = check_ctx(c)) return e;
    if (int e = check_eq(eq)) return e;
    if (!ph || !st) return fail(MG_EINVAL, "null physics or state");
    hipStream_t s = c->stream;
    const Geom &g0 = c->lev[0].g;
    if (eq == MG_EQ_POISSON) {
        if (!st->ne || !st->np || !st->V) return fail(MG_EINVAL, "Poisson needs V, ne and np");
        launch_set_electrodes(g0, st->V, ph->V_bottom, ph->V_top, s);
        launch_set_wall(g0, st->V, ph->V_bottom, ph->V_top, s);
        for (int l = 0; l < c->nlev; ++l)
            launch_poisson_assemble(c->lev[l].g, c->lev[l].op[eq], st->ne, st->np, ph->k, l == 0, ph->V_bottom,
                                    ph->V_top, s);
    } else {
        bool el = eq == MG_EQ_ELECTRON;
        double *n = el ? st->ne : st->np;
        const double *S = el ? st->Se : st->Sp;
        double mu = el ? ph->mu_e : ph->mu_p;
        double D = el ? ph->D_e : ph->D_p;
        if (!st->V || !n) return fail(MG_EINVAL, "continuity needs V and the density");
        if (!(D > 0) || !(mu >= 0)) return fail(MG_EINVAL, "need D > 0 and mu >= 0");
        double sgn = el ? -1.0 : 1.0;
        double q = -sgn * mu / D;
        double dt_inv = (dt > 0 && isfinite(dt)) ? 1.0 / dt : 0.0;
        const double *mun = el ? st->mue : st->mup, *Dn = el ? st->De : st->Dp;
        if ((mun == nullptr) != (Dn == nullptr)) return fail(MG_EINVAL, "node mobility and diffusion go together");
        launch_set_electrodes(g0, n, el ? ph->ne_bottom : ph->np_bottom, el ? ph->ne_top : ph->np_top, s);
        launch_set_wall(g0, n, 0.0, 0.0, s);
        const double *V = st->V;
        for (int l = 0; l < c->nlev; ++l) {
            const Level &L = c->lev[l];
            if (l > 0) {
                launch_inject(c->lev[l - 1].g, V, L.g, L.vinj, s);
                V = L.vinj;
                if (mun) {  // node transport injected like the potential
                    launch_inject(c->lev[l - 1].g, mun, L.g, L.muinj, s);
                    launch_inject(c->lev[l - 1].g, Dn, L.g, L.Dinj, s);
                    mun = L.muinj;
                    Dn = L.Dinj;
                }
            }
            launch_sg_assemble(L.g, L.op[eq], V, l == 0 ? n : nullptr, l == 0 ? S : nullptr, q, D, dt_inv, s, mun,
                               Dn, sgn);
        }
    }
    const Level &Lc = c->lev[c->nlev - 1];
    if (c->desc.prec == MG_FP32_IR)
        for (int l = 0; l < c->nlev; ++l) launch_op_to_f32(c->lev[l].g, c->lev[l].op[eq], c->lev[l].op32[eq], s);
    launch_coarse_factor(Lc.g, Lc.op[eq], c->coarse_scratch, Lc.cinv[eq], Lc.cinv32[eq], s);
    c->assembled[eq] = true;
    HIP_OK(hipGetLastError());
    return MG_OK;
}

int vcycle(mg_ctx *c, int eq, double *x, int32_t ncycles, double *relres_out) {
    if (int e = check_ctx(c)) return e;
    if (int e = check_eq(eq)) return e;
    if (!x) return fail(MG_EINVAL, "null x");
    if (!c->assembled[eq]) return fail(MG_EINVAL, "equation %d not assembled", eq);
    for (int k = 0; k < ncycles; ++k) one_cycle(c, eq, x);
    HIP_OK(hipGetLastError());
    if (relres_out) return relres64(c, eq, x, relres_out);
    return MG_OK;
}

int mg_relres(mg_ctx *c, int eq, const double *x, double *relres_out) {
    if (int e = check_ctx(c)) return e;
    if (int e = check_eq(eq)) return e;
    if (!x || !relres_out) return fail(MG_EINVAL, "null pointer");
    if (!c->assembled[eq]) return fail(MG_EINVAL, "equation %d not assembled", eq);
    return relres64(c, eq, x, relres_out);
}

int mg_solve(mg_ctx *c, int eq, double *x, double rtol, int32_t max_cycles, int32_t *cycles_out,
             double *relres_out) {
    if (int e = check_ctx(c)) return e;
    if (int e = check_eq(eq)) return e;
    if (!x) return fail(MG_EINVAL, "null x");
    if (!c->assembled[eq]) return fail(MG_EINVAL, "equation %d not assembled", eq);
    double rr = 0;
    int st = relres64(c, eq, x, &rr);
    if (st) return st;
    int k = 0;
    while (isfinite(rr) && rr > rtol && k < max_cycles) {
        one_cycle(c, eq, x);
        ++k;
        st = relres64(c, eq, x, &rr);
        if (st) return st;
    }
    if (cycles_out) *cycles_out = k;
    if (relres_out) *relres_out = rr;
    if (!isfinite(rr)) return fail(MG_ENONFINITE, "residual is not finite after %d cycles", k);
    if (rr > rtol) return fail(MG_ENOCONV, "relative residual %.3e > %.3e after %d cycles", rr, rtol, k);
    return MG_OK;
}

int mg_copy_coef(mg_ctx *c, int eq, int level, int which, double *dst) {
    if (int e = check_ctx(c)) return e;
    if (int e = check_eq(eq)) return e;
    if (level < 0 || level >= c->nlev || which < 0 || which > 5 || !dst)
        return fail(MG_EINVAL, "bad level/which/dst");
    const Level &L = c->lev[level];
    const double *src[6] = {L.op[eq].a, L.op[eq].b, L.op[eq].c, L.op[eq].d, L.op[eq].e, L.op[eq].f};
    HIP_OK(hipMemcpyAsync(dst, src[which], (size_t)(L.g.nr + 1) * L.g.pitch * sizeof(double),
                          hipMemcpyDeviceToDevice, c->stream));
    return MG_OK;
}

int mg_smooth_half(mg_ctx *c, int eq, double *x, int colour) {
    if (int e = check_ctx(c)) return e;
    if (int e = check_eq(eq)) return e;
    if (!x || (colour != 0 && colour != 1)) return fail(MG_EINVAL, "bad x or colour");
    const Level &L = c->lev[0];
    if (c->desc.smoother == MG_SMOOTH_RB)
        launch_rbgs<double>(L.g, L.op[eq], x, colour, c->stream);
    else
        launch_zline<double>(L.g, L.op[eq], x, colour, c->stream);
    HIP_OK(hipGetLastError());
    return MG_OK;
}

int mg_residual(mg_ctx *c, int eq, const double *x, double *r) {
    if (int e = check_ctx(c)) return e;
    if (int e = check_eq(eq)) return e;
    if (!x || !r) return fail(MG_EINVAL, "null x or r");
    const Level &L = c->lev[0];
    launch_residual<double, double, double>(L.g, L.op[eq], nullptr, x, r, nullptr, nullptr, c->stream);
    HIP_OK(hipGetLastError());
    return MG_OK;
}

static int decoupled_step(mg_ctx *c, const mg_physics *ph, mg_state *st, double dt, const mg_schedule *sc,
                          mg_report *rep) {
    int total = 0, cyc = 0;
    double rr = 0, worst = 0;
    // Poisson with the densities of step k
    int e = sg_assemble(c, MG_EQ_POISSON, ph, st, dt);
    if (e) return e;
    e = mg_solve(c, MG_EQ_POISSON, st->V, sc->lin_rtol, sc->max_cycles, &cyc, &rr);
    total += cyc;
    worst = rr > worst ? rr : worst;
    if (e) return e;
    // SG continuity for the electrons, then the ions, with the new potential
    for (int eq = MG_EQ_ELECTRON; eq <= MG_EQ_ION; ++eq) {
        e = sg_assemble(c, eq, ph, st, dt);
        if (e) return e;
        e = mg_solve(c, eq, eq == MG_EQ_ELECTRON ? st->ne : st->np, sc->lin_rtol, sc->max_cycles, &cyc, &rr);
        total += cyc;
        worst = rr > worst ? rr : worst;
        if (e) return e;
    }
    if (rep) {
        rep->vcycles += total;
        rep->final_relres = worst;
        rep->steps += 1;
    }
    return MG_OK;
}

int implicit_step(mg_ctx *c, const mg_physics *ph, mg_state *st, double dt, const mg_schedule *sc,
                  mg_report *rep) {
    if (int e = check_ctx(c)) return e;
    if (!ph || !st || !sc) return fail(MG_EINVAL, "null physics, state or schedule");
    if (!st->V || !st->ne || !st->np) return fail(MG_EINVAL, "state needs V, ne and np");
    if (!(dt > 0)) return fail(MG_EINVAL, "dt must be positive");
    if (sc->coupling == MG_COUPLE_DECOUPLED) return decoupled_step(c, ph, st, dt, sc, rep);
    if (sc->coupling != MG_COUPLE_NEWTON) return fail(MG_EINVAL, "bad coupling %d", sc->coupling);
    if (!st->Se || !st->Sp) return fail(MG_EINVAL, "the Newton step needs both sources");
    bool conv = false;
    int e = newton_implicit_step(c, ph, st, dt, sc, rep, &conv);
    if (e) return e;
    if (!conv) return fail(MG_ENOCONV, "Newton did not converge in %d iterations", sc->max_newton);
    return MG_OK;
}

int solve_steady(mg_ctx *c, const mg_physics *ph, mg_state *st, const mg_schedule *sc, mg_report *rep) {
    if (int e = check_ctx(c)) return e;
    if (!ph || !st || !sc) return fail(MG_EINVAL, "null physics, state or schedule");
    if (!st->V || !st->ne || !st->np || !st->Se || !st->Sp) return fail(MG_EINVAL, "incomplete state");
    if (!(sc->dt0 > 0) || !(sc->growth >= 1.0) || !(sc->dt_max >= sc->dt0))
        return fail(MG_EINVAL, "bad time-step schedule");
    if (sc->coupling == MG_COUPLE_NEWTON) return newton_solve_steady(c, ph, st, sc, rep);
    if (sc->coupling != MG_COUPLE_DECOUPLED) return fail(MG_EINVAL, "bad coupling %d", sc->coupling);
    // decoupled steps (stable only while dt stays below the dielectric
    // relaxation time); no rejection logic beyond solver failure
    mg_report local;
    memset(&local, 0, sizeof local);
    mg_report *R = rep ? rep : &local;
    memset(R, 0, sizeof *R);
    auto t0 = std::chrono::steady_clock::now();
    double dt = sc->dt0;
    int64_t p0 = (int64_t)(c->lev[0].g.nr + 1) * c->lev[0].g.pitch;
    int status = MG_ENOCONV;
    while (R->steps < sc->max_steps) {
        launch_copy_field(c->lev[0].g, st->ne, c->spare[0], c->stream);
        launch_copy_field(c->lev[0].g, st->np, c->spare[1], c->stream);
        int e = decoupled_step(c, ph, st, dt, sc, R);
        if (e) return e;
        R->t_end += dt;
        int nb = 0;
        launch_diff_norms(c->lev[0].g, st->ne, c->spare[0], c->partials, &nb, c->stream);
        launch_sum_partials(c->partials, nb, 2, c->scal, c->stream);
        launch_diff_norms(c->lev[0].g, st->np, c->spare[1], c->partials, &nb, c->stream);
        launch_sum_partials(c->partials, nb, 2, c->scal + 2, c->stream);
        HIP_OK(hipMemcpyAsync(c->pinned, c->scal, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_OK(hipStreamSynchronize(c->stream));
        const double *o = c->pinned;
        double ch = fmax(sqrt(o[0] / fmax(o[1], 1e-300)), sqrt(o[2] / fmax(o[3], 1e-300)));
        R->last_change = ch;
        if (!isfinite(ch)) {
            status = fail(MG_ENONFINITE, "density change is not finite");
            break;
        }
        if (ch < sc->steady_tol) {
            status = MG_OK;
            break;
        }
        dt = fmin(sc->growth * dt, sc->dt_max);
    }
    (void)p0;
    R->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (status == MG_ENOCONV) fail(MG_ENOCONV, "not steady after %d steps", R->steps);
    return status;
}

int mg_time_kernel(mg_ctx *c, int which, int eq, int32_t reps, double *avg_ms) {
    if (int e = check_ctx(c)) return e;
    if (!avg_ms || reps < 1) return fail(MG_EINVAL, "bad reps or null output");
    if (which == 0 || which == 4 || which == 5 || which == 6)
        return time_block_smoother(c, reps, which == 6 ? 3 : which == 5 ? 2 : which == 4 ? 1 : 0, eq, avg_ms);
    if (int e = check_eq(eq)) return e;
    if (!c->assembled[eq]) return fail(MG_EINVAL, "equation %d not assembled", eq);
    if (which < 1 || which > 3) return fail(MG_EINVAL, "bad kernel id %d", which);
    const Level &L = c->lev[0];
    double *x = c->spare[0], *r = c->spare[1];
    launch_copy_field(L.g, L.op[eq].f, x, c->stream);
    hipEvent_t a, b;
    HIP_OK(hipEventCreate(&a));
    HIP_OK(hipEventCreate(&b));
    HIP_OK(hipEventRecord(a, c->stream));
    for (int k = 0; k < reps; ++k) {
        if (which == 1)
            launch_zline<double>(L.g, L.op[eq], x, k & 1, c->stream);
        else if (which == 2)
            launch_rbgs<double>(L.g, L.op[eq], x, k & 1, c->stream);
        else
            launch_residual<double, double, double>(L.g, L.op[eq], nullptr, x, r, nullptr, nullptr, c->stream);
    }
    HIP_OK(hipEventRecord(b, c->stream));
    HIP_OK(hipEventSynchronize(b));
    float ms = 0;
    HIP_OK(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *avg_ms = ms / reps;
    return MG_OK;
}

int mg_steady_residual(mg_ctx *c, const mg_physics *ph, const mg_state *st, double *norm_out) {
    if (int e = check_ctx(c)) return e;
    if (!ph || !st || !norm_out || !st->V || !st->ne || !st->np || !st->Se || !st->Sp)
        return fail(MG_EINVAL, "null argument");
    return steady_residual(c, ph, st, norm_out);
}

int mg_boundary_flow(mg_ctx *c, const mg_physics *ph, const mg_state *st, double *out) {
    if (int e = check_ctx(c)) return e;
    if (!ph || !st || !out || !st->V || !st->ne || !st->np) return fail(MG_EINVAL, "null argument");
    if (!(ph->D_e > 0) || !(ph->D_p > 0)) return fail(MG_EINVAL, "need D_e, D_p > 0");
    const Geom &g = c->lev[0].g;
    hipStream_t s = c->stream;
    if ((st->mue == nullptr) != (st->De == nullptr) || (st->mup == nullptr) != (st->Dp == nullptr))
        return fail(MG_EINVAL, "node mobility and diffusion go together");
    launch_boundary_flow(g, st->V, st->ne, ph->mu_e / ph->D_e, ph->D_e, c->scal, s, st->mue, st->De, -1.0);
    launch_boundary_flow(g, st->V, st->np, -ph->mu_p / ph->D_p, ph->D_p, c->scal + 3, s, st->mup, st->Dp, 1.0);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(c->pinned, c->scal, 6 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    for (int k = 0; k < 6; ++k) out[k] = c->pinned[k];
    return MG_OK;
}

int mg_transport_table(mg_ctx *c, const double *V, const double *E_tab, const double *mu_tab, const double *D_tab,
                       int32_t ntab, double *mu_out, double *D_out) {
    if (int e = check_ctx(c)) return e;
    if (!V || !E_tab || !mu_tab || !D_tab || !mu_out || !D_out) return fail(MG_EINVAL, "null argument");
    if (ntab < 2) return fail(MG_EINVAL, "a table needs at least 2 entries (got %d)", ntab);
    launch_transport_table(c->lev[0].g, V, E_tab, mu_tab, D_tab, ntab, mu_out, D_out, c->stream);
    HIP_OK(hipGetLastError());
    return MG_OK;
}

int mg_newton_precond(mg_ctx *c, const mg_physics *ph, const mg_state *st, double dt, const double *r,
                      double *z) {
    if (int e = check_ctx(c)) return e;
    if (!ph || !st || !r || !z || !st->V || !st->ne || !st->np || !st->Se || !st->Sp)
        return fail(MG_EINVAL, "null argument");
    if (!(dt > 0)) return fail(MG_EINVAL, "dt must be > 0 (infinity for the steady Jacobian)");
    return newton_precond(c, ph, st, dt, r, z);
}

int wn_param_count(void) { return kWnParams; }

int wn_scratch_bytes(int32_t B, int32_t H, int32_t W, int64_t *bytes) {
    if (B < 1 || H < 1 || W < 1 || !bytes) return fail(MG_EINVAL, "bad image batch shape");
    *bytes = wn_scratch_size(B, H, W);
    return MG_OK;
}

static int wn_check(const void *a, const void *b, int32_t B, int32_t H, int32_t W, const void *scratch,
                    int64_t bytes) {
    if (!a || !b || !scratch) return fail(MG_EINVAL, "null pointer");
    if (B < 1 || H < 1 || W < 1) return fail(MG_EINVAL, "bad image batch shape %d x %d x %d", B, H, W);
    if (bytes < wn_scratch_size(B, H, W)) return fail(MG_ENOMEM, "scratch too small");
    if (reinterpret_cast<uintptr_t>(scratch) % 256) return fail(MG_EINVAL, "scratch must be 256-byte aligned");
    return MG_OK;
}

int wn_forward(const float *params, const float *in, float *out, int32_t B, int32_t H, int32_t W, void *scratch,
               int64_t scratch_bytes, void *stream) {
    if (int e = wn_check(params, in, B, H, W, scratch, scratch_bytes)) return e;
    if (!out) return fail(MG_EINVAL, "null output");
    return wn_forward_impl(params, in, out, B, H, W, scratch, reinterpret_cast<hipStream_t>(stream));
}

int wn_grad(const float *params, const float *in, const float *target, int32_t B, int32_t H, int32_t W,
            float *grad_out, double *loss_out, void *scratch, int64_t scratch_bytes, void *stream) {
    if (int e = wn_check(params, in, B, H, W, scratch, scratch_bytes)) return e;
    if (!target) return fail(MG_EINVAL, "null target");
    return wn_grad_impl(params, in, target, B, H, W, grad_out, loss_out, scratch,
                        reinterpret_cast<hipStream_t>(stream));
}

int wn_train_step(float *params, float *adam_m, float *adam_v, int32_t step, float lr, const float *in,
                  const float *target, int32_t B, int32_t H, int32_t W, double *loss_out, void *scratch,
                  int64_t scratch_bytes, void *stream) {
    if (int e = wn_check(params, in, B, H, W, scratch, scratch_bytes)) return e;
    if (!target || !adam_m || !adam_v || step < 1) return fail(MG_EINVAL, "bad Adam state or target");
    return wn_train_impl(params, adam_m, adam_v, step, lr, in, target, B, H, W, loss_out, scratch,
                         reinterpret_cast<hipStream_t>(stream));
}

int wn_features(mg_ctx *c, const mg_state *up, double V_top, double ratio, float *out, double *nscale_dev) {
    if (int e = check_ctx(c)) return e;
    if (!up || !up->V || !up->ne || !up->np || !out || !nscale_dev) return fail(MG_EINVAL, "null argument");
    if (!(V_top != 0) || !(ratio > 0)) return fail(MG_EINVAL, "need V_top != 0 and ratio > 0");
    launch_features(c->lev[0].g, up->V, up->ne, up->np, c->desc.R, c->desc.d, V_top, ratio, nscale_dev, out,
                    c->stream);
    HIP_OK(hipGetLastError());
    return MG_OK;
}

int wn_targets(mg_ctx *c, const mg_state *up, const mg_state *steady, double V_top, const double *nscale_dev,
               float *out) {
    if (int e = check_ctx(c)) return e;
    if (!up || !steady || !out || !nscale_dev) return fail(MG_EINVAL, "null argument");
    launch_targets(c->lev[0].g, up->V, up->ne, up->np, steady->V, steady->ne, steady->np, V_top, nscale_dev, out,
                   c->stream);
    HIP_OK(hipGetLastError());
    return MG_OK;
}

int wn_apply(mg_ctx *c, const mg_state *up, const float *pred, double V_top, const double *nscale_dev,
             const mg_physics *phys, mg_state *dst) {
    if (int e = check_ctx(c)) return e;
    if (!up || !pred || !nscale_dev || !phys || !dst) return fail(MG_EINVAL, "null argument");
    launch_apply(c->lev[0].g, up->V, up->ne, up->np, pred, V_top, nscale_dev, dst->V, dst->ne, dst->np, *phys,
                 c->stream);
    HIP_OK(hipGetLastError());
    return MG_OK;
}

int mg_set_tuning(mg_ctx *c, int32_t rows_per_block, int32_t fuse_max_n) {
    if (int e = check_ctx(c)) return e;
    if (rows_per_block != 1 && rows_per_block != 2 && rows_per_block != 4 && rows_per_block != 8 &&
        rows_per_block != 16)
        return fail(MG_EINVAL, "rows_per_block must be 1, 2, 4, 8 or 16");
    if (fuse_max_n < 0 || fuse_max_n > 128) return fail(MG_EINVAL, "fuse_max_n outside 0..128");
    if (fuse_max_n > 0) {
        // the fused range must hold at most kMaxFused levels and a coarsest
        // grid small enough for its LDS
        int first = c->nlev;
        for (int l = 0; l < c->nlev; ++l)
            if (c->lev[l].g.nr <= fuse_max_n && c->lev[l].g.nz <= fuse_max_n) {
                first = l;
                break;
            }
        if (c->nlev - first > 8) return fail(MG_EINVAL, "fuse_max_n = %d would fuse more than 8 levels", fuse_max_n);
    }
    for (int l = 0; l < c->nlev; ++l) c->lev[l].g.ty = rows_per_block;
    c->nw.fuse = fuse_max_n > 0;
    c->nw.fuse_max = fuse_max_n;
    drop_graphs(c);
    return MG_OK;
}

int mg_batch_query(const mg_grid_desc *desc, int32_t nprob, int64_t *stride_bytes, int64_t *workspace_bytes) {
    if (int st = validate(desc)) return st;
    if (desc->krylov_m < 1) return fail(MG_EINVAL, "a batch needs krylov_m >= 1 (Newton path)");
    if (nprob < 1 || nprob > 65535) return fail(MG_EINVAL, "nprob = %d outside 1..65535", nprob);
    int64_t ws = 0, so = 0, to = 0;
    int64_t total = batch_layout(desc, nprob, &ws, &so, &to);
    if (stride_bytes) *stride_bytes = to / nprob;
    if (workspace_bytes) *workspace_bytes = total;
    return MG_OK;
}

int mg_batch_setup(const mg_grid_desc *desc, int32_t nprob, void *workspace, int64_t workspace_bytes,
                   void *stream, mg_ctx **out) {
    if (int st = mg_batch_query(desc, nprob, nullptr, nullptr)) return st;
    if (!workspace || !out) return fail(MG_EINVAL, "null workspace or output");
    if (reinterpret_cast<uintptr_t>(workspace) % kAlign)
        return fail(MG_EINVAL, "workspace must be %d-byte aligned", (int)kAlign);
    return batch_setup(desc, nprob, workspace, workspace_bytes, stream, out);
}

int mg_batch_state(mg_ctx *c, int32_t p, mg_state *out) {
    if (int e = check_ctx(c)) return e;
    if (!out) return fail(MG_EINVAL, "null output");
    if (!c->ws_base) return fail(MG_EINVAL, "not a batch context");
    return batch_state(c, p, out);
}

int solve_steady_batch(mg_ctx *c, const mg_physics *phys, const mg_schedule *sc, mg_report *reports) {
    if (int e = check_ctx(c)) return e;
    if (!phys || !sc) return fail(MG_EINVAL, "null physics or schedule");
    if (!c->ws_base) return fail(MG_EINVAL, "not a batch context");
    if (sc->coupling != MG_COUPLE_NEWTON) return fail(MG_EINVAL, "batched solves use the Newton coupling");
    if (!(sc->dt0 > 0) || !(sc->growth >= 1.0) || !(sc->dt_max >= sc->dt0))
        return fail(MG_EINVAL, "bad time-step schedule");
    for (int p = 0; p < c->bt.n; ++p)
        if (!(phys[p].D_e > 0) || !(phys[p].D_p > 0)) return fail(MG_EINVAL, "problem %d: need D > 0", p);
    return batch_solve_steady(c, phys, sc, reports);
}

int solve_steady_batches(mg_ctx *const *batches, int32_t nbatch, const mg_physics *const *phys,
                         const mg_schedule *sc, mg_report *const *reports) {
    if (!batches || !phys || !sc || !reports) return fail(MG_EINVAL, "null argument");
    if (nbatch < 1 || nbatch > 64) return fail(MG_EINVAL, "nbatch = %d outside 1..64", nbatch);
    for (int i = 0; i < nbatch; ++i) {
        if (!batches[i] || !phys[i] || !reports[i]) return fail(MG_EINVAL, "batch %d: null argument", i);
        if (int e = check_ctx(batches[i])) return e;
        if (!batches[i]->ws_base) return fail(MG_EINVAL, "batch %d: not a batch context", i);
        for (int j = 0; j < i; ++j)
            if (batches[j] == batches[i]) return fail(MG_EINVAL, "batch %d is also batch %d", i, j);
    }
    // one host thread per batch, on the batch's device; each thread's status
    // and error message are collected and the first failing batch reported
    std::vector<int> status(nbatch, MG_OK);
    std::vector<std::string> msg(nbatch);
    std::vector<std::thread> threads;
    threads.reserve(nbatch);
    for (int i = 0; i < nbatch; ++i)
        threads.emplace_back([&, i] {
            mg_ctx *c = batches[i];
            if (hipSetDevice(c->device) != hipSuccess) {
                status[i] = MG_EHIP;
                msg[i] = "hipSetDevice failed";
                return;
            }
            status[i] = solve_steady_batch(c, phys[i], sc, reports[i]);
            if (status[i]) msg[i] = mg_last_error();
        });
    for (auto &t : threads) t.join();
    for (int i = 0; i < nbatch; ++i)
        if (status[i]) return fail(status[i], "batch %d: %s", i, msg[i].c_str());
    return MG_OK;
}

int prolong_state(mg_ctx *coarse, const mg_state *src, mg_ctx *fine, mg_state *dst, const mg_physics *ph) {
    if (!coarse || !fine || !src || !dst || !ph) return fail(MG_EINVAL, "null argument");
    const Geom &gc = coarse->lev[0].g;
    if (fine->nlev < 2 || fine->lev[1].g.nr != gc.nr || fine->lev[1].g.nz != gc.nz)
        return fail(MG_EINVAL, "fine grid must be the 2x refinement of the coarse grid");
    for (int j = 0; j <= gc.nz; ++j)
        if (coarse->zhost[j] != fine->zhost[2 * j])
            return fail(MG_EINVAL, "z nodes are not nested at j = %d", j);
    // tables of the fine level 0 carry the weights; the coarse fields use the
    // coarse context's pitch, which equals the fine context's level-1 pitch.
    const Geom &gf = fine->lev[0].g;
    hipStream_t s = fine->stream;
    HIP_OK(hipStreamSynchronize(coarse->stream));
    launch_prolong_state(gf, dst->V, gc, src->V, s);
    launch_prolong_state(gf, dst->ne, gc, src->ne, s);
    launch_prolong_state(gf, dst->np, gc, src->np, s);
    set_boundary(gf, dst->V, dst->ne, dst->np, *ph, s);
    HIP_OK(hipGetLastError());
    return MG_OK;
}

}  // extern "C"
