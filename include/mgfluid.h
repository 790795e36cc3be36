/*
 * mgfluid.h -- C ABI of the MI355X (gfx950) multigrid solver for the
 * axisymmetric 2D drift-diffusion fluid equations of Ristivojevic & Petrovic,
 * "Multigrid solver for axisymmetrical 2D fluid equations" (arXiv:0811.4446).
 *
 * Problem (Sec. 2): electron and ion densities n_e, n_p and potential V on
 * (r, z) in [0, R] x [0, d]; continuity Eqs. (1)-(2) with drift-diffusion
 * fluxes Eqs. (3)-(4), Poisson Eq. (5).  Axisymmetric; radial nodes
 * r_i = i R / nr (equidistant), axial nodes z_j given (non-equidistant).
 * Electrodes at z = 0 and z = d (Dirichlet), zero radial flux at r = 0, and
 * at r = R either zero radial flux or the Dirichlet wall of the paper's
 * experiment (Sec. 3; mg_grid_desc.r_outer_bc).
 *
 * Memory.  Every device field is a row-major (nr+1) x pitch array of
 * doubles, element (i, j) at [i*pitch + j], i = radial node, j = axial node,
 * z contiguous; pitch comes from mg_query.  Columns j > nz are padding and
 * never read.  All device memory (fields and the workspace) is allocated and
 * owned by the caller; the library owns only its host-side context.
 *
 * Streams.  Every call enqueues its kernels on the stream given to
 * mg_setup (a hipStream_t passed as void*).  Calls that must read a norm
 * (mg_solve, implicit_step, solve_steady, and vcycle with a non-NULL
 * relres_out) synchronise that stream before returning.
 *
 * Errors.  0 on success, a negative MG_E* code on failure; mg_last_error()
 * returns a message for the calling thread.  Arguments are validated before
 * any device work.  A context is not thread-safe; distinct contexts on
 * distinct streams are independent.
 */
#ifndef MGFLUID_H
#define MGFLUID_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MG_ABI_VERSION 2

#define MG_OK 0
#define MG_EINVAL (-1)      /* bad argument (null pointer, grid, enum, version) */
#define MG_EHIP (-2)        /* a HIP runtime call failed                        */
#define MG_ENOCONV (-3)     /* not converged within the cycle/step budget       */
#define MG_ENONFINITE (-4)  /* a norm became NaN or Inf                          */
#define MG_EREJECT (-5)     /* time step rejected past the retry budget          */
#define MG_ENOMEM (-6)      /* workspace smaller than mg_query reported          */

typedef struct mg_ctx mg_ctx;

typedef enum { MG_FP64 = 0, MG_FP32_IR = 1 } mg_prec;
typedef enum { MG_EQ_POISSON = 0, MG_EQ_ELECTRON = 1, MG_EQ_ION = 2 } mg_eq;
/* Smoothers.  MG_SMOOTH_RB: red-black point Gauss-Seidel (scalar
 * equations) and collective red-black (the 3x3 node blocks of the Newton
 * system, Eq. 14).  MG_SMOOTH_ZEBRA: zebra z-line Gauss-Seidel for the
 * scalar equations, collective red-black for the Newton system.
 * MG_SMOOTH_ZEBRA_BLOCK: zebra z-line for both; on the Newton system each
 * axial line's 3x3-block tridiagonal system along z is solved exactly
 * (block Thomas), even lines first, on every level above the coarsest. */
typedef enum { MG_SMOOTH_RB = 0, MG_SMOOTH_ZEBRA = 1, MG_SMOOTH_ZEBRA_BLOCK = 2 } mg_smoother;
typedef enum { MG_COUPLE_DECOUPLED = 0, MG_COUPLE_NEWTON = 2 } mg_coupling;

/* Grid and multigrid configuration.
 *   nr, nz       radial / axial intervals; min(nr, nz) = coarsest_n * 2^L and
 *                both divisible by 2^L (L coarsenings, nested grids)
 *   R, d         domain [0, R] x [0, d]
 *   z_host       host array of nz+1 strictly increasing axial nodes with
 *                z[0] = 0 and z[nz] = d; copied during mg_setup
 *   coarsest_n   smaller dimension of the coarsest grid (>= 2; default 8)
 *   nu1, nu2     pre- and post-smoothing sweeps of the V-cycle
 *   smoother     mg_smoother (above)
 *   prec         mg_prec: FP64 cycles, or FP32 cycles inside FP64
 *                iterative refinement
 *   krylov_m     restart length of the FGMRES solver of the coupled
 *                Newton systems (Eq. 14); 0 leaves that path (and its
 *                workspace) out, max 40
 *   r_outer_bc   boundary at r = R: MG_WALL_ZERO_FLUX (0: zero radial
 *                flux, half control volume) or MG_WALL_DIRICHLET (1: the
 *                paper's wall, Sec. 3: potential interpolated linearly in z
 *                between V_bottom and V_top, densities 0).  With the
 *                Dirichlet wall the nodes i = nr are fixed on every level:
 *                their equations are u = u_wall (identity rows), the rows
 *                of i = nr-1 couple to them through the face r_{nr-1/2}.  */
#define MG_WALL_ZERO_FLUX 0
#define MG_WALL_DIRICHLET 1
typedef struct {
    int32_t abi_version;
    int32_t nr, nz;
    double R, d;
    const double *z_host;
    int32_t coarsest_n, nu1, nu2;
    int32_t smoother, prec;
    int32_t krylov_m;
    int32_t r_outer_bc;
} mg_grid_desc;

/* Physics of Eqs. (3)-(5): mobilities, diffusion coefficients, the Poisson
 * coupling k = e n0 / eps0, and the electrode (Dirichlet) values. */
typedef struct {
    double mu_e, mu_p, D_e, D_p, k;
    double V_bottom, V_top;
    double ne_bottom, ne_top, np_bottom, np_top;
} mg_physics;

/* Device state in the field layout above (caller-owned).
 *   mue, De, mup, Dp  optional node values of the mobilities and diffusion
 *                     coefficients (Sec. 2: mu(E), D(E) supplied by lookup
 *                     tables or a Monte Carlo code, e.g. mg_transport_table);
 *                     NULL: the constants of mg_physics.  Set mue and De (or
 *                     mup and Dp) together.  Each face uses the arithmetic
 *                     mean of its two nodes' values, alpha = -s mu/D (Eq. 10)
 *                     with the face values; the values are held fixed during
 *                     a solve (the Newton Jacobian differentiates in V, n
 *                     only).  Not supported by batches. */
typedef struct {
    double *V, *ne, *np;
    const double *Se, *Sp;
    const double *mue, *De, *mup, *Dp;
} mg_state;

/* Time-stepping schedule (Sec. 2, last paragraphs): dt starts at dt0 and
 * is multiplied by `growth` after each accepted step, capped at dt_max.
 * The run stops when max over species of ||n^{k+1}-n^k||_2/||n^{k+1}||_2 <
 * steady_tol.  Linear solves stop at relative residual lin_rtol.  A step
 * is rejected (and retried with the previous dt, then halved) when a
 * solve fails or the Newton correction exceeds reject_limit. */
typedef struct {
    double dt0, growth, dt_max, steady_tol, lin_rtol;
    int32_t max_steps, max_cycles, coupling, max_newton;
    double newton_tol, reject_limit;
} mg_schedule;

/* Counts of a step or a steady run.  final_relres: weighted relative
 * residual of the last linear solve (Newton path: FGMRES's recurrence value
 * when that met lin_rtol, else the true residual of the iterate; decoupled
 * path: the largest final relres of the step's three V-cycle solves). */
typedef struct {
    int32_t steps, rejected, vcycles, newton_its;
    double last_change, final_relres, seconds, t_end;
} mg_report;

/* Pitch (elements per row of a level-0 field) and workspace size in bytes.
 * Pure host computation, no HIP call.  Returns MG_EINVAL for a bad grid. */
int mg_query(const mg_grid_desc *desc, int64_t *pitch_elems, int64_t *workspace_bytes);

/* Build a context over caller-allocated device workspace of at least the
 * size mg_query reported (256-byte aligned).  Computes the per-level grid
 * tables of Sec. 2 (nested coarse grids) and zeroes the workspace on
 * `stream`.  The context keeps pointers into the workspace; the caller keeps
 * it alive until mg_destroy. */
int mg_setup(const mg_grid_desc *desc, void *workspace, int64_t workspace_bytes,
             void *stream, mg_ctx **out);

/* Free the host-side context (the workspace stays the caller's). */
void mg_destroy(mg_ctx *ctx);

/* Assemble equation `eq` on every grid level.
 *   MG_EQ_POISSON   Eqs. (12)-(13) in finite-volume form with the charge of
 *                   st->ne, st->np on the finest level (dt unused)
 *   MG_EQ_ELECTRON, MG_EQ_ION
 *                   backward-Euler Scharfetter-Gummel operator, Eqs. (7)-(11),
 *                   with potential st->V (injected to the coarse levels),
 *                   old density st->ne / st->np and source st->Se / st->Sp;
 *                   dt <= 0 or dt = +inf gives the steady operator.
 * Also writes the electrode values of `phys` into the electrode rows of the
 * field that the equation solves for. */
int sg_assemble(mg_ctx *ctx, int eq, const mg_physics *phys, const mg_state *st, double dt);

/* Run `ncycles` V(nu1, nu2) cycles on equation `eq` (assembled before) for
 * the device field x (electrode rows hold the boundary values).  If
 * relres_out is non-NULL the strong-form relative residual after the last
 * cycle is written there (this synchronises the stream). */
int vcycle(mg_ctx *ctx, int eq, double *x, int32_t ncycles, double *relres_out);

/* V-cycles until the strong-form relative residual ||(f-Ax)/vol||_2 /
 * ||b/vol||_2 <= rtol, at most max_cycles.  MG_ENOCONV leaves the last
 * iterate in x.  In MG_FP32_IR mode each refinement step runs FP32 cycles
 * on the FP64 residual (defect correction). */
int mg_solve(mg_ctx *ctx, int eq, double *x, double rtol, int32_t max_cycles,
             int32_t *cycles_out, double *relres_out);

/* Strong-form relative residual of x for equation eq (synchronises). */
int mg_relres(mg_ctx *ctx, int eq, const double *x, double *relres_out);

/* One backward-Euler step of length dt, Eq. (7).
 *   MG_COUPLE_DECOUPLED: Poisson with the densities of step k, then the SG
 *     electron and ion equations with the new potential.
 *   MG_COUPLE_NEWTON: Newton-Raphson on the coupled system (Eq. 14); the
 *     report's last_change is the largest relative l1 size (per field) of
 *     the last Newton correction.
 * st is updated in place; rep (optional) receives counts. */
int implicit_step(mg_ctx *ctx, const mg_physics *phys, mg_state *st, double dt,
                  const mg_schedule *sched, mg_report *rep);

/* Backward-Euler steps with growing dt until the densities are steady
 * (Sec. 2, multilevel prolongation paragraph and the time-step rule). */
int solve_steady(mg_ctx *ctx, const mg_physics *phys, mg_state *st,
                 const mg_schedule *sched, mg_report *rep);

/* Weighted 2-norm of the steady residual F(u) of the coupled system
 * (Eqs. 7-13 with dt = infinity; Poisson rows scaled by 1/k, every row by
 * 1/vol) at the state st; needs krylov_m >= 1.  Synchronises. */
int mg_steady_residual(mg_ctx *ctx, const mg_physics *phys, const mg_state *st, double *norm_out);

/* Node transport from tables of the field strength (Sec. 2: mu(E), D(E)
 * from lookup tables): |E| = |grad V| at every node of the finest grid
 * (central differences, one-sided at the electrodes and at r = R, radial
 * component 0 on the axis), then piecewise-linear interpolation in the
 * table (E_tab strictly increasing, ntab >= 2; clamped outside), written to
 * mu_out and D_out (device fields, caller-owned, every node).  E_tab,
 * mu_tab, D_tab: device arrays of ntab doubles.  Asynchronous. */
int mg_transport_table(mg_ctx *ctx, const double *V, const double *E_tab, const double *mu_tab,
                       const double *D_tab, int32_t ntab, double *mu_out, double *D_out);

/* Particle flow out of the domain through its boundaries at the state st,
 * per radian of azimuth (multiply by 2 pi for the whole discharge, and by
 * the elementary charge for a current): the Scharfetter-Gummel face fluxes
 * of Eqs. (8)-(9) through the cathode (z = 0), the anode (z = d) and, with
 * the Dirichlet wall, the wall face r_{nr-1/2}, summed with the faces'
 * areas over the control volumes of the unknown nodes.  out (host, 6
 * doubles): electrons {cathode, anode, wall}, ions {cathode, anode, wall}.
 * The paper's observable (Sec. 3) is the ion current to the cathode,
 * 2 pi e out[3].  At a steady state each species' outflow sum equals its
 * source integral.  Synchronises. */
int mg_boundary_flow(mg_ctx *ctx, const mg_physics *phys, const mg_state *st, double *out);

/* The preconditioner of the Newton linear solves on its own (Sec. 2: the
 * Jacobian system of Eq. (14) solved by multigrid): assembles the 3x3-block
 * Jacobian at the state st on every level (coarse levels at the injected
 * state) for a backward-Euler step of size dt (dt = +inf: the steady
 * Jacobian), factors the coarsest level, and applies one collective
 * red-black block V(nu1, nu2) cycle from a zero guess: z = M r.  r and z are
 * device pointers to three consecutive planes (n_e, n_p, V rows), each
 * (nr+1) x pitch FP64, caller-owned; r's electrode rows are ignored, z's are
 * written as zero.  The block V-cycle runs in FP32 when the context was
 * built with MG_FP32_IR (r and z stay FP64).  Needs krylov_m >= 1 and a
 * single-problem context; overwrites the context's Newton work arrays.
 * MG_EINVAL: null pointers, dt <= 0 or NaN, batch context.  Synchronises. */
int mg_newton_precond(mg_ctx *ctx, const mg_physics *phys, const mg_state *st, double dt, const double *r,
                      double *z);

/* Multilevel prolongation (Sec. 2): interpolate the state of the grid of
 * `coarse` onto the twice finer grid of `fine` (bilinear, the multigrid
 * prolongation), electrode rows set from phys.  Both contexts must share R,
 * d and the nested z nodes. */
int prolong_state(mg_ctx *coarse, const mg_state *src, mg_ctx *fine, mg_state *dst,
                  const mg_physics *phys);

/* ---- batches of independent problems (a parameter sweep) ----
 * A batch holds nprob problems of one grid shape (desc; krylov_m >= 1) in
 * one workspace: problem p owns the p-th of nprob equal-stride regions
 * (its solver workspace and its V, ne, np, Se, Sp fields), and every kernel
 * launch advances all problems of the batch (problem index = blockIdx.z).
 * Physics (mobilities, voltages) may differ per problem; k must not. */

/* Stride between problem regions and total workspace bytes.  Pure host. */
int mg_batch_query(const mg_grid_desc *desc, int32_t nprob, int64_t *stride_bytes, int64_t *workspace_bytes);

/* Context over a caller-allocated batch workspace (256-byte aligned). */
int mg_batch_setup(const mg_grid_desc *desc, int32_t nprob, void *workspace, int64_t workspace_bytes,
                   void *stream, mg_ctx **out);

/* Device pointers of problem p's fields inside the batch workspace (the
 * caller writes the initial state and sources there). */
int mg_batch_state(mg_ctx *batch, int32_t p, mg_state *out);

/* Steady solves of every problem of the batch (Sec. 2 time-step rule,
 * coupled Newton; the schedule is shared, dt and the step decisions are per
 * problem); phys and reports are host arrays of nprob entries.  Returns the
 * worst per-problem status. */
int solve_steady_batch(mg_ctx *batch, const mg_physics *phys, const mg_schedule *sched, mg_report *reports);

/* Several batches at once (e.g. one per grid size of a parameter sweep with
 * uneven sizes): solve_steady_batch for every batch, each driven by a host
 * thread of its own on the device current at its setup, so that the
 * batches' launches overlap on the GPU when their contexts were set up on
 * different streams (on one stream they run one after another).  phys[i]
 * and reports[i] are host arrays of batch i's nprob entries; a batch may
 * appear once.  Blocks until every batch has finished; returns MG_OK or the
 * status of the lowest-numbered batch that failed, with its message. */
int solve_steady_batches(mg_ctx *const *batches, int32_t nbatch, const mg_physics *const *phys,
                         const mg_schedule *sched, mg_report *const *reports);

/* ---- learned warm start (replaces the coarse-to-fine extrapolation of the
 * multilevel prolongation, Sec. 2) ----
 * Network: four 3x3 convolutions with zero padding, 7 -> 32 -> 32 -> 32 -> 3
 * channels, GELU in its erf form (z Phi(z), not the tanh approximation;
 * Phi evaluated in FP32 to 2.4e-6 relative) after the first three.
 * Parameters: one FP32
 * device array of wn_param_count() values, per layer W[co][ci][3][3] then
 * b[co].  Images are FP32 NCHW: inputs [B][7][H][W], outputs and targets
 * [B][3][H][W], with H = nr+1 (radial nodes) and W = nz+1 (axial nodes).
 * The convolutions run in bf16 on MFMA with FP32 accumulation.  `scratch`
 * is caller-allocated device memory of wn_scratch_bytes(B, H, W) bytes.
 * wn_forward runs the four layers in one kernel per 16 x 16 output tile with
 * the activations on chip (batches beyond 2^24 such tiles return
 * MG_EINVAL); wn_grad and wn_train_step store every layer's activations in
 * scratch for the backward pass, so their forward outputs can differ from
 * wn_forward's in the last bf16 bits (summation order of the first layer).
 * All calls are asynchronous on `stream` unless they return a loss. */
int wn_param_count(void);
int wn_scratch_bytes(int32_t B, int32_t H, int32_t W, int64_t *bytes);
int wn_forward(const float *params, const float *in, float *out, int32_t B, int32_t H, int32_t W,
               void *scratch, int64_t scratch_bytes, void *stream);
/* Mean squared error over all outputs and its gradient w.r.t. params
 * (grad_out: device, wn_param_count() floats; loss_out: host, synchronises). */
int wn_grad(const float *params, const float *in, const float *target, int32_t B, int32_t H, int32_t W,
            float *grad_out, double *loss_out, void *scratch, int64_t scratch_bytes, void *stream);
/* One Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8; `step` counts from
 * 1) on params with moments adam_m, adam_v (device, FP32, zero initially). */
int wn_train_step(float *params, float *adam_m, float *adam_v, int32_t step, float lr, const float *in,
                  const float *target, int32_t B, int32_t H, int32_t W, double *loss_out, void *scratch,
                  int64_t scratch_bytes, void *stream);
/* wn_forward without a scratch argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the packed bf16 weights live in one
 * static device array per GPU (155 KB, held until the process ends), so the
 * call allocates nothing.  The forward pass keeps its activations on chip,
 * so the array does not grow with the image: any batch of at most 2^24
 * tiles of 16 x 16 pixels is accepted, larger ones return MG_EINVAL.  Same
 * kernels and results as wn_forward (bitwise).  Calls that overlap on one
 * GPU share that array and race: serialise them (one stream, or events).
 * Call with the stream's device current; the first call on a device looks
 * up its array's address. */
int wn_forward_noalloc(const float *params, const float *in, float *out, int32_t B, int32_t H, int32_t W,
                       void *stream);
/* Input planes of one sample (out: [7][H][W]) from the prolonged coarse
 * state `up` on the grid of `fine`: V/V_top, n_e/n_s, n_p/n_s, r/R, z/d,
 * V_top/5, log10(ratio)/3, where n_s (written to nscale_dev, one device
 * double) is the largest prolonged density. */
int wn_features(mg_ctx *fine, const mg_state *up, double V_top, double ratio, float *out, double *nscale_dev);
/* Training target: 100 x (steady - up) in the same units (out: [3][H][W]). */
int wn_targets(mg_ctx *fine, const mg_state *up, const mg_state *steady, double V_top, const double *nscale_dev,
               float *out);
/* Initial state from the prediction: dst = up + prediction / 100 in
 * physical units, densities clamped at zero, electrode rows from phys. */
int wn_apply(mg_ctx *fine, const mg_state *up, const float *pred, double V_top, const double *nscale_dev,
             const mg_physics *phys, mg_state *dst);

/* Launch shape chosen by the autotuner: radial rows per workgroup of the 2D
 * kernels (1, 2, 4, 8 or 16; the workgroup spans 64 axial nodes), and the
 * largest level (nr, nz <= fuse_max_n) run inside the single-workgroup
 * coarse sub-cycle of the Newton preconditioner (0 disables it).  Results
 * change only by summation order.  Default 4 and 16. */
int mg_set_tuning(mg_ctx *ctx, int32_t rows_per_block, int32_t fuse_max_n);

/* ---- introspection used by the tests (kernel-level parity) ---- */

/* Number of levels and the size of level l. */
int mg_levels(const mg_ctx *ctx);
int mg_level_shape(const mg_ctx *ctx, int level, int32_t *nr, int32_t *nz, int64_t *pitch);

/* Copy coefficient `which` (0..5 = a, b, c, d, e, f) of equation eq on
 * level l into the device buffer dst ((nr_l+1) x pitch_l doubles). */
int mg_copy_coef(mg_ctx *ctx, int eq, int level, int which, double *dst);

/* One smoothing half-sweep (colour/parity 0 or 1) of equation eq on level
 * 0 applied to x, with the configured smoother. */
int mg_smooth_half(mg_ctx *ctx, int eq, double *x, int colour);

/* r = f - A x on the unknown nodes of level 0 (0 on electrode rows). */
int mg_residual(mg_ctx *ctx, int eq, const double *x, double *r);

/* Time one kernel of the hot path: `reps` back-to-back launches on the
 * context's stream between two HIP events; *avg_ms receives the mean
 * duration of one launch.  which: 0 collective red-black block smoother
 * half-sweep of the Newton system (needs an assembled Jacobian), 1 zebra
 * z-line half-sweep, 2 point red-black half-sweep, 3 residual (scalar
 * equation `eq`, assembled before; level 0), 4 full collective red-black
 * sweep in one launch (both colours; assembled Jacobian), 5 two full
 * collective red-black sweeps in one launch (assembled Jacobian; what the
 * block V-cycle launches on small levels when nu1 and nu2 are even), 6 the
 * same two sweeps followed in the same launch by the residual restricted to
 * the next coarser level (the V-cycle's last pre-smoothing launch on those
 * levels; needs a coarser level).  For the block kernels (0, 4, 5, 6) `eq`
 * is the grid level (0 = finest).  Overwrites that level's work vectors
 * (and for 6 the coarser level's right-hand side) only.  Synchronises. */
int mg_time_kernel(mg_ctx *ctx, int which, int eq, int32_t reps, double *avg_ms);

/* Thread-local message of the last error. */
const char *mg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MGFLUID_H */
