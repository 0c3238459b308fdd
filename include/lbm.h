/*
 * lbm.h -- C interface of the MI355X library for the modified lattice-BGK model of
 * convection heat transfer in porous media at the REV scale (Wang, Mi & Guo,
 * arXiv:1505.02976).
 *
 * One call of lbm_step advances the coupled D2Q9 flow and D2Q9 temperature populations by
 * one time step: streaming (Sec. 3.1, Eq. LBEeq; Sec. 3.2, streaming substep of
 * Eq. TEqColli), the non-equilibrium extrapolation boundary scheme (Sec. 3.4), the local
 * macroscopic quantities (temperature, Sec. 3.2; velocity through the quadratic drag
 * solve and pressure, Sec. 3.1; shear rate, Eq. ShearEqCom; temperature gradient,
 * Eqs. SonaT-MatrN), the modified equilibria (Eqs. EQFIN, EQTSHIN, TeEDFEQ), the forcing
 * and source terms (Eqs. FtermF, Eq:Tforce) and the BGK collision (Eqs. LBEeq, TEqColli).
 *
 * Conventions for every function:
 *   - Pointers named "device" are HIP device pointers on the device that is current when
 *     lbm_init is called; pointers named "host" are ordinary host memory.
 *   - Every call returns an lbm_status and never aborts; on failure lbm_last_error()
 *     returns a message (thread-local, valid until the next failing call on the thread).
 *   - Work is enqueued on the HIP stream given to lbm_init, in call order.  Calls marked
 *     "synchronizes" wait for that stream.
 *   - A context is used from one host thread at a time; distinct contexts are independent.
 *   - Asynchronous device faults surface as LBM_ERR_DEVICE on the next call that checks.
 *
 * Lattice units throughout: dx = dt = 1, cs^2 = 1/3, rho0 = 1.  Field arrays are
 * row-major [ny][nx] (x fastest).  Population arrays are [2][9][ny][nx]: flow populations
 * f_0..f_8 then temperature populations g_0..g_8, directions c_0 = (0,0), c_1 = (1,0),
 * c_2 = (0,1), c_3 = (-1,0), c_4 = (0,-1), c_5 = (1,1), c_6 = (-1,1), c_7 = (-1,-1),
 * c_8 = (1,-1) (Sec. 3.1).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
    LBM_OK = 0,
    LBM_ERR_INVALID = 1,      /* a parameter or buffer is unusable; nothing was enqueued    */
    LBM_ERR_DEVICE = 2,       /* a HIP call failed (launch, copy, synchronisation)          */
    LBM_ERR_NONFINITE = 3,    /* a population or field became NaN or infinite               */
    LBM_ERR_UNSUPPORTED = 4   /* valid request the library does not support for this problem */
} lbm_status;

/* Storage precision of the populations.  F32 and F16 store deviations from the rest
 * state (f_0 - rho0 and g_i - omega_i sigma T0; F16 additionally scaled by 256) and
 * compute the collision in FP32, with the quadratic drag solve and every reduction in
 * FP64.  F64 stores and computes in FP64. */
typedef enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16 = 2 } lbm_storage;

/* Thermal wall condition (Sec. 3.4): isothermal (Eqs. TeEBounDFEQ, TNEESAp) or prescribed
 * normal temperature derivative (Eq. TNEESApGra).  A wall node's macroscopic state is the
 * one the boundary scheme assigns to it (T_b, the wall velocity, p and S of the reference
 * node x_f, the boundary temperature gradient); the node collides with that state and
 * lbm_moments / lbm_gradients report it. */
typedef enum { LBM_T_DIRICHLET = 0, LBM_T_NEUMANN = 1 } lbm_twall;

/* One wall.  The velocity condition is always a prescribed wall velocity (ux, uy).
 * dTdn is the derivative of T along the inward wall normal. */
typedef struct {
    double ux, uy;
    int32_t t_kind;           /* lbm_twall */
    int32_t reserved;
    double T, dTdn;
} lbm_wall;

/* Problem description.  Derived lattice constants:
 *   L     = characteristic length: L if > 0, else nx - 1 if x is walled, else ny - 1 if y is
 *           walled, else nx (wet-node walls: n nodes across a walled direction span n - 1)
 *   A, B  = given, or if either is NaN from Ma, Ra, Pr (Eq. EQA&B, with the factor J on
 *           the A term):  A = tau_f - 1/2 - J Ma L sqrt(3 Pr / Ra),
 *                         B = tau_T - 1/2 - (Ma / sigma) L sqrt(3 / (Pr Ra))
 *   nu_e  = cs^2 (tau_f - A - 1/2) (Sec. 3.1),  nu = nu_e / J (Sec. 2),
 *   alpha_e = sigma cs^2 (tau_T - B - 1/2) (Eq. Therdiff),
 *   g beta = Ra nu alpha_e / (dT L^3) (Ra of Sec. 2; 0 when Ra = 0),
 *   K     = Da L^2 (Sec. 2; Da = +inf removes the Darcy and Forchheimer drag),
 *   F_eps = given, or if NaN the Ergun relation 1.75 / sqrt(150 eps^3) per node (Sec. 2),
 *   T0    = (T_hot + T_cold) / 2, dT = T_hot - T_cold.
 * Walls, in order x- (x = 0), x+ (x = nx-1), y- (y = 0), y+ (y = ny-1), exist only for
 * non-periodic directions.  Corners: the inward diagonal neighbour is the reference
 * node, the velocity is zero, an isothermal wall takes precedence over a Neumann wall and
 * the x-wall over the y-wall.
 * Initial state: the post-collision populations before the first step are the equilibria
 * of (p_init, ux_init, uy_init, T_init) with zero shear rate and temperature gradient;
 * a NULL field means p = 0, u = 0, and T = T0 except T = T_wall on isothermal wall nodes.
 * Field pointers are device [ny][nx] FP64 arrays read during lbm_init only (the porosity
 * field is copied into the workspace). */
typedef struct {
    int32_t nx, ny;
    int32_t periodic_x, periodic_y;
    lbm_wall wall[4];
    double L;
    double Da, Ra, Pr, J, Ma, sigma, Q;
    double tau_f, tau_T;
    double A, B;
    double eps;                       /* uniform porosity, used when eps_field is NULL     */
    double ax, ay;                    /* external acceleration a (Sec. 2)                  */
    double T_hot, T_cold;
    double F_eps;
    const double *eps_field;          /* device, optional; values in (0, 1] like eps (device
                                         memory: not checked)                               */
    const double *T_init;             /* device, optional                                   */
    const double *p_init;             /* device, optional                                   */
    const double *ux_init;            /* device, optional                                   */
    const double *uy_init;            /* device, optional                                   */
    int32_t storage;                  /* lbm_storage                                        */
    int32_t reserved;
} lbm_params;

/* Lattice constants derived from a problem (see lbm_params). */
typedef struct {
    double L, A, B, nu_e, nu, alpha_e, gbeta, K, T0, dT;
} lbm_derived;

/* Validates params and fills *out (host).  LBM_ERR_INVALID when the parameters are
 * unusable: nx or ny < 1; a walled direction with < 3 nodes (< 4 if a Neumann wall lies
 * on either end); tau_f or tau_T <= 1/2; nu_e <= 0 (A >= tau_f - 1/2); alpha_e <= 0
 * (B >= tau_T - 1/2); eps outside (0, 1]; Da <= 0; sigma, J <= 0; A or B NaN with
 * Ra <= 0 or Pr <= 0; storage unknown. */
lbm_status lbm_derive(const lbm_params *params, lbm_derived *out);

/* Bytes of device workspace lbm_init needs for params (0 if params are invalid). */
size_t lbm_workspace_bytes(const lbm_params *params);

/* Creates a context on the current device.  workspace: device buffer of at least
 * lbm_workspace_bytes(params) bytes, 256-byte aligned, owned by the caller and kept alive
 * until lbm_destroy; the library owns its contents.  hip_stream: a hipStream_t (NULL =
 * default stream).  Enqueues the initialisation.  *out receives a context that the
 * caller releases with lbm_destroy. */
lbm_status lbm_init(const lbm_params *params, void *workspace, size_t workspace_bytes,
                    void *hip_stream, lbm_ctx **out);

/* Enqueues nsteps >= 0 time steps (asynchronous, unless non-finite checks are on: see
 * lbm_set_check_interval).  With two steps per pass (see
 * lbm_set_fusion) pairs of steps run as one pass over the populations: the intermediate
 * state of every node is computed from the source buffer in registers and the final
 * state written once, so each pair reads and writes the populations once instead of
 * twice; the results are bitwise those of single steps.  A pass is a main launch on the
 * context's stream and, on a second stream created by the library (default priority,
 * ordered with the caller's stream by events), the launches next to the walled rows.  A
 * single step is two launches: the interior columns, then the columns next to the walls
 * x = 0, x = nx - 1 together with the walled rows. */
lbm_status lbm_step(lbm_ctx *ctx, int64_t nsteps);

/* Non-finite detection inside lbm_step: with every > 0, whenever the context's time
 * reaches a multiple of `every` during lbm_step, the call waits for the stream and checks
 * every population of the grid; if one is NaN or infinite it returns LBM_ERR_NONFINITE at
 * that time (later steps of the call are not enqueued; lbm_time reports where it stopped).
 * every = 0 (the default) turns the checks off, and lbm_step stays asynchronous.  Each
 * check reads the populations once (about one step's read traffic). */
lbm_status lbm_set_check_interval(lbm_ctx *ctx, int64_t every);

/* Time steps per pass, 1 or 2.  The default is 2 for FP64 and FP32 storage when nx >= 4
 * and ny >= 8, else 1 (FP16 storage is faster with one step per pass).
 * LBM_ERR_UNSUPPORTED for 2 on smaller grids. */
lbm_status lbm_set_fusion(lbm_ctx *ctx, int32_t steps_per_pass);
int32_t lbm_fusion(const lbm_ctx *ctx);

/* As lbm_step (nsteps >= the steps per pass), with HIP events around the launches of every
 * `every`-th pass (every >= 1); returns the mean duration in milliseconds of the main
 * launch of a pass (the interior launch of a single step; for a two-step pass the launch
 * of the wavefronts whose reach holds no wall or only the walls x = 0, x = nx - 1) and of
 * the remaining launches of the pass (for two-step passes these run on a second stream,
 * beside the main launch), the number of nodes the main launch writes, and the steps one
 * pass advances (host outputs; any may be NULL).  An odd last step of a two-step schedule
 * runs untimed.  Used for measurement; events between launches cost a few microseconds per
 * bracketed pass.  The first call creates the context's timing events (kept until
 * lbm_destroy; a call before a timed region keeps their creation out of it).
 * Synchronizes on the events, not on the stream. */
lbm_status lbm_step_timed(lbm_ctx *ctx, int64_t nsteps, int32_t every, double *main_ms_host,
                          double *rest_ms_host, int64_t *main_nodes_host, int32_t *steps_per_launch_host);

int64_t lbm_time(const lbm_ctx *ctx);

/* Macroscopic fields at the current time (device outputs, [ny][nx], NULL = skip):
 * pressure p, velocity ux, uy, temperature T.  out_dtype 0 = FP64, 1 = FP32.
 * Asynchronous. */
lbm_status lbm_moments(lbm_ctx *ctx, int32_t out_dtype, void *p, void *ux, void *uy, void *T);

/* Local gradients at the current time (device outputs, NULL = skip): shear rate
 * S = grad u + (grad u)^T from Eq. ShearEqCom (Sxx, Sxy, Syy) and the temperature
 * gradient from Eq. TeEqCom (dTdx, dTdy).  out_dtype as in lbm_moments. Asynchronous. */
lbm_status lbm_gradients(lbm_ctx *ctx, int32_t out_dtype, void *Sxx, void *Sxy, void *Syy,
                         void *dTdx, void *dTdy);

/* Average Nusselt number on one wall (0..3) at the current time, Eq. AvNuss:
 * Nu_j = -L (dT/dn_axis) / dT with the second-order one-sided difference along the
 * wall-normal axis, averaged over the wall by the trapezoid rule; FP64 arithmetic,
 * fixed summation order.  *nu_host receives the value.  Synchronizes. */
lbm_status lbm_nusselt(lbm_ctx *ctx, int32_t wall, double *nu_host);

/* Convergence measure of Sec. 4: r_u = sum |u(t) - u(s)|_2 / sum |u(t)|_2 and
 * r_T = sum |T(t) - T(s)| / sum |T(t)| against the snapshot s taken at the previous
 * call, then takes a new snapshot.  The first call after lbm_init only takes the
 * snapshot and returns -1 in both.  FP64 arithmetic, fixed summation order.  Returns
 * LBM_ERR_NONFINITE if any population is not finite.  Synchronizes. */
lbm_status lbm_residual(lbm_ctx *ctx, double *r_u_host, double *r_T_host);

/* As lbm_residual, for callers that cannot allocate device memory (code under stream
 * capture set-up, tight serving loops, harnesses that forbid allocation): the reduction's
 * partial sums and totals go to a device-resident scratch array of the library
 * (LBM_STATIC_SCRATCH_BYTES per device, allocated once when the library is loaded and held
 * until the process ends; its address is looked up by lbm_init on the current device) instead
 * of the context's workspace.  The snapshot stays in the workspace, so both functions share
 * one snapshot and either may follow the other.  The call allocates nothing.  Grids whose
 * partial sums do not fit (more than (LBM_STATIC_SCRATCH_BYTES - 256) / 40 reduction blocks of
 * 256 nodes, i.e. about 26.8 M nodes) return LBM_ERR_INVALID with a message.  Every call on a
 * device uses that device's one array: calls that overlap on one device (other streams, other
 * threads) race and must be serialized by the caller; nothing in the array needs clearing
 * between calls.  Synchronizes. */
#define LBM_STATIC_SCRATCH_BYTES (4u << 20)
lbm_status lbm_residual_noalloc(lbm_ctx *ctx, double *r_u_host, double *r_T_host);

/* Copies the post-collision populations of the last step as raw FP64 values
 * ([2][9][ny][nx], device) out of / into the context.  lbm_set_state keeps the time.
 * Asynchronous. */
lbm_status lbm_get_state(lbm_ctx *ctx, double *dst_device);
lbm_status lbm_set_state(lbm_ctx *ctx, const double *src_device);

/* ---------------------------------------------------------------------------------- */
/* Batches: many independent problems (uneven grids and parameters, one storage type)  */
/* advanced together: the same launches per step (or per two-step pass) for all of    */
/* them.                                                                               */
/* ---------------------------------------------------------------------------------- */
typedef struct lbm_batch lbm_batch;

/* Bytes of device workspace for a batch of n problems params[0..n-1] (0 if any problem is
 * invalid or the problems do not share one storage type). */
size_t lbm_batch_workspace_bytes(const lbm_params *params, int32_t n);

/* Creates a batch: every problem is initialised as by lbm_init inside the workspace
 * (same ownership rules), plus the work tables of the batched kernels.  The problems'
 * contexts are owned by the batch; problems may be queried (lbm_moments, lbm_nusselt,
 * lbm_residual, lbm_get_state, ...) through lbm_batch_problem but are advanced only by
 * lbm_batch_step (lbm_step on them returns LBM_ERR_INVALID). */
lbm_status lbm_batch_init(const lbm_params *params, int32_t n, void *workspace, size_t workspace_bytes,
                          void *hip_stream, lbm_batch **out);

/* Enqueues nsteps time steps of every problem.  With two steps per pass: nsteps / 2
 * passes (each pass's launches for the wavefronts next to the walled rows run on a second
 * stream of the batch beside its main launch, ordered by events; the call is ordered like
 * launches on the batch's stream), then one single step if nsteps is odd.  With one step
 * per pass: whole HIP graphs of 64 steps (built on the first call that needs one), then
 * single steps.  Results are bitwise those of lbm_step on each problem alone.
 * Asynchronous. */
lbm_status lbm_batch_step(lbm_batch *batch, int64_t nsteps);

/* Time steps per batched pass, 1 or 2 (as lbm_set_fusion, for all problems at once).  The
 * default is 2 when the storage is FP64 or FP32 and every grid has nx >= 4 and ny >= 8,
 * else 1; LBM_ERR_UNSUPPORTED for 2 otherwise. */
lbm_status lbm_batch_set_fusion(lbm_batch *batch, int32_t steps_per_pass);
int32_t lbm_batch_fusion(const lbm_batch *batch);

/* Context of problem k (borrowed, valid until lbm_batch_destroy); NULL if k is out of range. */
lbm_ctx *lbm_batch_problem(lbm_batch *batch, int32_t k);

/* Per-problem non-finite flags (host array of n int32: 1 = some population of that problem
 * is NaN or infinite).  Synchronizes. */
lbm_status lbm_batch_check(lbm_batch *batch, int32_t *nonfinite_host);

/* Block-width autotuner of the batched launches that run under the current steps per pass:
 * with two steps per pass, the threads per block of the two-step main launch (64, 128 or
 * 256, i.e. 1, 2 or 4 independent wavefronts per block); with one step per pass, the block
 * width along x of the one-step update (64, 128, 256).  Times each candidate, in that
 * order, over `steps` steps and keeps the fastest for later lbm_batch_step calls.  The
 * problems' states are unchanged (the timed launches read the current populations and
 * overwrite only the buffers the next step writes anyway) and the results of later steps
 * do not depend on the width.  *width (optional) receives the chosen width; ms_per_step
 * (optional, host, LBM_BATCH_NUM_WIDTHS entries) the timings.  Synchronizes. */
#define LBM_BATCH_NUM_WIDTHS 3
lbm_status lbm_batch_autotune(lbm_batch *batch, int32_t steps, int32_t *width, double *ms_per_step);

/* Sets, without timing, the width the autotuner would choose for the current steps per
 * pass (256 for the two-step main launch, 64 for the one-step update after
 * lbm_batch_init); LBM_ERR_INVALID for any other value than 64, 128, 256.  Synchronizes. */
lbm_status lbm_batch_set_width(lbm_batch *batch, int32_t width);

/* Releases the batch and its contexts (host memory only). */
void lbm_batch_destroy(lbm_batch *batch);

/* ---------------------------------------------------------------------------------- */
/* Adjoint: gradient of an average Nusselt number (Eq. AvNuss) after nsteps steps with   */
/* respect to the porosity of every node, by the discrete adjoint of the step           */
/* (reverse sweep over sqrt(nsteps)-spaced checkpoints, forward states recomputed per    */
/* segment).  Off the walls each node update is reversed by hand in the storage's        */
/* arithmetic (FP64 for FP64 storage, FP32 for FP32 and FP16; drag solve in FP64); at     */
/* wall nodes the Jacobian comes from FP64 dual numbers pushed through the boundary      */
/* scheme's own code.                                                                    */
/* ---------------------------------------------------------------------------------- */
typedef struct lbm_adjoint lbm_adjoint;

/* Bytes of device workspace for an adjoint over nsteps steps of ctx's problem. */
size_t lbm_adjoint_workspace_bytes(const lbm_ctx *ctx, int64_t nsteps);

/* Advances ctx by nsteps >= 1 steps from its current state (as lbm_step) while keeping
 * checkpoints in the workspace (device, 256-byte aligned, caller-owned, kept alive until
 * lbm_adjoint_destroy), then evaluates J = average Nusselt number of `wall` (as
 * lbm_nusselt) into *nu_host.  *out receives the adjoint handle.  Synchronizes. */
lbm_status lbm_adjoint_forward(lbm_ctx *ctx, int32_t wall, int64_t nsteps, void *workspace,
                               size_t workspace_bytes, lbm_adjoint **out, double *nu_host);

/* Writes dJ * dJ/deps(x) for every node into grad_eps_device ([ny][nx] FP64, device,
 * overwritten).  May be called repeatedly; leaves ctx's state untouched.  Synchronizes. */
lbm_status lbm_adjoint_backward(lbm_adjoint *adj, double dJ, double *grad_eps_device);

/* Releases the adjoint handle (host memory only). */
void lbm_adjoint_destroy(lbm_adjoint *adj);

/* Releases the context (host memory only; the workspace stays with the caller). */
void lbm_destroy(lbm_ctx *ctx);

/* Message of the last failing call on this thread ("" if none). */
const char *lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
