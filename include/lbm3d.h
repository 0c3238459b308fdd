/*
 * lbm3d.h - C interface of the three-dimensional path: the modified lattice-BGK model of
 * Wang, Mi & Guo (arXiv:1505.02976), Secs. 2-3 (equilibria Eqs. EQFIN, EQTSHIN, TeEDFEQ;
 * forcing Eq. FtermF; sources Eq. Eq:Tforce; shear rate Eq. ShearEqCom; temperature
 * gradient Eqs. MatrM, MatrN, TeEqCom; drag solve of Sec. 3.1) on the D3Q19 lattice for the
 * flow and the temperature populations, with the non-equilibrium extrapolation of Sec. 3.4
 * at the walls.  Sec. 3.1 states the model for two dimensions and notes that it extends
 * to three; the tensor expressions carry over unchanged, with omega_0 = 1/3 in the
 * pressure formula and in the closed forms of s_0 and F_0 (App. A).
 *
 * Geometry: x, y and z each either periodic or bounded by walls at 0 and n - 1 (x_f is
 * the next node inward along the wall normal).  Buoyancy acts along +z.  A
 * wall node's macroscopic state is the one the boundary scheme assigns to it (T_b, the wall
 * velocity, p and S of x_f, the boundary temperature gradient); it collides with that
 * state, and lbm3_fields reports it.  On an edge or a vertex where two or three walls
 * meet, x_f is the inward diagonal neighbour, the wall is at rest, an isothermal wall's
 * temperature wins over a prescribed gradient (among isothermal walls x first, then y,
 * then z) and each prescribed gradient sets its own normal component of grad T, as at the
 * corners of the two-dimensional path (Sec. 3.4 applied along each normal).
 *
 * Units, status codes, storage types and thread rules are those of lbm.h.  Arrays are
 * [z][y][x] with x fastest; vector fields are consecutive planes (x, y, z components).
 * The populations live in a caller-provided device workspace as two buffers of 2 x 19
 * planes (flow, temperature), in deviation form as in two dimensions (FP16 scaled by 256, as
 * there); the arithmetic is in the storage precision (FP64 or FP32; FP32 for FP16 storage),
 * with the drag solve in FP64.
 */
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm3_ctx lbm3_ctx;

/* One wall (index 0: z = 0, 1: z = nz - 1, 2: x = 0, 3: x = nx - 1, 4: y = 0, 5: y = ny - 1;
 * walls of a periodic direction are ignored).  dTdn is the derivative of T along the inward normal; t_kind is
 * lbm_twall. */
typedef struct {
    double u[3];
    int32_t t_kind;
    int32_t reserved;
    double T, dTdn;
} lbm3_wall;

/* Problem description.  L = characteristic length: L if > 0, else nx - 1 (walled x), else
 * nz - 1 (walled z) or nz (periodic z).  A, B given, or if either is NaN from Ma, Ra, Pr (Eq. EQA&B).  nu_e, alpha_e,
 * g beta, K, T0 and dT follow as in two dimensions (lbm.h).  eps_field ([nz][ny][nx], FP64,
 * device, values in (0, 1]) gives the porosity per node and must stay valid until
 * lbm3_destroy (the kernels read it every step; K = Da L^2 stays uniform, F_eps follows the
 * Ergun relation per node unless given); NULL means the uniform eps.  T_init ([nz][ny][nx])
 * and u_init (3 planes) are optional FP64 device arrays read during lbm3_init only; NULL
 * means T = T0 (T_wall on isothermal wall nodes, in the order x, y, z where walls meet) and
 * u = 0; p starts at 0 (gauge pressure). */
typedef struct {
    int32_t nx, ny, nz, periodic_x, periodic_y, periodic_z;
    lbm3_wall wall[6];
    double L, Da, Ra, Pr, J, Ma, sigma, Q;
    double tau_f, tau_T, A, B;
    double eps;
    double a[3];                 /* external acceleration */
    double T_hot, T_cold;
    double F_eps;                /* NaN => Ergun relation 1.75 / sqrt(150 eps^3) */
    int32_t storage;             /* LBM_F64, LBM_F32 or LBM_F16 */
    int32_t reserved;
    const double *T_init;
    const double *u_init;
    const double *eps_field;
} lbm3_params;

/* Workspace bytes lbm3_init needs for this problem: two population buffers and 256 bytes
 * for reduction results (0 if the problem is invalid; lbm_last_error says why).  Unusable:
 * nx, ny, nz < 1 (periodic) or < 4 (walled); storage other than F64/F32/F16; tau <= 1/2;
 * nu_e, alpha_e or K not positive. */
size_t lbm3_workspace_bytes(const lbm3_params *params);

/* Creates a context on the current device.  workspace: device memory of at least
 * lbm3_workspace_bytes, 256-byte aligned, owned by the caller and unused by it until
 * lbm3_destroy.  hip_stream: the stream every launch goes to (NULL = default stream).
 * Writes the initial populations (equilibria of the initial fields, S = 0, grad T = 0)
 * and synchronizes the stream.  On error *out is NULL and nothing is left enqueued. */
lbm_status lbm3_init(const lbm3_params *params, void *workspace, size_t workspace_bytes,
                     void *hip_stream, lbm3_ctx **out);

/* Enqueues nsteps time steps (collide, stream, boundary scheme; per step one launch over
 * the interior nodes and, with walls, one over the wall nodes).  Asynchronous;
 * nsteps < 0 is LBM_ERR_INVALID. */
lbm_status lbm3_step(lbm3_ctx *ctx, int64_t nsteps);

/* Macroscopic fields at the current time into FP64 device arrays (any may be NULL):
 * p, u (3 planes), T, S = grad u + (grad u)^T (6 planes: xx, xy, xz, yy, yz, zz), grad T
 * (3 planes).  Asynchronous. */
lbm_status lbm3_fields(lbm3_ctx *ctx, double *p, double *u, double *T, double *S, double *gradT);

/* Pre-collision populations at the current time as FP64 device arrays [19][nz][ny][nx]
 * (f and g; the rest state added back), in the order of lbm3_lattice.  Asynchronous. */
lbm_status lbm3_populations(lbm3_ctx *ctx, double *f, double *g);

/* Average Nusselt number of wall 0 (z = 0), 1 (z = nz - 1), 2 (x = 0), 3 (x = nx - 1),
 * 4 (y = 0) or 5 (y = ny - 1) at the current time, as in two dimensions (Eq. AvNuss):
 * Nu = -L (dT/dn) / dT, n = +z, +x or +y along the wall's axis, with dT/dn from the
 * one-sided second-order difference into the fluid, averaged over the wall plane (a plain
 * mean along each periodic in-plane direction, the trapezoid rule along each walled one; a
 * heat flux along +n counts positive at both walls of a pair).  FP64 arithmetic in a fixed summation order.  Needs that wall to exist
 * (LBM_ERR_INVALID otherwise) and T_hot != T_cold.  *nu_host receives the value.
 * Synchronizes. */
lbm_status lbm3_nusselt(lbm3_ctx *ctx, int32_t wall, double *nu_host);

/* The library's D3Q19 velocities (c: 19 x 3 ints, host) in population order; returns 19. */
int32_t lbm3_lattice(int32_t *c);

/* Number of time steps taken. */
int64_t lbm3_time(const lbm3_ctx *ctx);

/* Releases the context (not the workspace).  Waits for the context's stream. */
void lbm3_destroy(lbm3_ctx *ctx);

#ifdef __cplusplus
}
#endif
