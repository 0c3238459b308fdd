/*
 * Oracle for the modified lattice-BGK model of convection heat transfer in porous
 * media at the REV scale (Wang, Mi & Guo, arXiv:1505.02976).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference against which the
 * GPU path is checked.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may build, load or call it; the product library never does.  It shares
 * no code, header, table or constant with the GPU path.
 *
 * Structure (deliberately unlike the GPU path): array-of-structures populations
 * [node][9], push streaming, and separate phases collide -> stream -> boundary scheme,
 * all in IEEE binary64 with no FMA contraction (-ffp-contract=off).  Each function
 * follows the paper's equations in the paper's notation; tensor contractions such as
 * uu:(c c - cs^2 I) are written out as double sums over the two Cartesian indices.
 *
 * Compiled twice: as real double, and with -DORC_COMPLEX as double complex so that a
 * complex-step perturbation of the porosity field yields exact directional derivatives
 * (sqrt is continued analytically; no modulus or comparison enters the time step).
 *
 * Readings of points the paper leaves open (also listed in the design notes):
 *   R1  pressure gauge: initial state has p = 0 (gauge pressure).
 *   R2  initial state: the post-collision populations at t = -1 are the equilibria of
 *       the initial fields (S = 0, grad T = 0); time 0 starts by streaming them and
 *       applying the boundary scheme.
 *   R3  r_0 is kept in f_0^eq with the full discrete S; the pressure formula has no r_0.
 *   R5  wall nodes: the boundary scheme rebuilds their pre-collision populations, and
 *       the node's macroscopic state is the one the scheme assigns: T_b, u_b, p(x_f),
 *       S(x_f), grad T_b (the force follows from u_b and T_b).  The node collides with
 *       the equilibrium of that state, which makes its post-collision populations
 *       f^eq(x_b) + (1 - 1/tau) f^neq(x_f) plus the source terms (the post-collision form
 *       of the non-equilibrium extrapolation); its reported fields are that state.
 *   R6  Neumann walls use p(x_f) in the boundary equilibrium.
 *   R7  Neumann walls: normal component of grad T prescribed, tangential from x_f.
 *   R8  corners: x_f is the inward diagonal neighbour, u_b = 0; an isothermal wall
 *       wins over an adiabatic one, and the x-wall wins over the y-wall.
 *   R9  wet-node walls; n nodes across a walled direction give L = n - 1.
 *   R10 the drag terms use the fluid viscosity nu = nu_e / J.
 *   R13 residual: sum of |phi(t)-phi(t-100)| over sum of |phi(t)|, L2 for u, L1 for T.
 *   R14 Nusselt number: second-order one-sided wall derivative, trapezoid rule.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>

#ifdef ORC_COMPLEX
#include <complex.h>
typedef double complex real;
#define R_SQRT(x) csqrt(x)
#define R_RE(x) creal(x)
#else
typedef double real;
#define R_SQRT(x) sqrt(x)
#define R_RE(x) (x)
#endif

/* ------------------------------------------------------------------------------ */
/* D2Q9 lattice (Sec. 3.1): c_0 = 0; c_i = (cos((i-1)pi/2), sin((i-1)pi/2)) for      */
/* i = 1..4; c_i = sqrt(2)(cos((i-5)pi/2 + pi/4), sin(...)) for i = 5..8;           */
/* weights 4/9, 1/9, 1/36; cs^2 = c^2/3 with c = dx/dt = 1.                          */
/* ------------------------------------------------------------------------------ */
static int CX[9], CY[9];
static double WGT[9];
static const double CS2 = 1.0 / 3.0;
static const double RHO0 = 1.0;
static int lattice_ready = 0;

static void build_lattice(void)
{
    if (lattice_ready) return;
    const double pi = 3.14159265358979323846;
    CX[0] = 0; CY[0] = 0; WGT[0] = 4.0 / 9.0;
    for (int i = 1; i <= 4; ++i) {
        double a = (i - 1) * pi / 2.0;
        CX[i] = (int)lround(cos(a));
        CY[i] = (int)lround(sin(a));
        WGT[i] = 1.0 / 9.0;
    }
    for (int i = 5; i <= 8; ++i) {
        double a = (i - 5) * pi / 2.0 + pi / 4.0;
        CX[i] = (int)lround(sqrt(2.0) * cos(a));
        CY[i] = (int)lround(sqrt(2.0) * sin(a));
        WGT[i] = 1.0 / 36.0;
    }
    lattice_ready = 1;
}

/* varpi_i = omega_i (i != 0), varpi_0 = -sum_{i != 0} varpi_i  (Eq. TeEDFEQ). */
static double varpi(int i)
{
    if (i != 0) return WGT[i];
    double s = 0.0;
    for (int k = 1; k < 9; ++k) s += WGT[k];
    return -s;
}

/* ------------------------------------------------------------------------------ */
/* Problem description                                                              */
/* ------------------------------------------------------------------------------ */
typedef struct {
    int32_t nx, ny, periodic_x, periodic_y;
    int32_t wall_kind[4];          /* 0 = isothermal (Dirichlet T), 1 = prescribed dT/dn */
    double wall_ux[4], wall_uy[4], wall_T[4], wall_dTdn[4];   /* order x-, x+, y-, y+ */
    double L;                      /* characteristic length; 0 => derived from the grid */
    double Da, Ra, Pr, J, Ma, sigma, Q;
    double tau_f, tau_T, A, B;     /* A, B: NaN => from Ma, Ra, Pr (Eq. EQA&B) */
    double eps;                    /* uniform porosity when no field is given */
    double ax, ay;                 /* external acceleration a */
    double T_hot, T_cold;
    double F_eps;                  /* NaN => Ergun relation */
} orc_params;

typedef struct {
    double L, A, B, nu_e, nu, alpha_e, gbeta, K, T0, dT;
    int ergun;
} orc_derived;

typedef struct {
    orc_params prm;
    orc_derived d;
    int n;
    real *eps;            /* porosity per node */
    real *f, *g;          /* pre-collision populations, [node][9] */
    real *fs, *gs;        /* post-collision populations, [node][9] */
    double *u_prev, *T_prev;   /* residual snapshot: ux, uy per node; T per node */
    int have_prev;
    int64_t t;
    struct orc_macro_s *mb;   /* per node: the boundary state of wall nodes (R5) */
} orc_sim;

typedef struct orc_macro_s {
    real eps, T, Gx, Gy, vx, vy, ux, uy, Fx, Fy, p;
    real Sxx, Sxy, Syy, dTx, dTy;
} orc_macro;

/* Parameter mapping: Sec. 2 (groups), Sec. 3.1 (nu_e), Eq. Therdiff (alpha_e),       */
/* Eq. EQA&B (A, B from Ma), Ra definition (g beta), Da definition (K).              */
static int derive(const orc_params *p, orc_derived *d)
{
    if (p->L > 0) d->L = p->L;
    else if (!p->periodic_x) d->L = p->nx - 1;
    else if (!p->periodic_y) d->L = p->ny - 1;
    else d->L = p->nx;
    d->T0 = 0.5 * (p->T_hot + p->T_cold);
    d->dT = p->T_hot - p->T_cold;
    if (isnan(p->A) || isnan(p->B)) {
        if (!(p->Ra > 0) || !(p->Pr > 0)) return -1;
        d->A = p->tau_f - 0.5 - p->J * p->Ma * d->L * sqrt(3.0 * p->Pr / p->Ra);
        d->B = p->tau_T - 0.5 - (p->Ma / p->sigma) * d->L * sqrt(3.0 / (p->Pr * p->Ra));
    } else {
        d->A = p->A;
        d->B = p->B;
    }
    d->nu_e = CS2 * (p->tau_f - d->A - 0.5);
    d->nu = d->nu_e / p->J;
    d->alpha_e = p->sigma * CS2 * (p->tau_T - d->B - 0.5);
    /* Ra = g beta dT L^3 / (nu alpha_e) */
    if (p->Ra > 0 && d->dT != 0.0)
        d->gbeta = p->Ra * d->nu * d->alpha_e / (d->dT * d->L * d->L * d->L);
    else
        d->gbeta = 0.0;
    d->K = p->Da * d->L * d->L;
    d->ergun = isnan(p->F_eps) ? 1 : 0;
    if (!(d->nu_e > 0) || !(d->alpha_e > 0) || !(d->K > 0)) return -2;
    return 0;
}

/* ------------------------------------------------------------------------------ */
/* Local computations at one node from its pre-collision populations              */
/* ------------------------------------------------------------------------------ */

/* f_i^{e(0)}: the flow EDF without the shear-rate term (Eq. EQFINApp). */
static void feq0(const orc_sim *s, real eps, real p, real ux, real uy, real out[9])
{
    (void)s;
    real u[2] = {ux, uy};
    for (int i = 0; i < 9; ++i) {
        double c[2] = {CX[i], CY[i]};
        real cu = c[0] * u[0] + c[1] * u[1];
        real uucc = 0.0;                     /* uu:(c c - cs^2 I) */
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                uucc += u[a] * u[b] * (c[a] * c[b] - CS2 * (a == b ? 1.0 : 0.0));
        real si = WGT[i] * (cu / CS2 + uucc / (2.0 * eps * CS2 * CS2));
        if (i == 0)
            out[i] = RHO0 - (1.0 - WGT[0]) * eps * p / CS2 + RHO0 * si;
        else
            out[i] = WGT[i] * eps * p / CS2 + RHO0 * si;
    }
}

/* r_i: the shear-rate term of the flow EDF (Eq. EQTSHIN), dt = 1. */
static void req(const orc_sim *s, real Sxx, real Sxy, real Syy, real out[9])
{
    real S[2][2] = {{Sxx, Sxy}, {Sxy, Syy}};
    for (int i = 0; i < 9; ++i) {
        double c[2] = {CX[i], CY[i]};
        real Scc = 0.0;                      /* S:(c c - cs^2 I) */
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                Scc += S[a][b] * (c[a] * c[b] - CS2 * (a == b ? 1.0 : 0.0));
        out[i] = WGT[i] * s->d.A * Scc / (2.0 * CS2);
    }
}

/* Full flow EDF f_i^{(eq)} = f_i^{e(0)} + rho0 r_i (Eq. EQFIN). */
static void feq_full(const orc_sim *s, real eps, real p, real ux, real uy,
                     real Sxx, real Sxy, real Syy, real out[9])
{
    real e0[9], r[9];
    feq0(s, eps, p, ux, uy, e0);
    req(s, Sxx, Sxy, Syy, r);
    for (int i = 0; i < 9; ++i) out[i] = e0[i] + RHO0 * r[i];
}

/* g_i^{e(0)}: the temperature EDF without the gradient term (Eq. TeEDFEQ). */
static void geq0(const orc_sim *s, real eps, real T, real ux, real uy, real p, real out[9])
{
    const double sigma = s->prm.sigma;
    real u[2] = {ux, uy};
    for (int i = 0; i < 9; ++i) {
        double c[2] = {CX[i], CY[i]};
        real cu = c[0] * u[0] + c[1] * u[1];
        real uucc = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                uucc += u[a] * u[b] * (c[a] * c[b] - CS2 * (a == b ? 1.0 : 0.0));
        out[i] = WGT[i] * T * (sigma + cu / CS2 + uucc / (2.0 * eps * CS2 * CS2))
               + varpi(i) * T * eps * p / (CS2 * RHO0);
    }
}

/* Full temperature EDF: g^{e(0)} + sigma omega_i B c_i . grad T (Eq. TeEDFEQ). */
static void geq_full(const orc_sim *s, real eps, real T, real ux, real uy, real p,
                     real dTx, real dTy, real out[9])
{
    geq0(s, eps, T, ux, uy, p, out);
    for (int i = 0; i < 9; ++i)
        out[i] += s->prm.sigma * WGT[i] * s->d.B * (CX[i] * dTx + CY[i] * dTy);
}

/* Porous-medium coefficients at porosity eps: F_eps (Ergun or given), c0, c1. */
static void porous_coeffs(const orc_sim *s, real eps, real *Feps, real *c0, real *c1)
{
    const double K = s->d.K, nu = s->d.nu;
    if (s->d.ergun) *Feps = 1.75 / R_SQRT(150.0 * eps * eps * eps);
    else *Feps = s->prm.F_eps;
    *c0 = 0.5 * (1.0 + eps * 0.5 * nu / K);
    *c1 = eps * 0.5 * (*Feps) / sqrt(K);
}

/* Macroscopic quantities at a node from pre-collision f_i, g_i, in the paper's order:
 * T (Sec. 3.2), G (Sec. 2), v and u (Sec. 3.1), F (Eq. ForceEq), p (Sec. 3.1 with the
 * closed forms of s_0 and F_0 from App. A), S (Eq. ShearEqCom), grad T (Eqs. MatrM,
 * MatrN solved as a 2x2 linear system, Eq. TeEqCom). */
static void node_macro(const orc_sim *s, real eps, const real *f, const real *g, orc_macro *m)
{
    const orc_params *P = &s->prm;
    const orc_derived *D = &s->d;
    const double sigma = P->sigma, Q = P->Q, tf = P->tau_f, tT = P->tau_T;
    m->eps = eps;

    real sg = 0.0;
    for (int i = 0; i < 9; ++i) sg += g[i];
    m->T = (sg + 0.5 * Q) / sigma;

    m->Gx = P->ax;
    m->Gy = P->ay + D->gbeta * (m->T - D->T0);

    real jx = 0.0, jy = 0.0;
    for (int i = 0; i < 9; ++i) { jx += CX[i] * f[i]; jy += CY[i] * f[i]; }
    m->vx = jx / RHO0 + 0.5 * eps * m->Gx;
    m->vy = jy / RHO0 + 0.5 * eps * m->Gy;

    real Feps, c0, c1;
    porous_coeffs(s, eps, &Feps, &c0, &c1);
    real vmag = R_SQRT(m->vx * m->vx + m->vy * m->vy);
    real den = c0 + R_SQRT(c0 * c0 + c1 * vmag);
    m->ux = m->vx / den;
    m->uy = m->vy / den;

    real umag = R_SQRT(m->ux * m->ux + m->uy * m->uy);
    m->Fx = -eps * D->nu / D->K * m->ux - eps * Feps / sqrt(D->K) * umag * m->ux + eps * m->Gx;
    m->Fy = -eps * D->nu / D->K * m->uy - eps * Feps / sqrt(D->K) * umag * m->uy + eps * m->Gy;

    real uF = m->ux * m->Fx + m->uy * m->Fy;
    real s0 = -WGT[0] / (2.0 * eps * CS2) * (m->ux * m->ux + m->uy * m->uy);
    real F0 = -WGT[0] * (1.0 - 1.0 / (2.0 * tf)) * uF / (eps * CS2);
    real sumf = 0.0;
    for (int i = 1; i < 9; ++i) sumf += f[i];
    m->p = CS2 / (eps * (1.0 - WGT[0])) * (sumf + tf * F0 + RHO0 * s0);

    /* shear rate */
    real e0[9];
    feq0(s, eps, m->p, m->ux, m->uy, e0);
    real Pi[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int i = 0; i < 9; ++i) {
        double c[2] = {CX[i], CY[i]};
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                Pi[a][b] += c[a] * c[b] * (f[i] - e0[i]);
    }
    real u[2] = {m->ux, m->uy}, F[2] = {m->Fx, m->Fy};
    real Sm[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            Sm[a][b] = (Pi[a][b] + 0.5 * RHO0 * (u[a] * F[b] / eps + F[a] * u[b] / eps))
                     / (CS2 * RHO0 * (D->A - tf));
    m->Sxx = Sm[0][0];
    m->Sxy = 0.5 * (Sm[0][1] + Sm[1][0]);
    m->Syy = Sm[1][1];

    /* temperature gradient: <M> grad T = <N> */
    real ge0[9];
    geq0(s, eps, m->T, m->ux, m->uy, m->p, ge0);
    real N[2] = {0.0, 0.0};
    for (int i = 0; i < 9; ++i) {
        N[0] += CX[i] * (g[i] - ge0[i]);
        N[1] += CY[i] * (g[i] - ge0[i]);
    }
    for (int a = 0; a < 2; ++a) N[a] += 0.5 * (m->T * F[a] + u[a] / sigma * Q);
    real M[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            M[a][b] = -eps * m->p / (2.0 * RHO0) * (a == b ? 1.0 : 0.0)
                    - 0.5 * (1.0 / eps - 1.0 / sigma) * u[a] * u[b]
                    + CS2 * sigma * (D->B - tT) * (a == b ? 1.0 : 0.0);
    real det = M[0][0] * M[1][1] - M[0][1] * M[1][0];
    m->dTx = (N[0] * M[1][1] - M[0][1] * N[1]) / det;
    m->dTy = (M[0][0] * N[1] - N[0] * M[1][0]) / det;
}

/* Discrete forcing F_i (Eq. FtermF), dt = 1. */
static void force_terms(const orc_sim *s, const orc_macro *m, real out[9])
{
    const double tf = s->prm.tau_f;
    real u[2] = {m->ux, m->uy}, F[2] = {m->Fx, m->Fy};
    for (int i = 0; i < 9; ++i) {
        double c[2] = {CX[i], CY[i]};
        real cF = c[0] * F[0] + c[1] * F[1];
        real t2 = 0.0;                       /* (uF + Fu):(c c - cs^2 I) */
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                t2 += (u[a] * F[b] + F[a] * u[b]) * (c[a] * c[b] - CS2 * (a == b ? 1.0 : 0.0));
        out[i] = WGT[i] * RHO0 * (1.0 - 1.0 / (2.0 * tf))
               * (cF / CS2 + t2 / (2.0 * m->eps * CS2 * CS2));
    }
}

/* Thermal source terms P_i and Q_i (Eq. Eq:Tforce), dt = 1. */
static void thermal_sources(const orc_sim *s, const orc_macro *m, real Pout[9], real Qout[9])
{
    const double tT = s->prm.tau_T, sigma = s->prm.sigma, Q = s->prm.Q;
    real u[2] = {m->ux, m->uy}, gT[2] = {m->dTx, m->dTy}, F[2] = {m->Fx, m->Fy};
    for (int i = 0; i < 9; ++i) {
        double c[2] = {CX[i], CY[i]};
        real vec[2];
        for (int a = 0; a < 2; ++a) vec[a] = m->T * F[a] + m->eps * m->p * gT[a] / RHO0;
        real cvec = c[0] * vec[0] + c[1] * vec[1];
        real uucg = 0.0;                     /* uu:(c grad T) */
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                uucg += u[a] * u[b] * c[a] * gT[b];
        Pout[i] = WGT[i] * (1.0 - 1.0 / (2.0 * tT))
                * (cvec / CS2 + (1.0 / m->eps - 1.0 / sigma) * uucg / CS2);
        real cu = c[0] * u[0] + c[1] * u[1];
        Qout[i] = WGT[i] * (1.0 - 1.0 / (2.0 * tT)) * (1.0 + cu / (sigma * CS2)) * Q;
    }
}

/* Collision of populations f, g with the equilibria and sources of the macroscopic
 * state m (Eqs. LBEeq and TEqColli). */
static void collide_state(const orc_sim *s, const orc_macro *mm, const real *f, const real *g,
                          real *fo, real *go)
{
    const orc_macro m = *mm;
    real fe[9], ge[9], Fi[9], Pi[9], Qi[9];
    feq_full(s, m.eps, m.p, m.ux, m.uy, m.Sxx, m.Sxy, m.Syy, fe);
    geq_full(s, m.eps, m.T, m.ux, m.uy, m.p, m.dTx, m.dTy, ge);
    force_terms(s, &m, Fi);
    thermal_sources(s, &m, Pi, Qi);
    const double tf = s->prm.tau_f, tT = s->prm.tau_T;
    for (int i = 0; i < 9; ++i) {
        fo[i] = f[i] - (f[i] - fe[i]) / tf + Fi[i];
        go[i] = g[i] - (g[i] - ge[i]) / tT + Pi[i] + Qi[i];
    }
}

/* Collision at an interior node: its state from its own populations. */
static void collide_node(const orc_sim *s, real eps, const real *f, const real *g,
                         real *fo, real *go)
{
    orc_macro m;
    node_macro(s, eps, f, g, &m);
    collide_state(s, &m, f, g, fo, go);
}

/* ------------------------------------------------------------------------------ */
/* Grid phases                                                                      */
/* ------------------------------------------------------------------------------ */
static int node_index(const orc_sim *s, int x, int y) { return y * s->prm.nx + x; }

/* Which walls a node lies on: xw in {-1 none, 0 (x-), 1 (x+)}, yw in {-1, 2, 3}. */
static void wall_of(const orc_sim *s, int x, int y, int *xw, int *yw)
{
    const orc_params *P = &s->prm;
    *xw = -1; *yw = -1;
    if (!P->periodic_x) { if (x == 0) *xw = 0; else if (x == P->nx - 1) *xw = 1; }
    if (!P->periodic_y) { if (y == 0) *yw = 2; else if (y == P->ny - 1) *yw = 3; }
}

static int is_wall_node(const orc_sim *s, int k)
{
    int xw, yw;
    wall_of(s, k % s->prm.nx, k / s->prm.nx, &xw, &yw);
    return xw >= 0 || yw >= 0;
}

/* Macroscopic state of node k at the current time: R5 for wall nodes. */
static void state_of(const orc_sim *s, int k, orc_macro *m)
{
    if (is_wall_node(s, k)) *m = s->mb[k];
    else node_macro(s, s->eps[k], s->f + 9 * k, s->g + 9 * k, m);
}

static void collide_all(orc_sim *s)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < s->n; ++k) {
        if (is_wall_node(s, k))
            collide_state(s, &s->mb[k], s->f + 9 * k, s->g + 9 * k, s->fs + 9 * k, s->gs + 9 * k);
        else
            collide_node(s, s->eps[k], s->f + 9 * k, s->g + 9 * k, s->fs + 9 * k, s->gs + 9 * k);
    }
}

/* Streaming (push): f_i(x + c_i, t + 1) = f*_i(x, t); periodic directions wrap,
 * populations leaving through a wall are dropped. */
static void stream_all(orc_sim *s)
{
    const int nx = s->prm.nx, ny = s->prm.ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int k = node_index(s, x, y);
            for (int i = 0; i < 9; ++i) {
                int xd = x + CX[i], yd = y + CY[i];
                if (s->prm.periodic_x) xd = (xd + nx) % nx;
                if (s->prm.periodic_y) yd = (yd + ny) % ny;
                if (xd < 0 || xd >= nx || yd < 0 || yd >= ny) continue;
                int kd = node_index(s, xd, yd);
                s->f[9 * kd + i] = s->fs[9 * k + i];
                s->g[9 * kd + i] = s->gs[9 * k + i];
            }
        }
}

/* Non-equilibrium extrapolation at one wall node (Sec. 3.4). */
static void nees_node(orc_sim *s, int x, int y, int xw, int yw)
{
    const orc_params *P = &s->prm;
    int dx = (xw == 0) ? 1 : (xw == 1) ? -1 : 0;
    int dy = (yw == 2) ? 1 : (yw == 3) ? -1 : 0;
    int kb = node_index(s, x, y);
    int kf = node_index(s, x + dx, y + dy);
    real *ff = s->f + 9 * kf, *gf = s->g + 9 * kf;

    orc_macro mf;
    node_macro(s, s->eps[kf], ff, gf, &mf);
    real fe_f[9], ge_f[9];
    feq_full(s, mf.eps, mf.p, mf.ux, mf.uy, mf.Sxx, mf.Sxy, mf.Syy, fe_f);
    geq_full(s, mf.eps, mf.T, mf.ux, mf.uy, mf.p, mf.dTx, mf.dTy, ge_f);

    /* wall velocity: a corner is at rest */
    real ubx = 0.0, uby = 0.0;
    if (xw >= 0 && yw < 0) { ubx = P->wall_ux[xw]; uby = P->wall_uy[xw]; }
    if (yw >= 0 && xw < 0) { ubx = P->wall_ux[yw]; uby = P->wall_uy[yw]; }

    real eb = s->eps[kb];
    real fe_b[9];
    feq_full(s, eb, mf.p, ubx, uby, mf.Sxx, mf.Sxy, mf.Syy, fe_b);
    for (int i = 0; i < 9; ++i) s->f[9 * kb + i] = fe_b[i] + (ff[i] - fe_f[i]);

    /* thermal condition */
    int dir = -1;
    if (xw >= 0 && P->wall_kind[xw] == 0) dir = xw;
    else if (yw >= 0 && P->wall_kind[yw] == 0) dir = yw;
    real Tb, gbx, gby;
    if (dir >= 0) {
        Tb = P->wall_T[dir];
        gbx = mf.dTx;
        gby = mf.dTy;
    } else {
        /* prescribed normal derivative: component along a walled axis is
         * (inward sign) * dT/dn; the other component comes from x_f */
        gbx = (xw >= 0) ? dx * P->wall_dTdn[xw] : mf.dTx;
        gby = (yw >= 0) ? dy * P->wall_dTdn[yw] : mf.dTy;
        int kff = node_index(s, x + 2 * dx, y + 2 * dy);
        real sgff = 0.0;
        for (int i = 0; i < 9; ++i) sgff += s->g[9 * kff + i];
        real Tff = (sgff + 0.5 * P->Q) / P->sigma;
        Tb = (4.0 * mf.T - Tff - 2.0 * (dx * gbx + dy * gby)) / 3.0;
    }
    real ge_b[9];
    geq_full(s, eb, Tb, ubx, uby, mf.p, gbx, gby, ge_b);
    for (int i = 0; i < 9; ++i) s->g[9 * kb + i] = ge_b[i] + (gf[i] - ge_f[i]);

    /* the node's state (R5): the boundary values, with G and F (Eq. ForceEq) at u_b, T_b */
    const orc_derived *D = &s->d;
    orc_macro *m = &s->mb[kb];
    real Feps, c0, c1;
    porous_coeffs(s, eb, &Feps, &c0, &c1);
    m->eps = eb;
    m->T = Tb;
    m->Gx = P->ax;
    m->Gy = P->ay + D->gbeta * (Tb - D->T0);
    m->vx = ubx; m->vy = uby;
    m->ux = ubx; m->uy = uby;
    real umag = R_SQRT(ubx * ubx + uby * uby);
    m->Fx = -eb * D->nu / D->K * ubx - eb * Feps / sqrt(D->K) * umag * ubx + eb * m->Gx;
    m->Fy = -eb * D->nu / D->K * uby - eb * Feps / sqrt(D->K) * umag * uby + eb * m->Gy;
    m->p = mf.p;
    m->Sxx = mf.Sxx; m->Sxy = mf.Sxy; m->Syy = mf.Syy;
    m->dTx = gbx; m->dTy = gby;
}

static void boundary_all(orc_sim *s)
{
    const int nx = s->prm.nx, ny = s->prm.ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int xw, yw;
            wall_of(s, x, y, &xw, &yw);
            if (xw >= 0 || yw >= 0) nees_node(s, x, y, xw, yw);
        }
}

/* ------------------------------------------------------------------------------ */
/* Exported interface (ctypes)                                                     */
/* ------------------------------------------------------------------------------ */
int orc_lattice(int32_t *cx, int32_t *cy, double *w)
{
    build_lattice();
    for (int i = 0; i < 9; ++i) { cx[i] = CX[i]; cy[i] = CY[i]; w[i] = WGT[i]; }
    return 0;
}

int orc_derive(const orc_params *p, double *out /* 10 */)
{
    orc_derived d;
    int rc = derive(p, &d);
    out[0] = d.L; out[1] = d.A; out[2] = d.B; out[3] = d.nu_e; out[4] = d.nu;
    out[5] = d.alpha_e; out[6] = d.gbeta; out[7] = d.K; out[8] = d.T0; out[9] = d.dT;
    return rc;
}

/* Initial fields (R1, R2): optional p, ux, uy, T per node; NULL means p = 0, u = 0,
 * T = T0 in the interior and T_wall on isothermal wall nodes. */
orc_sim *orc_create(const orc_params *p, const real *eps_field, const real *T_init,
                    const real *p_init, const real *ux_init, const real *uy_init)
{
    build_lattice();
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    s->prm = *p;
    if (derive(p, &s->d) != 0) { free(s); return NULL; }
    s->n = p->nx * p->ny;
    s->eps = (real *)malloc(sizeof(real) * s->n);
    s->f = (real *)malloc(sizeof(real) * 9 * s->n);
    s->g = (real *)malloc(sizeof(real) * 9 * s->n);
    s->fs = (real *)malloc(sizeof(real) * 9 * s->n);
    s->gs = (real *)malloc(sizeof(real) * 9 * s->n);
    s->u_prev = (double *)calloc(2 * (size_t)s->n, sizeof(double));
    s->T_prev = (double *)calloc((size_t)s->n, sizeof(double));
    s->mb = (orc_macro *)calloc((size_t)s->n, sizeof(orc_macro));
    for (int k = 0; k < s->n; ++k) s->eps[k] = eps_field ? eps_field[k] : (real)p->eps;
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            int k = node_index(s, x, y);
            real T = s->d.T0;
            if (T_init) T = T_init[k];
            else {
                int xw, yw;
                wall_of(s, x, y, &xw, &yw);
                if (xw >= 0 && p->wall_kind[xw] == 0) T = p->wall_T[xw];
                else if (yw >= 0 && p->wall_kind[yw] == 0) T = p->wall_T[yw];
            }
            real pp = p_init ? p_init[k] : 0.0;
            real ux = ux_init ? ux_init[k] : 0.0;
            real uy = uy_init ? uy_init[k] : 0.0;
            feq_full(s, s->eps[k], pp, ux, uy, 0.0, 0.0, 0.0, s->fs + 9 * k);
            geq_full(s, s->eps[k], T, ux, uy, pp, 0.0, 0.0, s->gs + 9 * k);
        }
    memcpy(s->f, s->fs, sizeof(real) * 9 * s->n);
    memcpy(s->g, s->gs, sizeof(real) * 9 * s->n);
    stream_all(s);
    boundary_all(s);
    s->t = 0;
    return s;
}

void orc_destroy(orc_sim *s)
{
    if (!s) return;
    free(s->eps); free(s->f); free(s->g); free(s->fs); free(s->gs);
    free(s->u_prev); free(s->T_prev); free(s->mb);
    free(s);
}

/* One time step: collide -> stream -> boundary scheme. */
void orc_step(orc_sim *s, int64_t nsteps)
{
    for (int64_t k = 0; k < nsteps; ++k) {
        collide_all(s);
        stream_all(s);
        boundary_all(s);
        s->t += 1;
    }
}

int64_t orc_time(const orc_sim *s) { return s->t; }

/* Macroscopic fields at the current time (wall nodes: their boundary state, R5); any
 * output may be NULL. */
void orc_macro_fields(const orc_sim *s, real *p, real *ux, real *uy, real *T,
                      real *Sxx, real *Sxy, real *Syy, real *dTx, real *dTy)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < s->n; ++k) {
        orc_macro m;
        state_of(s, k, &m);
        if (p) p[k] = m.p;
        if (ux) ux[k] = m.ux;
        if (uy) uy[k] = m.uy;
        if (T) T[k] = m.T;
        if (Sxx) Sxx[k] = m.Sxx;
        if (Sxy) Sxy[k] = m.Sxy;
        if (Syy) Syy[k] = m.Syy;
        if (dTx) dTx[k] = m.dTx;
        if (dTy) dTy[k] = m.dTy;
    }
}

/* Populations in structure-of-arrays order [9][ny][nx]. which: 0 = pre-collision at
 * the current time, 1 = post-collision of the previous step. */
void orc_get_populations(const orc_sim *s, int which, real *f_out, real *g_out)
{
    const real *f = which ? s->fs : s->f;
    const real *g = which ? s->gs : s->g;
    for (int i = 0; i < 9; ++i)
        for (int k = 0; k < s->n; ++k) {
            f_out[(size_t)i * s->n + k] = f[9 * k + i];
            g_out[(size_t)i * s->n + k] = g[9 * k + i];
        }
}

/* Replace the post-collision populations of the previous step ([9][ny][nx] order)
 * and re-derive the current pre-collision state by streaming and the boundary scheme. */
void orc_set_post_populations(orc_sim *s, const real *f_in, const real *g_in)
{
    for (int i = 0; i < 9; ++i)
        for (int k = 0; k < s->n; ++k) {
            s->fs[9 * k + i] = f_in[(size_t)i * s->n + k];
            s->gs[9 * k + i] = g_in[(size_t)i * s->n + k];
        }
    memcpy(s->f, s->fs, sizeof(real) * 9 * s->n);
    memcpy(s->g, s->gs, sizeof(real) * 9 * s->n);
    stream_all(s);
    boundary_all(s);
}

/* Average Nusselt number on a wall (Eq. Eq:AvNuss with R14):
 * Nu_j = -L (dT/dn_axis)_wall / dT, the derivative along the wall-normal axis by the
 * one-sided second-order difference, averaged over the wall by the trapezoid rule. */
void orc_nusselt(const orc_sim *s, int wall, real *out)
{
    const int nx = s->prm.nx, ny = s->prm.ny;
    real *T = (real *)malloc(sizeof(real) * s->n);
    orc_macro_fields(s, NULL, NULL, NULL, T, NULL, NULL, NULL, NULL, NULL);
    int along = (wall < 2) ? ny : nx;
    real acc = 0.0;
    for (int j = 0; j < along; ++j) {
        real T0v, T1v, T2v, sgn;
        if (wall == 0) { T0v = T[node_index(s, 0, j)]; T1v = T[node_index(s, 1, j)]; T2v = T[node_index(s, 2, j)]; sgn = 1.0; }
        else if (wall == 1) { T0v = T[node_index(s, nx - 1, j)]; T1v = T[node_index(s, nx - 2, j)]; T2v = T[node_index(s, nx - 3, j)]; sgn = -1.0; }
        else if (wall == 2) { T0v = T[node_index(s, j, 0)]; T1v = T[node_index(s, j, 1)]; T2v = T[node_index(s, j, 2)]; sgn = 1.0; }
        else { T0v = T[node_index(s, j, ny - 1)]; T1v = T[node_index(s, j, ny - 2)]; T2v = T[node_index(s, j, ny - 3)]; sgn = -1.0; }
        real dTdaxis = sgn * (-3.0 * T0v + 4.0 * T1v - T2v) / 2.0;
        real Nu = -s->d.L * dTdaxis / s->d.dT;
        real wtr = (j == 0 || j == along - 1) ? 0.5 : 1.0;
        acc += wtr * Nu;
    }
    free(T);
    *out = acc / (along - 1);
}

/* Convergence measure (Sec. 4, R13) against the snapshot taken at the previous call;
 * the first call only takes the snapshot and returns -1. */
int orc_residual(orc_sim *s, double *r_u, double *r_T)
{
    double num_u = 0, den_u = 0, num_T = 0, den_T = 0;
    int first = !s->have_prev;
    for (int k = 0; k < s->n; ++k) {
        orc_macro m;
        state_of(s, k, &m);
        double ux = R_RE(m.ux), uy = R_RE(m.uy), T = R_RE(m.T);
        double dux = ux - s->u_prev[2 * k], duy = uy - s->u_prev[2 * k + 1];
        num_u += sqrt(dux * dux + duy * duy);
        den_u += sqrt(ux * ux + uy * uy);
        num_T += fabs(T - s->T_prev[k]);
        den_T += fabs(T);
        s->u_prev[2 * k] = ux; s->u_prev[2 * k + 1] = uy; s->T_prev[k] = T;
    }
    s->have_prev = 1;
    if (first) { *r_u = -1; *r_T = -1; return 1; }
    *r_u = num_u / den_u;
    *r_T = num_T / den_T;
    return 0;
}

/* Single-node building blocks, exposed for the identity tests. */
void orc_node_macro(const orc_params *p, double eps_d, const real *f, const real *g, real *out /* 16 */)
{
    build_lattice();
    orc_sim s;
    memset(&s, 0, sizeof(s));
    s.prm = *p;
    derive(p, &s.d);
    orc_macro m;
    node_macro(&s, (real)eps_d, f, g, &m);
    real v[16] = {m.T, m.Gx, m.Gy, m.vx, m.vy, m.ux, m.uy, m.Fx, m.Fy, m.p,
                  m.Sxx, m.Sxy, m.Syy, m.dTx, m.dTy, m.eps};
    for (int i = 0; i < 16; ++i) out[i] = v[i];
}

/* All discrete terms at one node for given macroscopic values:
 * out rows: feq0, r_i (without rho0), geq0, B-term of geq, F_i, P_i, Q_i  (7 x 9). */
void orc_node_terms(const orc_params *p, double eps, double T, double ux, double uy, double pr,
                    double Sxx, double Sxy, double Syy, double dTx, double dTy,
                    double Fx, double Fy, real *out)
{
    build_lattice();
    orc_sim s;
    memset(&s, 0, sizeof(s));
    s.prm = *p;
    derive(p, &s.d);
    real tmp[9];
    feq0(&s, eps, pr, ux, uy, out + 0);
    req(&s, Sxx, Sxy, Syy, out + 9);
    geq0(&s, eps, T, ux, uy, pr, out + 18);
    geq_full(&s, eps, T, ux, uy, pr, dTx, dTy, tmp);
    for (int i = 0; i < 9; ++i) out[27 + i] = tmp[i] - out[18 + i];
    orc_macro m;
    memset(&m, 0, sizeof(m));
    m.eps = eps; m.T = T; m.ux = ux; m.uy = uy; m.p = pr; m.Fx = Fx; m.Fy = Fy;
    m.dTx = dTx; m.dTy = dTy;
    force_terms(&s, &m, out + 36);
    thermal_sources(&s, &m, out + 45, out + 54);
}

/* Collision of a single node (pre -> post), exposed for tests. */
void orc_node_collide(const orc_params *p, double eps, const real *f, const real *g,
                      real *fo, real *go)
{
    build_lattice();
    orc_sim s;
    memset(&s, 0, sizeof(s));
    s.prm = *p;
    derive(p, &s.d);
    collide_node(&s, eps, f, g, fo, go);
}
