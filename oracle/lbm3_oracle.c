/*
 * Oracle for the three-dimensional form of the modified lattice-BGK model of convection
 * heat transfer in porous media (Wang, Mi & Guo, arXiv:1505.02976).  Secs. 2-3 write the
 * model for any lattice (equilibria, forcing and sources as tensor expressions in c_i, u,
 * S and grad T; Sec. 3.1 notes the extension to three dimensions); this file takes them on
 * the D3Q19 lattice.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference against which the
 * GPU path is checked.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may build, load or call it; the product library never does.  It shares
 * no code, header, table or constant with the GPU path.
 *
 * Structure: array-of-structures populations [node][19], push streaming, separate phases
 * collide -> stream -> boundary scheme, IEEE binary64 with no FMA contraction.  Tensor
 * contractions are written out as sums over the three Cartesian indices; the temperature
 * gradient solves its 3 x 3 system <M> grad T = <N> (Eqs. MatrM, MatrN) by Cramer's rule.
 *
 * Geometry: each of x, y, z periodic, or walls at 0 and n - 1 treated by the
 * non-equilibrium extrapolation of Sec. 3.4 with x_f the next node inward (on an edge or a
 * vertex where two or three walls meet, the inward diagonal neighbour, with the rules of
 * the 2-D corners, R8: at rest, an isothermal wall's temperature first, in the order x, y,
 * z, and each prescribed gradient setting its own normal component of grad T).
 *
 * Readings (the 2-D readings R1-R3, R5-R7, R9, R10, R12-R14 carry over unchanged):
 *   R21 lattice: D3Q19 for the flow and the temperature populations (the temperature
 *       equilibrium's u u term needs isotropic fourth moments, which D3Q7 lacks);
 *       weights 1/3 (rest), 1/18 (axes), 1/36 (edges), cs^2 = 1/3.  The pressure formula
 *       of Sec. 3.1 and the closed forms of s_0 and F_0 (App. A) take omega_0 = 1/3.
 *   R22 buoyancy G = g beta (T - T0) along +z; L given, else nx - 1 with walls in x, else
 *       nz - 1 with walls in z, else nz.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q19 19

static int C3[Q19][3];
static double W3[Q19];
static const double CS2 = 1.0 / 3.0;
static const double RHO0 = 1.0;
static int lattice_ready = 0;

/* D3Q19: rest, the six axis directions, the twelve edge directions (R21). */
static void build_lattice(void)
{
    if (lattice_ready) return;
    int k = 0;
    C3[k][0] = C3[k][1] = C3[k][2] = 0;
    W3[k++] = 1.0 / 3.0;
    for (int a = 0; a < 3; ++a)
        for (int s = -1; s <= 1; s += 2) {
            C3[k][0] = C3[k][1] = C3[k][2] = 0;
            C3[k][a] = s;
            W3[k++] = 1.0 / 18.0;
        }
    for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b)
            for (int sa = -1; sa <= 1; sa += 2)
                for (int sb = -1; sb <= 1; sb += 2) {
                    C3[k][0] = C3[k][1] = C3[k][2] = 0;
                    C3[k][a] = sa;
                    C3[k][b] = sb;
                    W3[k++] = 1.0 / 36.0;
                }
    lattice_ready = 1;
}

/* varpi_i = omega_i (i != 0), varpi_0 = -sum_{i != 0} omega_i  (Eq. TeEDFEQ). */
static double varpi(int i) { return i == 0 ? -(1.0 - W3[0]) : W3[i]; }

typedef struct {
    int32_t nx, ny, nz, periodic_x, periodic_y, periodic_z;
    int32_t wall_kind[6];          /* z = 0, z = nz - 1, x = 0, x = nx - 1, y = 0, y = ny - 1:
                                      0 isothermal, 1 prescribed dT/dn */
    double wall_u[6][3];           /* wall velocity */
    double wall_T[6], wall_dTdn[6];/* dTdn: derivative along the inward normal */
    double L;                      /* characteristic length; 0 => nz - 1 */
    double Da, Ra, Pr, J, Ma, sigma, Q;
    double tau_f, tau_T, A, B;     /* A, B: NaN => from Ma, Ra, Pr (Eq. EQA&B) */
    double eps;                    /* porosity when no field is given */
    double a[3];                   /* external acceleration */
    double T_hot, T_cold;
    double F_eps;                  /* NaN => Ergun relation */
} o3_params;

typedef struct {
    double L, A, B, nu_e, nu, alpha_e, gbeta, K, T0, dT;
    int ergun;
} o3_derived;

typedef struct {
    double eps, T, G[3], u[3], F[3], p;
    double S[3][3], dT[3];
} o3_macro;

typedef struct {
    o3_params prm;
    o3_derived d;
    int n;
    double *eps;                   /* porosity per node */
    double *f, *g, *fs, *gs;       /* pre- and post-collision populations, [node][19] */
    o3_macro *mb;                  /* per node: the boundary state of wall nodes (R5) */
    int64_t t;
} o3_sim;

/* Parameter mapping as in two dimensions (Sec. 2, Sec. 3.1, Eq. Therdiff, Eq. EQA&B). */
static int derive(const o3_params *p, o3_derived *d)
{
    d->L = p->L > 0 ? p->L : (!p->periodic_x ? p->nx - 1 : (p->periodic_z ? p->nz : p->nz - 1));
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
    if (p->Ra > 0 && d->dT != 0.0)
        d->gbeta = p->Ra * d->nu * d->alpha_e / (d->dT * d->L * d->L * d->L);
    else
        d->gbeta = 0.0;
    d->K = p->Da * d->L * d->L;
    d->ergun = isnan(p->F_eps) ? 1 : 0;
    if (!(d->nu_e > 0) || !(d->alpha_e > 0) || !(d->K > 0)) return -2;
    return 0;
}

static double delta(int a, int b) { return a == b ? 1.0 : 0.0; }

/* f_i^{e(0)} (Eq. EQFIN without the shear-rate term). */
static void feq0(double eps, double p, const double u[3], double out[Q19])
{
    for (int i = 0; i < Q19; ++i) {
        double cu = 0.0, uucc = 0.0;
        for (int a = 0; a < 3; ++a) cu += C3[i][a] * u[a];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) uucc += u[a] * u[b] * (C3[i][a] * C3[i][b] - CS2 * delta(a, b));
        double si = W3[i] * (cu / CS2 + uucc / (2.0 * eps * CS2 * CS2));
        out[i] = (i == 0 ? RHO0 - (1.0 - W3[0]) * eps * p / CS2 : W3[i] * eps * p / CS2) + RHO0 * si;
    }
}

/* Full flow EDF: f^{e(0)} + rho0 r_i with r_i = omega_i A S:(c c - cs^2 I) / (2 cs^2). */
static void feq_full(const o3_sim *s, double eps, double p, const double u[3], double S[3][3], double out[Q19])
{
    feq0(eps, p, u, out);
    for (int i = 0; i < Q19; ++i) {
        double Scc = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Scc += S[a][b] * (C3[i][a] * C3[i][b] - CS2 * delta(a, b));
        out[i] += RHO0 * W3[i] * s->d.A * Scc / (2.0 * CS2);
    }
}

/* g_i^{e(0)} (Eq. TeEDFEQ without the gradient term). */
static void geq0(const o3_sim *s, double eps, double T, const double u[3], double p, double out[Q19])
{
    const double sigma = s->prm.sigma;
    for (int i = 0; i < Q19; ++i) {
        double cu = 0.0, uucc = 0.0;
        for (int a = 0; a < 3; ++a) cu += C3[i][a] * u[a];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) uucc += u[a] * u[b] * (C3[i][a] * C3[i][b] - CS2 * delta(a, b));
        out[i] = W3[i] * T * (sigma + cu / CS2 + uucc / (2.0 * eps * CS2 * CS2))
               + varpi(i) * T * eps * p / (CS2 * RHO0);
    }
}

static void geq_full(const o3_sim *s, double eps, double T, const double u[3], double p, const double dT[3],
                     double out[Q19])
{
    geq0(s, eps, T, u, p, out);
    for (int i = 0; i < Q19; ++i) {
        double cg = 0.0;
        for (int a = 0; a < 3; ++a) cg += C3[i][a] * dT[a];
        out[i] += s->prm.sigma * W3[i] * s->d.B * cg;
    }
}

static void porous_coeffs(const o3_sim *s, double eps, double *Feps, double *c0, double *c1)
{
    const double K = s->d.K, nu = s->d.nu;
    *Feps = s->d.ergun ? 1.75 / sqrt(150.0 * eps * eps * eps) : s->prm.F_eps;
    *c0 = 0.5 * (1.0 + eps * 0.5 * nu / K);
    *c1 = eps * 0.5 * *Feps / sqrt(K);
}

/* F of Eq. ForceEq at velocity u and buoyancy G. */
static void force_of(const o3_sim *s, double eps, const double u[3], const double G[3], double F[3])
{
    double Feps, c0, c1;
    porous_coeffs(s, eps, &Feps, &c0, &c1);
    double um = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (int a = 0; a < 3; ++a)
        F[a] = -eps * s->d.nu / s->d.K * u[a] - eps * Feps / sqrt(s->d.K) * um * u[a] + eps * G[a];
}

/* det of a 3 x 3 matrix */
static double det3(double M[3][3])
{
    return M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1])
         - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0])
         + M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
}

/* Macroscopic state of a node from its pre-collision populations, in the order of the
 * 2-D model: T, G, v and u (drag solve), F, p, S (Eq. ShearEqCom), grad T (Eqs. MatrM,
 * MatrN, TeEqCom). */
static void node_macro(const o3_sim *s, double eps, const double *f, const double *g, o3_macro *m)
{
    const o3_params *P = &s->prm;
    const o3_derived *D = &s->d;
    const double sigma = P->sigma, Q = P->Q, tf = P->tau_f, tT = P->tau_T;
    m->eps = eps;
    double sg = 0.0;
    for (int i = 0; i < Q19; ++i) sg += g[i];
    m->T = (sg + 0.5 * Q) / sigma;
    for (int a = 0; a < 3; ++a) m->G[a] = P->a[a];
    m->G[2] += D->gbeta * (m->T - D->T0);

    double v[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q19; ++i)
        for (int a = 0; a < 3; ++a) v[a] += C3[i][a] * f[i];
    for (int a = 0; a < 3; ++a) v[a] = v[a] / RHO0 + 0.5 * eps * m->G[a];
    double Feps, c0, c1;
    porous_coeffs(s, eps, &Feps, &c0, &c1);
    double vm = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    double den = c0 + sqrt(c0 * c0 + c1 * vm);
    for (int a = 0; a < 3; ++a) m->u[a] = v[a] / den;
    force_of(s, eps, m->u, m->G, m->F);

    double uF = 0.0, uu = 0.0;
    for (int a = 0; a < 3; ++a) { uF += m->u[a] * m->F[a]; uu += m->u[a] * m->u[a]; }
    double s0 = -W3[0] / (2.0 * eps * CS2) * uu;
    double F0 = -W3[0] * (1.0 - 1.0 / (2.0 * tf)) * uF / (eps * CS2);
    double sumf = 0.0;
    for (int i = 1; i < Q19; ++i) sumf += f[i];
    m->p = CS2 / (eps * (1.0 - W3[0])) * (sumf + tf * F0 + RHO0 * s0);

    double e0[Q19];
    feq0(eps, m->p, m->u, e0);
    double Pi[3][3] = {{0}};
    for (int i = 0; i < Q19; ++i)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Pi[a][b] += C3[i][a] * C3[i][b] * (f[i] - e0[i]);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            m->S[a][b] = (Pi[a][b] + 0.5 * RHO0 * (m->u[a] * m->F[b] + m->F[a] * m->u[b]) / eps)
                       / (CS2 * RHO0 * (D->A - tf));

    double ge0[Q19];
    geq0(s, eps, m->T, m->u, m->p, ge0);
    double N[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q19; ++i)
        for (int a = 0; a < 3; ++a) N[a] += C3[i][a] * (g[i] - ge0[i]);
    for (int a = 0; a < 3; ++a) N[a] += 0.5 * (m->T * m->F[a] + m->u[a] / sigma * Q);
    double M[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            M[a][b] = -eps * m->p / (2.0 * RHO0) * delta(a, b) - 0.5 * (1.0 / eps - 1.0 / sigma) * m->u[a] * m->u[b]
                    + CS2 * sigma * (D->B - tT) * delta(a, b);
    double dM = det3(M);
    for (int c = 0; c < 3; ++c) {
        double Mc[3][3];
        memcpy(Mc, M, sizeof(Mc));
        for (int a = 0; a < 3; ++a) Mc[a][c] = N[a];
        m->dT[c] = det3(Mc) / dM;
    }
}

/* F_i (Eq. FtermF), P_i and Q_i (Eq. Eq:Tforce), dt = 1. */
static void sources(const o3_sim *s, const o3_macro *m, double Fi[Q19], double Pi[Q19], double Qi[Q19])
{
    const double tf = s->prm.tau_f, tT = s->prm.tau_T, sigma = s->prm.sigma, Q = s->prm.Q;
    for (int i = 0; i < Q19; ++i) {
        double cF = 0.0, cu = 0.0, t2 = 0.0, cvec = 0.0, uucg = 0.0;
        for (int a = 0; a < 3; ++a) {
            cF += C3[i][a] * m->F[a];
            cu += C3[i][a] * m->u[a];
            cvec += C3[i][a] * (m->T * m->F[a] + m->eps * m->p * m->dT[a] / RHO0);
        }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                t2 += (m->u[a] * m->F[b] + m->F[a] * m->u[b]) * (C3[i][a] * C3[i][b] - CS2 * delta(a, b));
                uucg += m->u[a] * m->u[b] * C3[i][a] * m->dT[b];
            }
        Fi[i] = W3[i] * RHO0 * (1.0 - 1.0 / (2.0 * tf)) * (cF / CS2 + t2 / (2.0 * m->eps * CS2 * CS2));
        Pi[i] = W3[i] * (1.0 - 1.0 / (2.0 * tT)) * (cvec / CS2 + (1.0 / m->eps - 1.0 / sigma) * uucg / CS2);
        Qi[i] = W3[i] * (1.0 - 1.0 / (2.0 * tT)) * (1.0 + cu / (sigma * CS2)) * Q;
    }
}

/* BGK collision with the equilibria and sources of state m (Eqs. LBEeq, TEqColli). */
static void collide_state(const o3_sim *s, const o3_macro *m, const double *f, const double *g,
                          double *fo, double *go)
{
    double fe[Q19], ge[Q19], Fi[Q19], Pi[Q19], Qi[Q19], S[3][3];
    memcpy(S, m->S, sizeof(S));
    feq_full(s, m->eps, m->p, m->u, S, fe);
    geq_full(s, m->eps, m->T, m->u, m->p, m->dT, ge);
    sources(s, m, Fi, Pi, Qi);
    for (int i = 0; i < Q19; ++i) {
        fo[i] = f[i] - (f[i] - fe[i]) / s->prm.tau_f + Fi[i];
        go[i] = g[i] - (g[i] - ge[i]) / s->prm.tau_T + Pi[i] + Qi[i];
    }
}

static int idx(const o3_sim *s, int x, int y, int z) { return (z * s->prm.ny + y) * s->prm.nx + x; }

/* The walls a node lies on: zw in {-1, 0 (z = 0), 1 (z = nz - 1)}, xw in {-1, 2 (x = 0),
 * 3 (x = nx - 1)}, yw in {-1, 4 (y = 0), 5 (y = ny - 1)}. */
static void wall_of(const o3_sim *s, int x, int y, int z, int *xw, int *yw, int *zw)
{
    const o3_params *P = &s->prm;
    *xw = -1; *yw = -1; *zw = -1;
    if (!P->periodic_x) { if (x == 0) *xw = 2; else if (x == P->nx - 1) *xw = 3; }
    if (!P->periodic_y) { if (y == 0) *yw = 4; else if (y == P->ny - 1) *yw = 5; }
    if (!P->periodic_z) { if (z == 0) *zw = 0; else if (z == P->nz - 1) *zw = 1; }
}

static int is_wall(const o3_sim *s, int k)
{
    int xw, yw, zw;
    wall_of(s, k % s->prm.nx, (k / s->prm.nx) % s->prm.ny, k / (s->prm.nx * s->prm.ny), &xw, &yw, &zw);
    return xw >= 0 || yw >= 0 || zw >= 0;
}

static void collide_all(o3_sim *s)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < s->n; ++k) {
        o3_macro m;
        if (is_wall(s, k)) m = s->mb[k];
        else node_macro(s, s->eps[k], s->f + Q19 * k, s->g + Q19 * k, &m);
        collide_state(s, &m, s->f + Q19 * k, s->g + Q19 * k, s->fs + Q19 * k, s->gs + Q19 * k);
    }
}

/* Push streaming, periodic where so set; populations leaving through a wall are dropped. */
static void stream_all(o3_sim *s)
{
    const int nx = s->prm.nx, ny = s->prm.ny, nz = s->prm.nz;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int k = idx(s, x, y, z);
                for (int i = 0; i < Q19; ++i) {
                    int zd = z + C3[i][2], xd = x + C3[i][0], yd = y + C3[i][1];
                    if (s->prm.periodic_z) zd = (zd + nz) % nz;
                    if (s->prm.periodic_x) xd = (xd + nx) % nx;
                    if (s->prm.periodic_y) yd = (yd + ny) % ny;
                    if (zd < 0 || zd >= nz || xd < 0 || xd >= nx || yd < 0 || yd >= ny) continue;
                    int kd = idx(s, xd, yd, zd);
                    s->f[Q19 * kd + i] = s->fs[Q19 * k + i];
                    s->g[Q19 * kd + i] = s->gs[Q19 * k + i];
                }
            }
}

/* Non-equilibrium extrapolation at wall node (x, y, z) (Sec. 3.4) and its state (R5). */
static void nees_node(o3_sim *s, int x, int y, int z)
{
    const o3_params *P = &s->prm;
    int xw, yw, zw;
    wall_of(s, x, y, z, &xw, &yw, &zw);
    const int dx = xw == 2 ? 1 : (xw == 3 ? -1 : 0), dz = zw == 0 ? 1 : (zw == 1 ? -1 : 0);
    const int dy = yw == 4 ? 1 : (yw == 5 ? -1 : 0);
    const int kb = idx(s, x, y, z), kf = idx(s, x + dx, y + dy, z + dz);
    const int kff = idx(s, x + 2 * dx, y + 2 * dy, z + 2 * dz);
    const double *ff = s->f + Q19 * kf, *gf = s->g + Q19 * kf;
    o3_macro mf;
    node_macro(s, s->eps[kf], ff, gf, &mf);
    const double eb = s->eps[kb];
    double fe_f[Q19], ge_f[Q19], fe_b[Q19], ge_b[Q19];
    feq_full(s, mf.eps, mf.p, mf.u, mf.S, fe_f);
    geq_full(s, mf.eps, mf.T, mf.u, mf.p, mf.dT, ge_f);
    /* an edge or a vertex is at rest (R8) */
    const double zero[3] = {0.0, 0.0, 0.0};
    const int nwalls = (xw >= 0) + (yw >= 0) + (zw >= 0);
    const double *ub = nwalls > 1 ? zero : P->wall_u[xw >= 0 ? xw : (yw >= 0 ? yw : zw)];
    feq_full(s, eb, mf.p, ub, mf.S, fe_b);
    for (int i = 0; i < Q19; ++i) s->f[Q19 * kb + i] = fe_b[i] + (ff[i] - fe_f[i]);

    /* an isothermal wall wins over a prescribed-gradient one; among isothermal walls x, then
     * y, then z (R8) */
    const int dir = (xw >= 0 && P->wall_kind[xw] == 0) ? xw
                  : ((yw >= 0 && P->wall_kind[yw] == 0) ? yw : ((zw >= 0 && P->wall_kind[zw] == 0) ? zw : -1));
    double Tb, gb[3] = {mf.dT[0], mf.dT[1], mf.dT[2]};
    if (dir >= 0) {
        Tb = P->wall_T[dir];
    } else {
        if (xw >= 0) gb[0] = dx * P->wall_dTdn[xw];
        if (yw >= 0) gb[1] = dy * P->wall_dTdn[yw];
        if (zw >= 0) gb[2] = dz * P->wall_dTdn[zw];
        double sgff = 0.0;
        for (int i = 0; i < Q19; ++i) sgff += s->g[Q19 * kff + i];
        double Tff = (sgff + 0.5 * P->Q) / P->sigma;
        Tb = (4.0 * mf.T - Tff - 2.0 * (dx * gb[0] + dy * gb[1] + dz * gb[2])) / 3.0;
    }
    geq_full(s, eb, Tb, ub, mf.p, gb, ge_b);
    for (int i = 0; i < Q19; ++i) s->g[Q19 * kb + i] = ge_b[i] + (gf[i] - ge_f[i]);

    o3_macro *m = &s->mb[kb];
    m->eps = eb;
    m->T = Tb;
    for (int a = 0; a < 3; ++a) { m->u[a] = ub[a]; m->G[a] = P->a[a]; m->dT[a] = gb[a]; }
    m->G[2] += s->d.gbeta * (Tb - s->d.T0);
    force_of(s, eb, m->u, m->G, m->F);
    m->p = mf.p;
    memcpy(m->S, mf.S, sizeof(m->S));
}

static void boundary_all(o3_sim *s)
{
    const int nx = s->prm.nx, ny = s->prm.ny;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < s->n; ++k)
        if (is_wall(s, k)) nees_node(s, k % nx, (k / nx) % ny, k / (nx * ny));
}

/* ---------------------------------------------------------------------------- */
/* Exported interface (ctypes)                                                   */
/* ---------------------------------------------------------------------------- */
int o3_lattice(int32_t *c, double *w)
{
    build_lattice();
    for (int i = 0; i < Q19; ++i) {
        for (int a = 0; a < 3; ++a) c[3 * i + a] = C3[i][a];
        w[i] = W3[i];
    }
    return Q19;
}

int o3_derive(const o3_params *p, double *out /* 10 */)
{
    o3_derived d;
    int r = derive(p, &d);
    double v[10] = {d.L, d.A, d.B, d.nu_e, d.nu, d.alpha_e, d.gbeta, d.K, d.T0, d.dT};
    memcpy(out, v, sizeof(v));
    return r;
}

/* Initial fields (R1, R2): optional porosity, T, u per node ([z][y][x], u as three planes);
 * NULL means the uniform eps, u = 0 and T = T0 inside, T_wall on isothermal wall nodes.
 * p = 0. */
o3_sim *o3_create(const o3_params *p, const double *eps_field, const double *T_init, const double *u_init)
{
    build_lattice();
    o3_sim *s = (o3_sim *)calloc(1, sizeof(o3_sim));
    s->prm = *p;
    if ((!p->periodic_z && p->nz < 4) || (!p->periodic_x && p->nx < 4) || (!p->periodic_y && p->ny < 4)
        || derive(p, &s->d) != 0) { free(s); return NULL; }
    s->n = p->nx * p->ny * p->nz;
    s->f = (double *)malloc(sizeof(double) * Q19 * s->n);
    s->g = (double *)malloc(sizeof(double) * Q19 * s->n);
    s->fs = (double *)malloc(sizeof(double) * Q19 * s->n);
    s->gs = (double *)malloc(sizeof(double) * Q19 * s->n);
    s->mb = (o3_macro *)calloc((size_t)s->n, sizeof(o3_macro));
    s->eps = (double *)malloc(sizeof(double) * s->n);
    for (int k = 0; k < s->n; ++k) s->eps[k] = eps_field ? eps_field[k] : p->eps;
    double S0[3][3] = {{0}}, g0[3] = {0, 0, 0};
    for (int k = 0; k < s->n; ++k) {
        int z = k / (p->nx * p->ny);
        double T = s->d.T0;
        int xw, yw, zw;
        wall_of(s, k % p->nx, (k / p->nx) % p->ny, z, &xw, &yw, &zw);
        if (T_init) T = T_init[k];
        else if (xw >= 0 && p->wall_kind[xw] == 0) T = p->wall_T[xw];
        else if (yw >= 0 && p->wall_kind[yw] == 0) T = p->wall_T[yw];
        else if (zw >= 0 && p->wall_kind[zw] == 0) T = p->wall_T[zw];
        double u[3] = {0, 0, 0};
        if (u_init)
            for (int a = 0; a < 3; ++a) u[a] = u_init[(size_t)a * s->n + k];
        feq_full(s, s->eps[k], 0.0, u, S0, s->fs + Q19 * k);
        geq_full(s, s->eps[k], T, u, 0.0, g0, s->gs + Q19 * k);
    }
    memcpy(s->f, s->fs, sizeof(double) * Q19 * s->n);
    memcpy(s->g, s->gs, sizeof(double) * Q19 * s->n);
    stream_all(s);
    boundary_all(s);
    s->t = 0;
    return s;
}

void o3_destroy(o3_sim *s)
{
    if (!s) return;
    free(s->eps); free(s->f); free(s->g); free(s->fs); free(s->gs); free(s->mb);
    free(s);
}

void o3_step(o3_sim *s, int64_t nsteps)
{
    for (int64_t k = 0; k < nsteps; ++k) {
        collide_all(s);
        stream_all(s);
        boundary_all(s);
        s->t += 1;
    }
}

/* Fields at the current time, [z][y][x] each: p, u (3 planes), T, S (xx, xy, xz, yy, yz,
 * zz), grad T (3 planes); any output may be NULL.  Wall nodes report their state (R5). */
void o3_fields(const o3_sim *s, double *p, double *u, double *T, double *S, double *dT)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < s->n; ++k) {
        o3_macro m;
        if (is_wall(s, k)) m = s->mb[k];
        else node_macro(s, s->eps[k], s->f + Q19 * k, s->g + Q19 * k, &m);
        if (p) p[k] = m.p;
        if (T) T[k] = m.T;
        for (int a = 0; a < 3; ++a) {
            if (u) u[(size_t)a * s->n + k] = m.u[a];
            if (dT) dT[(size_t)a * s->n + k] = m.dT[a];
        }
        if (S) {
            const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
            for (int c = 0; c < 6; ++c) S[(size_t)c * s->n + k] = 0.5 * (m.S[ia[c]][ib[c]] + m.S[ib[c]][ia[c]]);
        }
    }
}

/* Populations [19][nz][ny][nx]; which: 0 = pre-collision now, 1 = post-collision of the
 * previous step. */
void o3_get_populations(const o3_sim *s, int which, double *f_out, double *g_out)
{
    const double *f = which ? s->fs : s->f, *g = which ? s->gs : s->g;
    for (int i = 0; i < Q19; ++i)
        for (int k = 0; k < s->n; ++k) {
            f_out[(size_t)i * s->n + k] = f[Q19 * k + i];
            g_out[(size_t)i * s->n + k] = g[Q19 * k + i];
        }
}

/* Average Nusselt number of wall w (0: z = 0, 1: z = nz - 1, 2: x = 0, 3: x = nx - 1,
 * 4: y = 0, 5: y = ny - 1) as in two dimensions (R14): -L dT/dn / dT, n the wall's axis
 * (+z, +x, +y), by the one-sided second-order difference into the fluid, averaged over the
 * wall plane by the trapezoid rule along each walled in-plane direction and a plain mean
 * along each periodic one. */
double o3_nusselt(const o3_sim *s, int w)
{
    const int nn[3] = {s->prm.nx, s->prm.ny, s->prm.nz};
    const int per[3] = {s->prm.periodic_x, s->prm.periodic_y, s->prm.periodic_z};
    const int ax = w < 2 ? 2 : (w < 4 ? 0 : 1), hi = w & 1;
    double *T = (double *)malloc(sizeof(double) * s->n);
    o3_fields(s, NULL, NULL, T, NULL, NULL);
    double acc = 0.0, cells = 1.0;
    for (int b = 0; b < 3; ++b)
        if (b != ax) cells *= per[b] ? nn[b] : nn[b] - 1;
    int c[3];
    for (c[2] = 0; c[2] < nn[2]; ++c[2])
        for (c[1] = 0; c[1] < nn[1]; ++c[1])
            for (c[0] = 0; c[0] < nn[0]; ++c[0]) {
                if (c[ax] != (hi ? nn[ax] - 1 : 0)) continue;
                double Tv[3], wt = 1.0;
                for (int d = 0; d < 3; ++d) {
                    int e[3] = {c[0], c[1], c[2]};
                    e[ax] = hi ? nn[ax] - 1 - d : d;
                    Tv[d] = T[idx(s, e[0], e[1], e[2])];
                }
                for (int b = 0; b < 3; ++b)
                    if (b != ax && !per[b] && (c[b] == 0 || c[b] == nn[b] - 1)) wt *= 0.5;
                const double dn = (hi ? -1.0 : 1.0) * (-3.0 * Tv[0] + 4.0 * Tv[1] - Tv[2]) / 2.0;
                acc += wt * (-s->d.L * dn / s->d.dT);
            }
    free(T);
    return acc / cells;
}

/* ---------------------------------------------------------------------------- */
/* Single-node building blocks, exposed for the identity pins.  They run the same */
/* functions as the time step on one node of the problem p (its derived constants */
/* A, B, nu, K, ...), with the porosity eps given.                                */
/* ---------------------------------------------------------------------------- */
static int node_context(const o3_params *p, o3_sim *s)
{
    build_lattice();
    memset(s, 0, sizeof(*s));
    s->prm = *p;
    return derive(p, &s->d);
}

/* Macroscopic state of a node from its pre-collision populations f[19], g[19]:
 * out = T, G (3), u (3), F (3), p, S (9, row-major), grad T (3): 23 values. */
int o3_node_macro(const o3_params *p, double eps, const double *f, const double *g, double *out)
{
    o3_sim s;
    int r = node_context(p, &s);
    o3_macro m;
    node_macro(&s, eps, f, g, &m);
    int k = 0;
    out[k++] = m.T;
    for (int a = 0; a < 3; ++a) out[k++] = m.G[a];
    for (int a = 0; a < 3; ++a) out[k++] = m.u[a];
    for (int a = 0; a < 3; ++a) out[k++] = m.F[a];
    out[k++] = m.p;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) out[k++] = m.S[a][b];
    for (int a = 0; a < 3; ++a) out[k++] = m.dT[a];
    return r;
}

/* The discrete terms of one node for prescribed macroscopic values (T, u[3], p, S[9]
 * row-major, grad T[3], F[3]): out rows of 19 values, in order f^{e(0)} (Eq. EQFIN
 * without the shear-rate term), r_i (the A S term of Eq. EQTSHIN, without rho0),
 * g^{e(0)} (Eq. TeEDFEQ without the gradient term), the B grad T term of g^eq, F_i
 * (Eq. FtermF), P_i and Q_i (Eq. Eq:Tforce): 7 x 19 values. */
int o3_node_terms(const o3_params *p, double eps, double T, const double *u, double pr, const double *S9,
                  const double *dT, const double *F, double *out)
{
    o3_sim s;
    int r = node_context(p, &s);
    double S[3][3], full[Q19];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) S[a][b] = S9[3 * a + b];
    feq0(eps, pr, u, out);
    feq_full(&s, eps, pr, u, S, full);
    for (int i = 0; i < Q19; ++i) out[Q19 + i] = (full[i] - out[i]) / RHO0;
    geq0(&s, eps, T, u, pr, out + 2 * Q19);
    geq_full(&s, eps, T, u, pr, dT, full);
    for (int i = 0; i < Q19; ++i) out[3 * Q19 + i] = full[i] - out[2 * Q19 + i];
    o3_macro m;
    memset(&m, 0, sizeof(m));
    m.eps = eps;
    m.T = T;
    m.p = pr;
    for (int a = 0; a < 3; ++a) { m.u[a] = u[a]; m.F[a] = F[a]; m.dT[a] = dT[a]; }
    sources(&s, &m, out + 4 * Q19, out + 5 * Q19, out + 6 * Q19);
    return r;
}

/* Collision of one bulk node: pre-collision f, g -> post-collision fo, go. */
int o3_node_collide(const o3_params *p, double eps, const double *f, const double *g, double *fo, double *go)
{
    o3_sim s;
    int r = node_context(p, &s);
    o3_macro m;
    node_macro(&s, eps, f, g, &m);
    collide_state(&s, &m, f, g, fo, go);
    return r;
}
