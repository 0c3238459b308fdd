// Device-side arithmetic of one lattice node for the modified lattice-BGK model of
// convection heat transfer in porous media (Wang, Mi & Guo, arXiv:1505.02976).
//
// Populations are held as deviations from the rest state, f'_i = f_i - rho0 delta_i0 and
// g'_i = g_i - omega_i sigma T0, so that FP32 arithmetic keeps the small physical signal
// (every moment used below is linear in the populations, so the rest state drops out
// exactly).  Tensor contractions are expanded into scalar forms, e.g.
//   uu:(c c - cs^2 I) = (c.u)^2 - cs^2 |u|^2,   S:(c c - cs^2 I) = c.S.c - cs^2 tr S,
//   (uF + Fu):(c c - cs^2 I) = 2 (c.u)(c.F) - 2 cs^2 u.F,   uu:(c grad T) = (c.u)(u.grad T),
// with cs^2 = 1/3 and rho0 = 1 folded into the constants.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace lbm {

// D2Q9 (Sec. 3.1)
__device__ constexpr int CXd[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int CYd[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__host__ __device__ constexpr double Wd(int i) { return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0); }

// Kernel parameter block (plain data, passed by value).
struct KParams {
    int nx, ny, px, py;          // grid, periodic flags
    int pitch;                   // row pitch in elements
    int nwall;                   // number of wall-node slots enumerated by the wall kernels
    long long plane;             // stride between population planes, elements
    double tau_f, tau_T, A, B, sigma, Q, gbeta, T0, ax, ay;
    double nu_over_K, inv_sqrtK; // 0 when K is infinite
    double Feps;                 // Forchheimer coefficient when not from Ergun
    int ergun;
    int field;                   // porosity field present
    const double *eps_field;     // [ny][nx] (workspace copy) or null
    // coefficients for the uniform porosity
    double eps, c0, c1, dlin, dquad;
    double wall_ux[4], wall_uy[4], wall_T[4], wall_dTdn[4];
    int wall_kind[4];
    float hscale, hinv;          // FP16 storage scale
};

// Storage traits: load/store of a deviation value.
template <typename S> struct Store;
template <> struct Store<double> {
    static __device__ __forceinline__ double ld(const double *p, float) { return *p; }
    static __device__ __forceinline__ void st(double *p, double v, float) { __builtin_nontemporal_store(v, p); }
};
template <> struct Store<float> {
    static __device__ __forceinline__ float ld(const float *p, float) { return *p; }
    static __device__ __forceinline__ void st(float *p, float v, float) { __builtin_nontemporal_store(v, p); }
};
template <> struct Store<__half> {
    static __device__ __forceinline__ float ld(const __half *p, float inv) { return __half2float(*p) * inv; }
    static __device__ __forceinline__ void st(__half *p, float v, float scale) { *p = __float2half(v * scale); }
};

// Constants in the arithmetic type R.
template <typename R> struct Cst {
    R itf, itT;        // 1 / tau
    R fF, fT;          // 1 - 1 / (2 tau)
    R A, sigB, sig, isig, Q, gb, ax, ay;
    R Sden;            // 1 / (cs^2 (A - tau_f))
    R aM0;             // cs^2 sigma (B - tau_T)
    R halfQ;
};

template <typename R> __device__ __forceinline__ Cst<R> make_cst(const KParams &P)
{
    Cst<R> k;
    k.itf = R(1.0 / P.tau_f);
    k.itT = R(1.0 / P.tau_T);
    k.fF = R(1.0 - 0.5 / P.tau_f);
    k.fT = R(1.0 - 0.5 / P.tau_T);
    k.A = R(P.A);
    k.sigB = R(P.sigma * P.B);
    k.sig = R(P.sigma);
    k.isig = R(1.0 / P.sigma);
    k.Q = R(P.Q);
    k.halfQ = R(0.5 * P.Q);
    k.gb = R(P.gbeta);
    k.ax = R(P.ax);
    k.ay = R(P.ay);
    k.Sden = R(3.0 / (P.A - P.tau_f));
    k.aM0 = R(P.sigma * (P.B - P.tau_T) / 3.0);
    return k;
}

// Porosity-dependent coefficients (Sec. 3.1 for c0 and c1; Eq. ForceEq for the drag).
template <typename R> struct EpsC {
    R eps, ieps, dlin, dquad, bM;
    double c0, c1, epsd;
};

template <typename R> __device__ __forceinline__ EpsC<R> eps_uniform(const KParams &P)
{
    EpsC<R> e;
    e.epsd = P.eps;
    e.eps = R(P.eps);
    e.ieps = R(1.0 / P.eps);
    e.c0 = P.c0;
    e.c1 = P.c1;
    e.dlin = R(P.dlin);
    e.dquad = R(P.dquad);
    e.bM = R(0.5 * (1.0 / P.eps - 1.0 / P.sigma));
    return e;
}

template <typename R> __device__ __forceinline__ EpsC<R> eps_at(const KParams &P, int x, int y)
{
    if (!P.field) return eps_uniform<R>(P);
    const double eps = P.eps_field[(long long)y * P.nx + x];
    const double Fe = P.ergun ? 1.75 / sqrt(150.0 * eps * eps * eps) : P.Feps;
    EpsC<R> e;
    e.epsd = eps;
    e.eps = R(eps);
    e.ieps = R(1.0 / eps);
    e.c0 = 0.5 * (1.0 + 0.5 * eps * P.nu_over_K);
    e.c1 = 0.5 * eps * Fe * P.inv_sqrtK;
    e.dlin = R(eps * P.nu_over_K);
    e.dquad = R(eps * Fe * P.inv_sqrtK);
    e.bM = R(0.5 * (1.0 / eps - 1.0 / P.sigma));
    return e;
}

// Macroscopic quantities of a node (Td = T - T0).
template <typename R> struct Macro {
    R Td, ux, uy, Fx, Fy, p, Sxx, Sxy, Syy, gx, gy;
};

// Local quantities from pre-collision deviations f'[9], g'[9]:
//   sigma T = sum g + Q/2 (Sec. 3.2); G = g beta (T - T0) j + a (Sec. 2);
//   v = sum c f + eps G / 2 and u = v / (c0 + sqrt(c0^2 + c1 |v|)) in FP64 (Sec. 3.1);
//   F (Eq. ForceEq); p from sum_{i>0} f_i with tau_f F_0 and s_0 (Sec. 3.1, closed forms
//   of App. A); S (Eq. ShearEqCom) with sum c c f^{e(0)} = eps p I + u u / eps;
//   grad T = <M>^{-1} <N> (Eqs. MatrM, MatrN) for <M> = a I - b u u by the
//   Sherman-Morrison form, whose denominator is the second factor of Eq. detMatr.
template <typename R>
__device__ __forceinline__ void node_macro(const R *f, const R *g, const Cst<R> &k,
                                           const EpsC<R> &e, Macro<R> &m)
{
    const R sg = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
    m.Td = (sg + k.halfQ) * k.isig;
    const R Gx = k.ax;
    const R Gy = k.ay + k.gb * m.Td;

    const R jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    const R jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
    const double vx = double(jx) + 0.5 * e.epsd * double(Gx);
    const double vy = double(jy) + 0.5 * e.epsd * double(Gy);
    const double vm = sqrt(vx * vx + vy * vy);
    const double iden = 1.0 / (e.c0 + sqrt(e.c0 * e.c0 + e.c1 * vm));
    m.ux = R(vx * iden);
    m.uy = R(vy * iden);
    const R um = R(vm * iden);

    const R dl = e.dlin + e.dquad * um;
    m.Fx = e.eps * Gx - dl * m.ux;
    m.Fy = e.eps * Gy - dl * m.uy;

    const R uu = m.ux * m.ux + m.uy * m.uy;
    const R uF = m.ux * m.Fx + m.uy * m.Fy;
    const R s18 = ((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8]));
    // s_0 = -omega_0 |u|^2 / (2 eps cs^2),  F_0 = -omega_0 fF (u.F) / (eps cs^2)
    const R s0 = R(-2.0 / 3.0) * uu * e.ieps;
    const R F0 = R(-4.0 / 3.0) * k.fF * uF * e.ieps;
    const R tau_f = R(1) / k.itf;
    m.p = R(0.6) * e.ieps * (s18 + tau_f * F0 + s0);

    const R ep = e.eps * m.p;
    const R Pxx = ((f[1] + f[3]) + (f[5] + f[6])) + (f[7] + f[8]);
    const R Pyy = ((f[2] + f[4]) + (f[5] + f[6])) + (f[7] + f[8]);
    const R Pxy = (f[5] - f[6]) + (f[7] - f[8]);
    m.Sxx = (Pxx - ep - (m.ux * m.ux - m.ux * m.Fx) * e.ieps) * k.Sden;
    m.Syy = (Pyy - ep - (m.uy * m.uy - m.uy * m.Fy) * e.ieps) * k.Sden;
    m.Sxy = (Pxy - (m.ux * m.uy - R(0.5) * (m.ux * m.Fy + m.Fx * m.uy)) * e.ieps) * k.Sden;

    const R jgx = (g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7]);
    const R jgy = (g[2] - g[4]) + (g[5] + g[6]) - (g[7] + g[8]);
    m.gx = jgx;   // temporarily hold the thermal flux; finished in node_gradT
    m.gy = jgy;
}

// Completes grad T once the absolute temperature is known (T = T0 + Td).
template <typename R>
__device__ __forceinline__ void node_gradT(Macro<R> &m, R T0, const Cst<R> &k, const EpsC<R> &e)
{
    const R T = T0 + m.Td;
    const R Nx = m.gx - T * m.ux + R(0.5) * (T * m.Fx + m.ux * k.Q * k.isig);
    const R Ny = m.gy - T * m.uy + R(0.5) * (T * m.Fy + m.uy * k.Q * k.isig);
    const R a = k.aM0 - R(0.5) * e.eps * m.p;
    const R uu = m.ux * m.ux + m.uy * m.uy;
    const R uN = m.ux * Nx + m.uy * Ny;
    const R c = e.bM * uN / (a - e.bM * uu);
    const R ia = R(1) / a;
    m.gx = (Nx + c * m.ux) * ia;
    m.gy = (Ny + c * m.uy) * ia;
}

template <typename R>
__device__ __forceinline__ void node_macro_full(const R *f, const R *g, R T0, const Cst<R> &k,
                                                const EpsC<R> &e, Macro<R> &m)
{
    node_macro(f, g, k, e, m);
    node_gradT(m, T0, k, e);
}

// Flow equilibrium deviation f^eq_i - rho0 delta_i0 (Eqs. EQFIN, EQTSHIN) for pressure
// term ep = eps p, velocity u at porosity 1/ieps, and shear rate S.
template <typename R>
__device__ __forceinline__ R feq_i(int i, R ep, R ux, R uy, R ieps, R Sxx, R Sxy, R Syy, R A)
{
    const R uu = ux * ux + uy * uy;
    const R trS = Sxx + Syy;
    if (i == 0)
        return R(-5.0 / 3.0) * ep - R(2.0 / 3.0) * uu * ieps - R(2.0 / 9.0) * A * trS;
    const R cx = R(CXd[i]), cy = R(CYd[i]);
    const R cu = cx * ux + cy * uy;
    const R cSc = cx * cx * Sxx + R(2) * cx * cy * Sxy + cy * cy * Syy;
    return R(Wd(i)) * (R(3) * ep + R(3) * cu + (R(4.5) * cu * cu - R(1.5) * uu) * ieps
                       + A * (R(1.5) * cSc - R(0.5) * trS));
}

// Temperature equilibrium deviation g^eq_i - omega_i sigma T0 (Eq. TeEDFEQ) for
// temperature T = T0 + Td, velocity u, eps p, porosity 1/ieps and gradient (gx, gy).
template <typename R>
__device__ __forceinline__ R geq_i(int i, R Td, R T, R ux, R uy, R ieps, R ep, R gx, R gy,
                                   const Cst<R> &k)
{
    const R uu = ux * ux + uy * uy;
    if (i == 0)
        return R(4.0 / 9.0) * k.sig * Td - R(2.0 / 3.0) * T * uu * ieps - R(5.0 / 3.0) * T * ep;
    const R cx = R(CXd[i]), cy = R(CYd[i]);
    const R cu = cx * ux + cy * uy;
    const R cg = cx * gx + cy * gy;
    return R(Wd(i)) * (k.sig * Td + T * (R(3) * cu + (R(4.5) * cu * cu - R(1.5) * uu) * ieps)
                       + R(3) * T * ep + k.sigB * cg);
}

// BGK collision with forcing and sources, in place (Eqs. LBEeq, FtermF, TEqColli,
// Eq:Tforce):  f* = f - (f - f^eq)/tau_f + F_i,  g* = g - (g - g^eq)/tau_T + P_i + Q_i.
template <typename R>
__device__ __forceinline__ void node_collide(R *f, R *g, const Macro<R> &m, R T0,
                                             const Cst<R> &k, const EpsC<R> &e)
{
    const R T = T0 + m.Td;
    const R ep = e.eps * m.p;
    const R uF = m.ux * m.Fx + m.uy * m.Fy;
    const R ugT = m.ux * m.gx + m.uy * m.gy;
    const R vx = T * m.Fx + ep * m.gx;   // T F + eps p grad T / rho0
    const R vy = T * m.Fy + ep * m.gy;
    const R bP = e.ieps - k.isig;         // 1/eps - 1/sigma
    const R of = R(1) - k.itf, og = R(1) - k.itT;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const R cx = R(CXd[i]), cy = R(CYd[i]);
        const R w = R(Wd(i));
        const R cu = cx * m.ux + cy * m.uy;
        const R fe = feq_i<R>(i, ep, m.ux, m.uy, e.ieps, m.Sxx, m.Sxy, m.Syy, k.A);
        const R cF = cx * m.Fx + cy * m.Fy;
        const R Fi = w * k.fF * (R(3) * cF + (R(9) * cu * cF - R(3) * uF) * e.ieps);
        f[i] = of * f[i] + k.itf * fe + Fi;

        const R ge = geq_i<R>(i, m.Td, T, m.ux, m.uy, e.ieps, ep, m.gx, m.gy, k);
        const R Pi = w * k.fT * R(3) * ((cx * vx + cy * vy) + bP * cu * ugT);
        const R Qi = w * k.fT * (R(1) + R(3) * cu * k.isig) * k.Q;
        g[i] = og * g[i] + k.itT * ge + Pi + Qi;
    }
}

// ---------------------------------------------------------------------------------
// Grid helpers
// ---------------------------------------------------------------------------------
__device__ __forceinline__ bool on_wall(const KParams &P, int x, int y)
{
    return (!P.px && (x == 0 || x == P.nx - 1)) || (!P.py && (y == 0 || y == P.ny - 1));
}

// Pull gather: pre-collision f_i(x, t) = f*_i(x - c_i, t - 1), periodic wrap.
template <typename S, typename R>
__device__ __forceinline__ void gather(const S *__restrict__ src, const KParams &P, int x, int y,
                                       R *f, R *g)
{
    const int xm = (x == 0) ? P.nx - 1 : x - 1;
    const int xp = (x == P.nx - 1) ? 0 : x + 1;
    const int ym = (y == 0) ? P.ny - 1 : y - 1;
    const int yp = (y == P.ny - 1) ? 0 : y + 1;
    const long long r0 = (long long)y * P.pitch, rm = (long long)ym * P.pitch,
                    rp = (long long)yp * P.pitch;
    const long long off[9] = {r0 + x, r0 + xm, rm + x, r0 + xp, rp + x,
                              rm + xm, rm + xp, rp + xp, rp + xm};
    const float inv = P.hinv;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        f[i] = R(Store<S>::ld(src + i * P.plane + off[i], inv));
        g[i] = R(Store<S>::ld(src + (9 + i) * P.plane + off[i], inv));
    }
}

template <typename S, typename R>
__device__ __forceinline__ void store_node(S *__restrict__ dst, const KParams &P, int x, int y,
                                           const R *f, const R *g)
{
    const long long o = (long long)y * P.pitch + x;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        Store<S>::st(dst + i * P.plane + o, f[i], P.hscale);
        Store<S>::st(dst + (9 + i) * P.plane + o, g[i], P.hscale);
    }
}

// Wall classification: xw in {-1, 0, 1}, yw in {-1, 2, 3}; inward step (dx, dy).
struct WallInfo { int xw, yw, dx, dy; };

__device__ __forceinline__ WallInfo wall_info(const KParams &P, int x, int y)
{
    WallInfo w;
    w.xw = -1; w.yw = -1;
    if (!P.px) { if (x == 0) w.xw = 0; else if (x == P.nx - 1) w.xw = 1; }
    if (!P.py) { if (y == 0) w.yw = 2; else if (y == P.ny - 1) w.yw = 3; }
    w.dx = (w.xw == 0) ? 1 : (w.xw == 1 ? -1 : 0);
    w.dy = (w.yw == 2) ? 1 : (w.yw == 3 ? -1 : 0);
    return w;
}

// Non-equilibrium extrapolation (Sec. 3.4, Eqs. FNEESEQFIN, NEESVel, TeEBounDFEQ,
// TNEESAp, TNEESApGra): rebuilds the pre-collision populations of wall node (x, y) from
// the streamed populations of its reference node x_f (and x_ff on Neumann walls).
template <typename S, typename R>
__device__ __forceinline__ void wall_populations(const S *__restrict__ src, const KParams &P,
                                                 const Cst<R> &k, int x, int y, R *f, R *g)
{
    const WallInfo w = wall_info(P, x, y);
    const int xf = x + w.dx, yf = y + w.dy;
    R ff[9], gf[9];
    gather<S, R>(src, P, xf, yf, ff, gf);
    const EpsC<R> ef = eps_at<R>(P, xf, yf);
    Macro<R> mf;
    const R T0 = R(P.T0);
    node_macro_full<R>(ff, gf, T0, k, ef, mf);
    const R Tf = T0 + mf.Td;
    const R epf = ef.eps * mf.p;

    R ubx = R(0), uby = R(0);
    if (w.xw >= 0 && w.yw < 0) { ubx = R(P.wall_ux[w.xw]); uby = R(P.wall_uy[w.xw]); }
    if (w.yw >= 0 && w.xw < 0) { ubx = R(P.wall_ux[w.yw]); uby = R(P.wall_uy[w.yw]); }
    const EpsC<R> eb = eps_at<R>(P, x, y);
    const R epb = eb.eps * mf.p;   // eps at the wall node, pressure of x_f

#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const R feb = feq_i<R>(i, epb, ubx, uby, eb.ieps, mf.Sxx, mf.Sxy, mf.Syy, k.A);
        const R fef = feq_i<R>(i, epf, mf.ux, mf.uy, ef.ieps, mf.Sxx, mf.Sxy, mf.Syy, k.A);
        f[i] = feb + (ff[i] - fef);
    }

    int dir = -1;
    if (w.xw >= 0 && P.wall_kind[w.xw] == 0) dir = w.xw;
    else if (w.yw >= 0 && P.wall_kind[w.yw] == 0) dir = w.yw;
    R Tdb, gbx, gby;
    if (dir >= 0) {
        Tdb = R(P.wall_T[dir] - P.T0);
        gbx = mf.gx;
        gby = mf.gy;
    } else {
        gbx = (w.xw >= 0) ? R(w.dx * P.wall_dTdn[w.xw]) : mf.gx;
        gby = (w.yw >= 0) ? R(w.dy * P.wall_dTdn[w.yw]) : mf.gy;
        const int xff = x + 2 * w.dx, yff = y + 2 * w.dy;
        const int xm = (xff == 0) ? P.nx - 1 : xff - 1;
        const int xp = (xff == P.nx - 1) ? 0 : xff + 1;
        const int ym = (yff == 0) ? P.ny - 1 : yff - 1;
        const int yp = (yff == P.ny - 1) ? 0 : yff + 1;
        const long long r0 = (long long)yff * P.pitch, rm = (long long)ym * P.pitch,
                        rp = (long long)yp * P.pitch;
        const long long off[9] = {r0 + xff, r0 + xm, rm + xff, r0 + xp, rp + xff,
                                  rm + xm, rm + xp, rp + xp, rp + xm};
        R sgff = R(0);
#pragma unroll
        for (int i = 0; i < 9; ++i)
            sgff += R(Store<S>::ld(src + (9 + i) * P.plane + off[i], P.hinv));
        const R Tdff = (sgff + k.halfQ) * k.isig;
        Tdb = (R(4) * mf.Td - Tdff - R(2) * (R(w.dx) * gbx + R(w.dy) * gby)) * R(1.0 / 3.0);
    }
    const R Tb = T0 + Tdb;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const R geb = geq_i<R>(i, Tdb, Tb, ubx, uby, eb.ieps, epb, gbx, gby, k);
        const R gef = geq_i<R>(i, mf.Td, Tf, mf.ux, mf.uy, ef.ieps, epf, mf.gx, mf.gy, k);
        g[i] = geb + (gf[i] - gef);
    }
}

// Wall-node slot s -> (x, y); returns false for slots that are not wall nodes of this
// grid.  Slots: [0, nx) bottom row, [nx, 2nx) top row, then [2nx, 2nx+ny) left column,
// [2nx+ny, 2nx+2ny) right column; columns skip the corner rows already covered.
__device__ __forceinline__ bool wall_slot(const KParams &P, int s, int &x, int &y)
{
    const int nx = P.nx, ny = P.ny;
    if (s < nx) { if (P.py) return false; x = s; y = 0; return true; }
    s -= nx;
    if (s < nx) { if (P.py) return false; x = s; y = ny - 1; return true; }
    s -= nx;
    if (s < ny) {
        if (P.px) return false;
        if (!P.py && (s == 0 || s == ny - 1)) return false;
        x = 0; y = s; return true;
    }
    s -= ny;
    if (s < ny) {
        if (P.px) return false;
        if (!P.py && (s == 0 || s == ny - 1)) return false;
        x = nx - 1; y = s; return true;
    }
    return false;
}

}  // namespace lbm
