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

// Population layout per storage type: rows of tiles of T consecutive nodes, each tile
// holding its 18 directions contiguously, [y][x / T][q][x % T], so that the 36 streams of a
// wavefront touch one contiguous block of memory per row instead of 36 distant planes.
// T = 62 for FP64 and FP32 (a two-step wavefront writes exactly one tile segment per
// direction), 128 for FP16.

namespace lbm {

template <typename S> struct TileOf;
template <> struct TileOf<double> { static constexpr int v = 62; };
template <> struct TileOf<float> { static constexpr int v = 62; };
template <> struct TileOf<__half> { static constexpr int v = 128; };
// Columns one wavefront updates: a whole tile when tiles are narrower than a wavefront
// (so that its stores cover whole tile segments), else 64.
template <typename S> struct Wspan {
    static constexpr int v = TileOf<S>::v < 64 ? TileOf<S>::v : 64;
};
inline constexpr int tile_of_storage(int storage)
{
    return storage == 0 ? TileOf<double>::v : (storage == 1 ? TileOf<float>::v : TileOf<__half>::v);
}

// D2Q9 (Sec. 3.1)
__device__ constexpr int CXd[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int CYd[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__host__ __device__ constexpr double Wd(int i) { return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0); }

// Forward-mode dual number (value, derivative) in FP64, used by the adjoint to evaluate
// directional derivatives of the node update with the same templated code.
struct Dual {
    double v, d;
    __host__ __device__ constexpr Dual() : v(0.0), d(0.0) {}
    __host__ __device__ explicit constexpr Dual(double a) : v(a), d(0.0) {}
    __host__ __device__ constexpr Dual(double a, double b) : v(a), d(b) {}
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__device__ __forceinline__ Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ __forceinline__ Dual operator/(Dual a, Dual b)
{
    const double q = a.v / b.v;
    return Dual(q, (a.d - q * b.d) / b.v);
}
__device__ __forceinline__ Dual &operator+=(Dual &a, Dual b) { a = a + b; return a; }
__device__ __forceinline__ Dual sqrt(Dual a)
{
    const double r = ::sqrt(a.v);
    return Dual(r, r > 0.0 ? 0.5 * a.d / r : 0.0);
}
using ::sqrt;   // keep the FP32/FP64 overloads visible next to the dual one

// Type of the FP64 quantities of the drag solve for arithmetic type R.
template <typename R> struct DragT { using T = double; };
template <> struct DragT<Dual> { using T = Dual; };

// 1 / tau and 1 - 1 / tau in the arithmetic type R with it + o == 1 exactly: the collision
// forms o f + it (...), whose zeroth moment then carries the state's own moment with the
// factor o + it = 1 (a rounded pair would scale the temperature deviation by 1 + 6e-8 per
// FP32 step).  o = fl(1 - fl(1 / tau)) and it = fl(1 - o): for tau > 1/2 one of the two
// subtractions is exact by Sterbenz's lemma, and then so is the other.
template <typename R> inline void relax_pair(double tau, R &it, R &o)
{
    const R i0 = R(1.0 / tau);
    o = R(1) - i0;
    it = R(1) - o;
}

// Products of launch constants that the collision uses, per direction class (0 axes,
// 1 diagonals) and per node, in the arithmetic type R.
template <typename R> struct ClassK {
    R w, w3;                     // omega, 3 omega
    R witf, witT;                // omega / tau_f, omega / tau_T
    R wQ;                        // (omega fT) Q
    R bsg;                       // (omega / tau_T) sigma B
    R w3fT, w3fF;                // 3 omega fT, 3 omega fF
};
template <typename R> struct NodeK {
    R A15, hA;                   // 1.5 A, 0.5 A
    R itTsig, fTQ, Qisig;        // sigma / tau_T, fT Q, Q / sigma
    R c9fF, cuFc;                // 9 fF, (-4/3 fF) tau_f
};

// Per-launch constants in the arithmetic type R, computed once on the host.
template <typename R> struct Cst {
    R itf, itT;        // 1 / tau
    R of, og;          // 1 - 1 / tau
    R fF, fT;          // 1 - 1 / (2 tau)
    R tau_f;
    R A, sigB, sig, isig, Q, halfQ, gb, ax, ay;
    R Sden;            // 1 / (cs^2 (A - tau_f))
    R aM0;             // cs^2 sigma (B - tau_T)
    R w1, w5;          // lattice weights 1/9, 1/36
    R w3a, w3d;        // 3 omega of axis / diagonal directions with 2 w3a + 4 w3d = 1 in R
    ClassK<R> cls[2];  // the products above, formed by derive_consts
    NodeK<R> nod;
};

// The products, formed from the base constants of a Cst in R (host and device: the
// stored copies and the ones a kernel forms itself are the same values).
template <typename R> __host__ __device__ inline ClassK<R> class_k_formed(const Cst<R> &k, int c)
{
    ClassK<R> d;
    const R w = c == 0 ? k.w1 : k.w5, w3 = c == 0 ? k.w3a : k.w3d;
    d.w = w;
    d.w3 = w3;
    d.witf = w * k.itf;
    d.witT = w * k.itT;
    d.wQ = (w * k.fT) * k.Q;
    d.bsg = (k.itT * w) * k.sigB;
    d.w3fT = w3 * k.fT;
    d.w3fF = w3 * k.fF;
    return d;
}

template <typename R> __host__ __device__ inline NodeK<R> node_k_formed(const Cst<R> &k)
{
    NodeK<R> d;
    d.A15 = R(1.5) * k.A;
    d.hA = R(0.5) * k.A;
    d.itTsig = k.itT * k.sig;
    d.fTQ = k.fT * k.Q;
    d.Qisig = k.Q * k.isig;
    d.c9fF = R(9) * k.fF;
    d.cuFc = (R(-4.0 / 3.0) * k.fF) * k.tau_f;
    return d;
}

// Stores the products in a Cst whose base constants are set.
template <typename R> __host__ __device__ inline void derive_consts(Cst<R> &c)
{
    c.cls[0] = class_k_formed(c, 0);
    c.cls[1] = class_k_formed(c, 1);
    c.nod = node_k_formed(c);
}

// The products as a kernel uses them: read from the Cst (PRE), or formed from its base
// constants (then the compiler keeps them in vector registers across the kernel's loops).
// Kernels that update one or two nodes per thread read them; a kernel that updates many
// nodes per wavefront forms them when that holds fewer registers.
template <bool PRE, typename R> __device__ __forceinline__ ClassK<R> class_k(const Cst<R> &k, int c)
{
    if constexpr (PRE) return k.cls[c];
    else return class_k_formed(k, c);
}

template <bool PRE, typename R> __device__ __forceinline__ NodeK<R> node_k(const Cst<R> &k)
{
    if constexpr (PRE) return k.nod;
    else return node_k_formed(k);
}

// Porosity-dependent coefficients in R (uniform porosity: computed on the host).
template <typename R> struct EpsR {
    R eps, ieps, dlin, dquad, bM;
};

// Kernel parameter block (plain data, passed by value).
struct KParams {
    int nx, ny, px, py;          // grid, periodic flags
    int ntx;                     // tiles per row (tiled layout)
    int nwall;                   // number of wall-node slots enumerated by the wall kernels
    int nwall_rows;              // slots of the two walled rows (the step's wall launch)
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
    Cst<double> cd;
    Cst<float> cf;
    EpsR<double> ed;
    EpsR<float> ef;
};

template <typename R> __device__ __forceinline__ const Cst<R> &cst(const KParams &P);
template <> __device__ __forceinline__ const Cst<double> &cst<double>(const KParams &P) { return P.cd; }
template <> __device__ __forceinline__ const Cst<float> &cst<float>(const KParams &P) { return P.cf; }
template <typename R> __device__ __forceinline__ const EpsR<R> &epsu(const KParams &P);
template <> __device__ __forceinline__ const EpsR<double> &epsu<double>(const KParams &P) { return P.ed; }
template <> __device__ __forceinline__ const EpsR<float> &epsu<float>(const KParams &P) { return P.ef; }

// Reciprocal: IEEE division in FP64 arithmetic, the hardware reciprocal (1 ulp) in FP32.
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ Dual rcp(Dual x) { return Dual(1.0) / x; }

// Element index of population q (0..17) of node (x, y) inside a population buffer of
// storage type S.
template <typename S>
__device__ __forceinline__ long long pidx(const KParams &P, int q, int x, int y)
{
    constexpr int T = TileOf<S>::v;
    return ((long long)(y * P.ntx + x / T) * 18 + q) * T + (x % T);
}

// FP64 reciprocal from the hardware estimate refined by two Newton steps (used by the
// FP64 drag solve of the FP32/FP16 paths, where the result is rounded to FP32).
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

// FP64 square root from the hardware reciprocal-square-root estimate and one Newton step
// (relative error below 1e-13, used where the result is rounded to FP32): sqrt_pos_nr for
// x > 0, sqrt_nr for x >= 0 (0 for x <= 0, where the estimate is infinite).
__device__ __forceinline__ double sqrt_pos_nr(double x)
{
    const double r = __builtin_amdgcn_rsq(x);
    const double s = x * r;
    const double e = fma(-s, s, x);
    return fma(e, 0.5 * r, s);
}
__device__ __forceinline__ double sqrt_nr(double x)
{
    const double s = sqrt_pos_nr(x);
    return x > 0.0 ? s : 0.0;
}

// Storage traits: load/store of a deviation value.  Stores are non-temporal (the next
// step reads them from HBM anyway); loads are plain (non-temporal loads measured slower).
template <typename T> __device__ __forceinline__ T ld_stream(const T *p) { return *p; }
template <typename S> struct Store;
template <> struct Store<double> {
    static __device__ __forceinline__ double ld(const double *p, float) { return ld_stream(p); }
    static __device__ __forceinline__ void st(double *p, double v, float) { __builtin_nontemporal_store(v, p); }
};
template <> struct Store<float> {
    static __device__ __forceinline__ float ld(const float *p, float) { return ld_stream(p); }
    static __device__ __forceinline__ void st(float *p, float v, float) { __builtin_nontemporal_store(v, p); }
};
template <> struct Store<__half> {
    static __device__ __forceinline__ float ld(const __half *p, float inv)
    {
        const unsigned short b = ld_stream(reinterpret_cast<const unsigned short *>(p));
        // one mixed-precision FMA converts and scales (the +0 keeps it an FMA)
        return __builtin_fmaf(__half2float(__ushort_as_half(b)), inv, 0.0f);
    }
    static __device__ __forceinline__ void st(__half *p, float v, float scale)
    {
        __builtin_nontemporal_store(__half_as_ushort(__float2half(v * scale)),
                                    reinterpret_cast<unsigned short *>(p));
    }
};

template <typename R> __device__ __forceinline__ const Cst<R> &make_cst(const KParams &P)
{
    return cst<R>(P);
}

// Porosity-dependent coefficients (Sec. 3.1 for c0 and c1; Eq. ForceEq for the drag).
template <typename R> struct EpsC {
    using D = typename DragT<R>::T;
    R eps, ieps, dlin, dquad, bM;
    D c0, c1, epsd;
};

template <typename R> __device__ __forceinline__ EpsC<R> eps_uniform(const KParams &P)
{
    const EpsR<R> &u = epsu<R>(P);
    EpsC<R> e;
    e.epsd = P.eps;
    e.eps = u.eps;
    e.ieps = u.ieps;
    e.dlin = u.dlin;
    e.dquad = u.dquad;
    e.bM = u.bM;
    e.c0 = P.c0;
    e.c1 = P.c1;
    return e;
}

// Coefficients at porosity eps (any of double, Dual): F_eps from the Ergun relation or
// as given, c0 and c1 of the velocity solve, the drag coefficients of Eq. ForceEq and
// b = (1/eps - 1/sigma)/2 of Eq. MatrM.
template <typename R>
__device__ __forceinline__ EpsC<R> eps_coeffs(const KParams &P, typename DragT<R>::T eps)
{
    using D = typename DragT<R>::T;
    const D ie = D(1.0) / eps;
    const D Fe = P.ergun ? D(1.75) / sqrt(D(150.0) * eps * eps * eps) : D(P.Feps);
    EpsC<R> e;
    e.epsd = eps;
    e.eps = R(eps);
    e.ieps = R(ie);
    e.c0 = D(0.5) * (D(1.0) + D(0.5) * eps * D(P.nu_over_K));
    e.c1 = D(0.5) * eps * Fe * D(P.inv_sqrtK);
    e.dlin = R(eps * D(P.nu_over_K));
    e.dquad = R(eps * Fe * D(P.inv_sqrtK));
    e.bM = R(D(0.5) * (ie - D(P.cd.isig)));   // isig = 1 / sigma, rounded once on the host
    return e;
}

__device__ __forceinline__ double eps_value(const KParams &P, int x, int y)
{
    return P.field ? P.eps_field[(long long)y * P.nx + x] : P.eps;
}

template <typename R> __device__ __forceinline__ EpsC<R> eps_at(const KParams &P, int x, int y)
{
    if (!P.field) return eps_uniform<R>(P);
    return eps_coeffs<R>(P, P.eps_field[(long long)y * P.nx + x]);
}

// Macroscopic quantities of a node (Td = T - T0).
template <typename R> struct Macro {
    R Td, ux, uy, Fx, Fy, p, Sxx, Sxy, Syy, gx, gy;
};

// FP64 part of the velocity computation (Sec. 3.1): u = v / (c0 + sqrt(c0^2 + c1 |v|)).
// Returns 1 / (c0 + sqrt(c0^2 + c1 |v|)) and |v|.  |v| is not differentiable at v = 0; the
// dual version takes the derivative of |v| there as 0, the limit in which u(v) is C^1
// with du/dv = I / (2 c0).
template <typename R, typename D>
__device__ __forceinline__ D drag_factor(D vx, D vy, D c0, D c1, D &vm)
{
    vm = sqrt(vx * vx + vy * vy);
    return D(1.0) / (c0 + sqrt(c0 * c0 + c1 * vm));
}
template <>
__device__ __forceinline__ double drag_factor<float, double>(double vx, double vy, double c0, double c1,
                                                             double &vm)
{
    vm = sqrt_nr(vx * vx + vy * vy);
    return rcp_nr(c0 + sqrt_pos_nr(c0 * c0 + c1 * vm));   // c0 > 0, c1 >= 0
}

// Local quantities from pre-collision deviations f'[9], g'[9]:
//   sigma T = sum g + Q/2 (Sec. 3.2); G = g beta (T - T0) j + a (Sec. 2);
//   v = sum c f + eps G / 2 and u = v / (c0 + sqrt(c0^2 + c1 |v|)) in FP64 (Sec. 3.1);
//   F (Eq. ForceEq); p from sum_{i>0} f_i with tau_f F_0 and s_0 (Sec. 3.1, closed forms
//   of App. A); S (Eq. ShearEqCom) with sum c c f^{e(0)} = eps p I + u u / eps;
//   grad T = <M>^{-1} <N> (Eqs. MatrM, MatrN) for <M> = a I - b u u by the
//   Sherman-Morrison form, whose denominator is the second factor of Eq. detMatr.
template <typename R, bool PRE = true>
__device__ __forceinline__ void node_macro(const R *f, const R *g, const Cst<R> &k,
                                           const EpsC<R> &e, Macro<R> &m)
{
    const R sg = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
    m.Td = (sg + k.halfQ) * k.isig;
    const R Gx = k.ax;
    const R Gy = k.ay + k.gb * m.Td;

    const R jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    const R jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
    using D = typename DragT<R>::T;
    const D vx = D(jx) + D(0.5) * e.epsd * D(Gx);
    const D vy = D(jy) + D(0.5) * e.epsd * D(Gy);
    D vm;
    const D iden = drag_factor<R, D>(vx, vy, e.c0, e.c1, vm);
    m.ux = R(vx * iden);
    m.uy = R(vy * iden);
    const R um = R(vm * iden);

    const R dl = e.dlin + e.dquad * um;
    m.Fx = e.eps * Gx - dl * m.ux;
    m.Fy = e.eps * Gy - dl * m.uy;

    const R uu = m.ux * m.ux + m.uy * m.uy;
    const R uF = m.ux * m.Fx + m.uy * m.Fy;
    const R s18 = ((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8]));
    // rho0 s_0 = -omega_0 |u|^2 / (2 eps cs^2),  tau_f F_0 = -omega_0 tau_f fF (u.F) / (eps cs^2);
    // their coefficients depend only on the porosity and the launch constants
    const R cuu = R(-2.0 / 3.0) * e.ieps, cuF = node_k<PRE>(k).cuFc * e.ieps;
    m.p = (R(0.6) * e.ieps) * (s18 + cuu * uu + cuF * uF);

    const R ep = e.eps * m.p;
    const R Pxx = ((f[1] + f[3]) + (f[5] + f[6])) + (f[7] + f[8]);
    const R Pyy = ((f[2] + f[4]) + (f[5] + f[6])) + (f[7] + f[8]);
    const R Pxy = (f[5] - f[6]) + (f[7] - f[8]);
    m.Sxx = (Pxx - ep - (m.ux * m.ux - m.ux * m.Fx) * e.ieps) * k.Sden;
    m.Syy = (Pyy - ep - (m.uy * m.uy - m.uy * m.Fy) * e.ieps) * k.Sden;
    m.Sxy = (Pxy - (m.ux * m.uy - R(0.5) * (m.ux * m.Fy + m.Fx * m.uy)) * e.ieps) * k.Sden;

    m.gx = (g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7]);   // thermal flux; finished in
    m.gy = (g[2] - g[4]) + (g[5] + g[6]) - (g[7] + g[8]);   // node_gradT
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
    // one reciprocal for both factors: 1 / (a (a - b |u|^2))
    const R d = a - e.bM * uu;
    const R r = rcp(a * d);
    const R c = (e.bM * uN) * (a * r);
    const R ia = d * r;
    m.gx = (Nx + c * m.ux) * ia;
    m.gy = (Ny + c * m.uy) * ia;
}

template <typename R, bool PRE = true>
__device__ __forceinline__ void node_macro_full(const R *f, const R *g, R T0, const Cst<R> &k,
                                                const EpsC<R> &e, Macro<R> &m)
{
    node_macro<R, PRE>(f, g, k, e, m);
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

// Per-node coefficients of the pair updates (collide_pair).
template <typename R> struct PairC {
    R b0;     // even part of f^eq / omega apart from the (c.u)^2 and c.S.c terms
    R k45;    // 4.5 / eps
    R c9;     // 9 (1 - 1/(2 tau_f)) / eps
    R m3b5;   // -3 (1 - 1/(2 tau_f)) (u.F) / eps
    R b1;     // even part of g^eq / omega apart from the (c.u)^2 term
    R T45;    // 4.5 T / eps
    R s;      // T / tau_T + (1 - 1/(2 tau_T)) ((1/eps - 1/sigma) u.grad T + Q / sigma), the
              // coefficient of 3 omega (c.u) in the odd part of g*
};

// BGK collision with forcing and sources, in place (Eqs. LBEeq, FtermF, TEqColli,
// Eq:Tforce):  f* = f - (f - f^eq)/tau_f + F_i,  g* = g - (g - g^eq)/tau_T + P_i + Q_i.
//
// Directions come in opposite pairs (i, i') with c_i' = -c_i and equal weights.  Every
// term splits into a part even in c (f^eq: pressure, u u and S terms; F_i: the (c.u)(c.F)
// and u.F terms; g^eq: sigma T, u u and pressure terms; Q_i: the constant part) and a part
// odd in c (the c.u, c.F, c.grad T, P_i and (c.u) Q terms), so each pair is updated as
//   f*_i = (1 - 1/tau) f_i + E + O,   f*_i' = (1 - 1/tau) f_i' + E - O.
// E collects 1/tau times the even part of the equilibrium plus the even part of the source;
// the terms are grouped around the per-node coefficients q so that a pair costs few
// multiply-adds.
//
// The odd parts carry 3 omega_i (c_i . u) and friends, whose first moment over the lattice
// must be exactly u: 3 omega is taken as w3a (axes) and w3d (diagonals) with
// 2 w3a + 4 w3d = 1 in the arithmetic type, otherwise the rounded weights would scale the
// momentum by a fixed factor every step.
//
// c = class of the pair (0 axes, 1 diagonals); cu = c.u, cF = c.F, cSc = c.S.c,
// cg = c.grad T, cv = c.(T F + eps p grad T / rho0).
template <typename R, bool PRE>
__device__ __forceinline__ void collide_pair(R &fa, R &fb, R &ga, R &gb, int c, R cu, R cF, R cSc, R cg, R cv,
                                             const PairC<R> &q, const Cst<R> &k, R &Ef_sum, R &Eg_sum)
{
    const ClassK<R> d = class_k<PRE>(k, c);
    const R w = d.w, w3 = d.w3, witf = d.witf, witT = d.witT, wQ = d.wQ, bsg = d.bsg;
    const R w3fT = d.w3fT, w3fF = d.w3fF, A15 = node_k<PRE>(k).A15;
    const R cu2 = cu * cu;
    // f: E = omega [(b0 + 4.5 (c.u)^2 / eps + 1.5 A c.S.c) / tau_f + fF (9 (c.u)(c.F) - 3 u.F) / eps],
    //    O = 3 omega [(c.u) / tau_f + fF c.F]
    const R Ee = A15 * cSc + (q.k45 * cu2 + q.b0);
    const R Es = q.c9 * (cu * cF) + q.m3b5;
    const R Ef = witf * Ee + w * Es;
    const R Of = k.itf * (w3 * cu) + w3fF * cF;
    fa = k.of * fa + (Ef + Of);
    fb = k.of * fb + (Ef - Of);

    // g: E = omega [(b1 + 4.5 T (c.u)^2 / eps) / tau_T + fT Q],
    //    O = 3 omega (c.u) s + omega sigma B c.grad T / tau_T + 3 omega fT c.v
    const R Eg = witT * (q.T45 * cu2 + q.b1) + wQ;
    const R Og = (w3 * q.s) * cu + (bsg * cg + w3fT * cv);
    ga = k.og * ga + (Eg + Og);
    gb = k.og * gb + (Eg - Og);
    Ef_sum += Ef;
    Eg_sum += Eg;
}

// The rest direction is updated from the other eight so that the moment identities
// sum_i f^eq_i = rho0, sum_i F_i = 0, sum_i g^eq_i = sigma T and
// sum_i Q_i = (1 - 1/(2 tau_T)) Q (App. A and Sec. 3.2 moment lists) hold in the
// arithmetic itself, not only up to the rounding of the lattice weights: the zeroth
// moments are what a step accumulates, so a rounding bias there would drift the mass
// and the thermal energy.
template <typename R, bool PRE = true>
__device__ __forceinline__ void node_collide(R *f, R *g, const Macro<R> &m, R T0,
                                             const Cst<R> &k, const EpsC<R> &e)
{
    const NodeK<R> n = node_k<PRE>(k);
    const R T = T0 + m.Td;
    const R ep = e.eps * m.p;
    const R uu = m.ux * m.ux + m.uy * m.uy;
    const R trS = m.Sxx + m.Syy;
    const R uF = m.ux * m.Fx + m.uy * m.Fy;
    const R ugT = m.ux * m.gx + m.uy * m.gy;
    const R vx = T * m.Fx + ep * m.gx;   // T F + eps p grad T / rho0
    const R vy = T * m.Fy + ep * m.gy;

    PairC<R> q;
    q.b0 = R(3) * ep - R(1.5) * uu * e.ieps - n.hA * trS;
    q.b1 = k.sig * m.Td - R(1.5) * T * uu * e.ieps + R(3) * T * ep;
    q.k45 = R(4.5) * e.ieps;
    q.c9 = n.c9fF * e.ieps;
    q.m3b5 = R(-3) * (k.fF * uF * e.ieps);
    q.T45 = q.k45 * T;
    q.s = k.itT * T + k.fT * ((e.ieps - k.isig) * ugT + n.Qisig);
    R Ef = R(0), Eg = R(0);
    // (1, 3): c = (1, 0)
    collide_pair<R, PRE>(f[1], f[3], g[1], g[3], 0, m.ux, m.Fx, m.Sxx, m.gx, vx, q, k, Ef, Eg);
    // (2, 4): c = (0, 1)
    collide_pair<R, PRE>(f[2], f[4], g[2], g[4], 0, m.uy, m.Fy, m.Syy, m.gy, vy, q, k, Ef, Eg);
    // (5, 7): c = (1, 1)
    collide_pair<R, PRE>(f[5], f[7], g[5], g[7], 1, m.ux + m.uy, m.Fx + m.Fy, m.Sxx + R(2) * m.Sxy + m.Syy,
                    m.gx + m.gy, vx + vy, q, k, Ef, Eg);
    // (6, 8): c = (-1, 1)
    collide_pair<R, PRE>(f[6], f[8], g[6], g[8], 1, m.uy - m.ux, m.Fy - m.Fx, m.Sxx - R(2) * m.Sxy + m.Syy,
                    m.gy - m.gx, vy - vx, q, k, Ef, Eg);
    // rest direction: f^eq_0 + tau_f F_0 and g^eq_0 + tau_T Q_0 from the zeroth moments
    f[0] = k.of * f[0] - R(2) * Ef;
    g[0] = k.og * g[0] + (n.itTsig * m.Td + n.fTQ) - R(2) * Eg;
}

// ---------------------------------------------------------------------------------
// Grid helpers
// ---------------------------------------------------------------------------------
__device__ __forceinline__ bool on_wall(const KParams &P, int x, int y)
{
    return (!P.px && (x == 0 || x == P.nx - 1)) || (!P.py && (y == 0 || y == P.ny - 1));
}

// Offsets in the tiled layout: element of (q, x, y) = y * row + tile_off(x) + q * T with
// row = ntx * 18 * T and tile_off(x) = (x / T) * 18 * T + x % T (32-bit within a row).
template <int T> __device__ __forceinline__ unsigned tile_off(int x)
{
    const unsigned u = (unsigned)x;
    return (u / T) * (18u * T) + (u % T);
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
    const float inv = P.hinv;
    constexpr int T = TileOf<S>::v;
    // three row bases and three in-row offsets; direction i comes from (x - cx_i, y - cy_i)
    const long long row = (long long)P.ntx * (18 * T);
    const S *r0 = src + (long long)y * row, *rm = src + (long long)ym * row, *rp = src + (long long)yp * row;
    const unsigned o0 = tile_off<T>(x), om = tile_off<T>(xm), op = tile_off<T>(xp);
    const S *b[9] = {r0 + o0, r0 + om, rm + o0, r0 + op, rp + o0, rm + om, rm + op, rp + op, rp + om};
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        f[i] = R(Store<S>::ld(b[i] + i * T, inv));
        g[i] = R(Store<S>::ld(b[i] + (9 + i) * T, inv));
    }
}

template <typename S, typename R>
__device__ __forceinline__ void store_node(S *__restrict__ dst, const KParams &P, int x, int y,
                                           const R *f, const R *g)
{
    constexpr int T = TileOf<S>::v;
    S *b = dst + (long long)y * ((long long)P.ntx * (18 * T)) + tile_off<T>(x);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        Store<S>::st(b + i * T, f[i], P.hscale);
        Store<S>::st(b + (9 + i) * T, g[i], P.hscale);
    }
}

// Arithmetic types per storage type: R for the collision, M for the node moments
// (p, u, S, grad T); the same type in every mode (FP64 for FP64 storage, FP32 for FP32 and
// FP16 storage).  With the moment-preserving weights of node_collide, FP32 arithmetic
// keeps the FP32 path within about 1e-6 of the FP64 result after 1000 steps of the
// 128 x 128 cavity.
template <typename S> struct Prec;
template <> struct Prec<double> { using R = double; using M = double; };
template <> struct Prec<float> { using R = float; using M = float; };
template <> struct Prec<__half> { using R = float; using M = float; };

template <typename A, typename B> struct same_t { static constexpr bool v = false; };
template <typename A> struct same_t<A, A> { static constexpr bool v = true; };

// Moments and collision of one node in R, in place on f, g.
template <typename R, typename M, bool PRE = true>
__device__ __forceinline__ void node_update(R *f, R *g, const KParams &P, int x, int y)
{
    static_assert(same_t<R, M>::v, "moments and collision share the arithmetic type");
    Macro<R> m;
    node_macro_full<R, PRE>(f, g, R(P.T0), cst<R>(P), eps_at<R>(P, x, y), m);
    node_collide<R, PRE>(f, g, m, R(P.T0), cst<R>(P), eps_at<R>(P, x, y));
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
// Thermal condition of a wall node: index of the isothermal wall that applies (-1 if the
// node is on prescribed-gradient walls only).
__device__ __forceinline__ int thermal_dirichlet_wall(const KParams &P, const WallInfo &w)
{
    if (w.xw >= 0 && P.wall_kind[w.xw] == 0) return w.xw;
    if (w.yw >= 0 && P.wall_kind[w.yw] == 0) return w.yw;
    return -1;
}

// Td = T - T0 of node (x, y) from its streamed temperature populations (sigma T = sum g + Q/2).
template <typename S, typename R>
__device__ __forceinline__ R gather_Td(const S *__restrict__ src, const KParams &P, const Cst<R> &k,
                                       int x, int y)
{
    const int xm = (x == 0) ? P.nx - 1 : x - 1;
    const int xp = (x == P.nx - 1) ? 0 : x + 1;
    const int ym = (y == 0) ? P.ny - 1 : y - 1;
    const int yp = (y == P.ny - 1) ? 0 : y + 1;
    const int sx[9] = {x, xm, x, xp, x, xm, xp, xp, xm};
    const int sy[9] = {y, y, ym, y, yp, ym, ym, yp, yp};
    R sg = R(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) sg += R(Store<S>::ld(src + pidx<S>(P, 9 + i, sx[i], sy[i]), P.hinv));
    return (sg + k.halfQ) * k.isig;
}

// Non-equilibrium extrapolation (Sec. 3.4, Eqs. FNEESEQFIN, NEESVel, TeEBounDFEQ,
// TNEESAp, TNEESApGra): pre-collision populations of wall node (x, y) from the streamed
// populations ff, gf of its reference node x_f and, on prescribed-gradient walls, Td of
// the next node x_ff.  f, g may alias ff, gf.  mb receives the node's macroscopic state,
// the one the scheme assigns to x_b: T_b, u_b, p and S of x_f, the boundary grad T, and
// G and F (Eq. ForceEq) at u_b and T_b.  The node collides with that state (wall_collide),
// which gives the post-collision form of the extrapolation,
// f^eq(x_b) + (1 - 1/tau) f^neq(x_f) plus the source terms.
template <typename R, bool PRE = true>
__device__ __forceinline__ void wall_from_ref(const KParams &P, const Cst<R> &k, int x, int y,
                                              const EpsC<R> &ef, const EpsC<R> &eb,
                                              const R *ff, const R *gf, R Tdff, R *f, R *g,
                                              Macro<R> &mb)
{
    const WallInfo w = wall_info(P, x, y);
    Macro<R> mf;
    const R T0 = R(P.T0);
    node_macro_full<R, PRE>(ff, gf, T0, k, ef, mf);
    const R Tf = T0 + mf.Td;
    const R epf = ef.eps * mf.p;

    R ubx = R(0), uby = R(0);
    double ubm = 0.0;              // |u_b|, a constant of the wall
    const int vw = (w.xw >= 0 && w.yw < 0) ? w.xw : (w.yw >= 0 && w.xw < 0) ? w.yw : -1;
    if (vw >= 0) {
        ubx = R(P.wall_ux[vw]);
        uby = R(P.wall_uy[vw]);
        ubm = sqrt(P.wall_ux[vw] * P.wall_ux[vw] + P.wall_uy[vw] * P.wall_uy[vw]);
    }
    const R epb = eb.eps * mf.p;   // eps at the wall node, pressure of x_f

    const int dir = thermal_dirichlet_wall(P, w);
    R Tdb, gbx, gby;
    if (dir >= 0) {
        Tdb = R(P.wall_T[dir] - P.T0);
        gbx = mf.gx;
        gby = mf.gy;
    } else {
        gbx = (w.xw >= 0) ? R(w.dx * P.wall_dTdn[w.xw]) : mf.gx;
        gby = (w.yw >= 0) ? R(w.dy * P.wall_dTdn[w.yw]) : mf.gy;
        Tdb = (R(4) * mf.Td - Tdff - R(2) * (R(w.dx) * gbx + R(w.dy) * gby)) * R(1.0 / 3.0);
    }
    const R Tb = T0 + Tdb;

    // f_i = f_i(x_f) + f^eq_i(x_b) - f^eq_i(x_f), and likewise g, with the equilibria of
    // feq_i and geq_i written as differences: both take the shear rate of x_f, so their
    // shear terms cancel and are not formed.  Per node: the differences of eps p, of
    // |u|^2 / eps, and for g of sigma Td, T |u|^2 / eps and T eps p.
    const R uub = (ubx * ubx + uby * uby) * eb.ieps;
    const R uuf = (mf.ux * mf.ux + mf.uy * mf.uy) * ef.ieps;
    const R dep = epb - epf, duu = uub - uuf;
    const R dsT = k.sig * (Tdb - mf.Td), dTuu = Tb * uub - Tf * uuf, dTep = Tb * epb - Tf * epf;
    const R Tbi = Tb * eb.ieps, Tfi = Tf * ef.ieps;
    f[0] = ff[0] + (R(-5.0 / 3.0) * dep - R(2.0 / 3.0) * duu);
    g[0] = gf[0] + (R(4.0 / 9.0) * dsT - R(2.0 / 3.0) * dTuu - R(5.0 / 3.0) * dTep);
    const R fe = R(3) * dep - R(1.5) * duu;                  // even, direction-independent
    const R ge = dsT - R(1.5) * dTuu + R(3) * dTep;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const R cx = R(CXd[i]), cy = R(CYd[i]), wi = R(Wd(i));
        const R cub = cx * ubx + cy * uby, cuf = cx * mf.ux + cy * mf.uy;
        const R cgb = cx * gbx + cy * gby, cgf = cx * mf.gx + cy * mf.gy;
        f[i] = ff[i] + wi * (fe + R(3) * (cub - cuf) + R(4.5) * (cub * cub * eb.ieps - cuf * cuf * ef.ieps));
        g[i] = gf[i] + wi * (ge + R(3) * (Tb * cub - Tf * cuf) + R(4.5) * (Tbi * cub * cub - Tfi * cuf * cuf)
                             + k.sigB * (cgb - cgf));
    }

    mb.Td = Tdb;
    mb.ux = ubx;
    mb.uy = uby;
    const R dl = eb.dlin + eb.dquad * R(ubm);
    mb.Fx = eb.eps * k.ax - dl * ubx;
    mb.Fy = eb.eps * (k.ay + k.gb * Tdb) - dl * uby;
    mb.p = mf.p;
    mb.Sxx = mf.Sxx;
    mb.Sxy = mf.Sxy;
    mb.Syy = mf.Syy;
    mb.gx = gbx;
    mb.gy = gby;
}

// Collision of wall node (x, y) with the state mb the boundary scheme assigned to it.
template <typename R, bool PRE = true>
__device__ __forceinline__ void wall_collide(R *f, R *g, const Macro<R> &mb, const KParams &P, int x, int y)
{
    node_collide<R, PRE>(f, g, mb, R(P.T0), cst<R>(P), eps_at<R>(P, x, y));
}

// The boundary scheme with the reference nodes' populations gathered from memory.
template <typename S, typename R, bool PRE = true>
__device__ __forceinline__ void wall_populations(const S *__restrict__ src, const KParams &P,
                                                 const Cst<R> &k, int x, int y, R *f, R *g,
                                                 Macro<R> &mb)
{
    const WallInfo w = wall_info(P, x, y);
    R ff[9], gf[9];
    gather<S, R>(src, P, x + w.dx, y + w.dy, ff, gf);
    R Tdff = R(0);
    if (thermal_dirichlet_wall(P, w) < 0) Tdff = gather_Td<S, R>(src, P, k, x + 2 * w.dx, y + 2 * w.dy);
    wall_from_ref<R, PRE>(P, k, x, y, eps_at<R>(P, x + w.dx, y + w.dy), eps_at<R>(P, x, y), ff, gf, Tdff, f, g, mb);
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
