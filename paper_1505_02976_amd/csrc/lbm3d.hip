// Three-dimensional path: the modified lattice-BGK model (Secs. 2-3) on the D3Q19 lattice
// for the flow and the temperature populations, with x, y and z each periodic or bounded by
// walls under the non-equilibrium extrapolation (Sec. 3.4).  One thread per
// node: pull streaming from the previous step's post-collision buffer, the node's
// macroscopic state, BGK collision with forcing and sources, store.  Populations are kept
// as 38 planes [q][z][y][x] (flow 0-18, temperature 19-37) in deviation form (f_0 - rho0,
// g_i - omega_i sigma T0), FP64, FP32 or FP16 (scaled by 256), with arithmetic in the storage
// precision, FP32 for FP16 (the drag solve in FP64).
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>

#include "../../include/lbm3d.h"
#include "lbm_error.h"

namespace lbm3 {

constexpr int NQ = 19;
// rest, the six axis directions, the twelve edge directions; opposite velocities adjacent
__device__ constexpr int CX[NQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
__device__ constexpr int CY[NQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
__device__ constexpr int CZ[NQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
__host__ __device__ constexpr double W(int i) { return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }

// Per-launch constants in the arithmetic type R, computed once on the host (no division or
// conversion of launch constants is left to the node code).
template <typename R> struct C3 {
    R itf, itT, of, og;            // 1 / tau, 1 - 1 / tau
    R fF, fT;                      // 1 - 1 / (2 tau)
    R tfh;                         // tau_f - 1/2
    R sig, isig, Q, halfQ, T0, gb;
    R a[3];
    R Sden;                        // 1 / (cs^2 (A - tau_f))
    R aM0;                         // cs^2 sigma (B - tau_T)
    R sigB3;                       // sigma B / 3 (the gradient term of g^eq per 3 omega)
    R A, A15;                      // A, 1.5 A
    R eps, ieps, dlin, dquad, bM;  // the uniform porosity's coefficients
};

// 1 / tau and 1 - 1 / tau in R with it + o == 1 exactly (o = fl(1 - fl(1 / tau)),
// it = fl(1 - o); for tau > 1/2 one of the two subtractions is exact by Sterbenz's lemma,
// and then so is the other): the collision's o f + it (...) then carries the state's zeroth
// moment with the factor 1, where a rounded pair would scale the temperature deviation by
// up to 1 + 6e-8 per FP32 step.
template <typename R> inline void relax_pair(double tau, R &it, R &o)
{
    const R i0 = R(1.0 / tau);
    o = R(1) - i0;
    it = R(1) - o;
}

// Launch constants (host-computed, passed by value).
struct K3 {
    int nx, ny, nz, px, py, pz;
    long long n;
    double tau_f, tau_T, A, B, sigma, Q, eps, T0, gbeta;
    double a[3];
    double c0, c1, dlin, dquad;      // drag solve: c0, c1; force: eps nu / K, eps F_eps / sqrt(K)
    const double *eps_field;         // porosity per node, or NULL for the uniform eps
    double nuK, isqK, Feps;          // nu / K, 1 / sqrt(K), F_eps (if not from the Ergun relation)
    int ergun;
    double L, dT;                    // characteristic length and temperature difference
    // walls: 0 z = 0, 1 z = nz - 1, 2 x = 0, 3 x = nx - 1, 4 y = 0, 5 y = ny - 1
    int wkind[6];
    double wu[6][3], wT[6], wdTdn[6];
    C3<double> cd;
    C3<float> cf;
};

template <typename R> __device__ __forceinline__ const C3<R> &cst3(const K3 &K);
template <> __device__ __forceinline__ const C3<double> &cst3<double>(const K3 &K) { return K.cd; }
template <> __device__ __forceinline__ const C3<float> &cst3<float>(const K3 &K) { return K.cf; }

// FP64 reciprocal and square root for the drag solve of the FP32 and FP16 paths, whose
// results are rounded to FP32: the hardware estimates refined by Newton steps (relative
// error below 1e-13).  The FP64 path keeps IEEE division and square root.
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ double sqrt_nr(double x)
{
    const double r = __builtin_amdgcn_rsq(x);
    const double s = x * r;
    return x > 0.0 ? fma(fma(-s, s, x), 0.5 * r, s) : 0.0;
}
template <typename R> __device__ __forceinline__ double drag_rcp(double x) { return rcp_nr(x); }
template <> __device__ __forceinline__ double drag_rcp<double>(double x) { return 1.0 / x; }
template <typename R> __device__ __forceinline__ double drag_sqrt(double x) { return sqrt_nr(x); }
template <> __device__ __forceinline__ double drag_sqrt<double>(double x) { return sqrt(x); }

// The walls node (x, y, z) lies on: zw in {-1, 0, 1}, xw in {-1, 2, 3}, yw in {-1, 4, 5}.
__device__ __forceinline__ void wall_of(const K3 &K, int x, int y, int z, int &xw, int &yw, int &zw)
{
    xw = K.px ? -1 : (x == 0 ? 2 : (x == K.nx - 1 ? 3 : -1));
    yw = K.py ? -1 : (y == 0 ? 4 : (y == K.ny - 1 ? 5 : -1));
    zw = K.pz ? -1 : (z == 0 ? 0 : (z == K.nz - 1 ? 1 : -1));
}

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Porosity-dependent coefficients of one node (Sec. 2, Eq. ForceEq; Sec. 3.1 drag solve; b of
// Eq. MatrM), in R; c0 and c1 of the drag solve in FP64.
template <typename R> struct Por {
    R eps, ieps, dlin, dquad, bM;
    double c0, c1;
};

template <typename R> __device__ __forceinline__ Por<R> por_of(const K3 &K, size_t k)
{
    Por<R> e;
    if (!K.eps_field) {
        const C3<R> &c = cst3<R>(K);
        e.eps = c.eps; e.ieps = c.ieps; e.dlin = c.dlin; e.dquad = c.dquad; e.bM = c.bM;
        e.c0 = K.c0; e.c1 = K.c1;
    } else {
        const double eps = K.eps_field[k];
        const double Feps = K.ergun ? 1.75 / sqrt(150.0 * eps * eps * eps) : K.Feps;
        const double ie = 1.0 / eps;
        e.eps = R(eps);
        e.ieps = R(ie);
        e.c0 = 0.5 * (1.0 + eps * 0.5 * K.nuK);
        e.c1 = eps * 0.5 * Feps * K.isqK;
        e.dlin = R(eps * K.nuK);
        e.dquad = R(eps * Feps * K.isqK);
        e.bM = R(0.5 * (ie - K.cd.isig));   // isig = 1 / sigma, rounded once on the host
    }
    return e;
}

// Arithmetic type of a storage type: FP64 storage computes in FP64, FP32 storage in FP32
// (the drag solve in FP64 for both).  The flow populations are handled as deviations
// throughout: the rest state is f_0 = rho0 and f_i = 0 otherwise, so the moments the node
// needs (sum over i > 0, first and second moments) involve only small values, and f_0
// enters as f_0 - rho0.
template <typename S> struct Arith;
template <> struct Arith<double> { using R = double; };
template <> struct Arith<float> { using R = float; };
template <> struct Arith<__half> { using R = float; };

// Load and store of one stored deviation.  FP16 holds 256 times the deviation: the
// deviations are small, and the scale keeps them clear of FP16's subnormal range.  Stores
// are non-temporal: the next step reads them from HBM, not from this launch's caches.
template <typename S> struct St3 {
    template <typename R> static __device__ __forceinline__ R ld(const S *p) { return R(*p); }
    template <typename R> static __device__ __forceinline__ void st(S *p, R v) { __builtin_nontemporal_store(S(v), p); }
};
template <> struct St3<__half> {
    template <typename R> static __device__ __forceinline__ R ld(const __half *p)
    {
        return R(__half2float(*p) * (1.0f / 256.0f));
    }
    template <typename R> static __device__ __forceinline__ void st(__half *p, R v)
    {
        __builtin_nontemporal_store(__half_as_ushort(__float2half(float(v) * 256.0f)),
                                    reinterpret_cast<unsigned short *>(p));
    }
};

// Pre-collision populations of node (x, y, z) pulled from the post-collision buffer, in the
// deviation form they are stored in (f_0 - rho0, g_q - omega_q sigma T0).  The source node of
// direction q is (x - c_q) with periodic wrap (a walled direction never leaves the grid:
// only nodes off its walls are pulled).  Offsets within a plane of populations are 32-bit
// (the host keeps a plane below 2^31 nodes), so each load adds one offset to the plane's
// base address.
template <typename S, typename R>
__device__ __forceinline__ void pull(const S *__restrict__ src, const K3 &K, int x, int y, int z, R *f, R *g)
{
    // source column, row and plane offsets for c = 0, +1 (from x - 1) and -1 (from x + 1)
    const unsigned nx = (unsigned)K.nx, pl = (unsigned)K.nx * (unsigned)K.ny;
    const unsigned xo[3] = {(unsigned)x, (unsigned)wrap(x - 1, K.nx), (unsigned)wrap(x + 1, K.nx)};
    const unsigned yo[3] = {(unsigned)y * nx, (unsigned)wrap(y - 1, K.ny) * nx, (unsigned)wrap(y + 1, K.ny) * nx};
    const unsigned zo[3] = {(unsigned)z * pl, (unsigned)wrap(z - 1, K.nz) * pl, (unsigned)wrap(z + 1, K.nz) * pl};
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int ix = CX[q] == 0 ? 0 : (CX[q] > 0 ? 1 : 2);
        const int iy = CY[q] == 0 ? 0 : (CY[q] > 0 ? 1 : 2);
        const int iz = CZ[q] == 0 ? 0 : (CZ[q] > 0 ? 1 : 2);
        const unsigned k = zo[iz] + yo[iy] + xo[ix];
        f[q] = St3<S>::template ld<R>(src + (size_t)q * K.n + k);
        g[q] = St3<S>::template ld<R>(src + (size_t)(NQ + q) * K.n + k);
    }
}

// G and F (Eq. ForceEq) at velocity u and temperature T = T0 + Td.
template <typename R>
__device__ __forceinline__ void force(const K3 &K, const Por<R> &e, const R *u, R Td, R *F)
{
    const C3<R> &c = cst3<R>(K);
    const R um = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const R dl = e.dlin + e.dquad * um;
    F[0] = e.eps * c.a[0] - dl * u[0];
    F[1] = e.eps * c.a[1] - dl * u[1];
    F[2] = e.eps * (c.a[2] + c.gb * Td) - dl * u[2];
}

// Macroscopic state; Td = T - T0; S as xx, xy, xz, yy, yz, zz.
template <typename R> struct Mac {
    R Td, T, u[3], F[3], p, S[6], gT[3];
};

// Contractions with the lattice velocities over their nonzero components only.  D3Q19 has
// no velocity component other than 0 and +-1, and q is a compile-time constant once the
// loops over directions are unrolled, so the selections fold away and no multiplication by
// 0 or 1 is left (which IEEE arithmetic would otherwise have to carry out).
// c_q . v
template <typename R> __device__ __forceinline__ R cdot(int q, const R *v)
{
    const int c[3] = {CX[q], CY[q], CZ[q]};
    R r = R(0);
    bool any = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (c[a] == 0) continue;
        const R t = c[a] > 0 ? v[a] : -v[a];
        r = any ? r + t : t;
        any = true;
    }
    return r;
}
// c_q . S . c_q for the symmetric S stored as xx, xy, xz, yy, yz, zz
template <typename R> __device__ __forceinline__ R cScq(int q, const R *S)
{
    const int c[3] = {CX[q], CY[q], CZ[q]};
    constexpr int ix[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    R r = R(0);
    bool any = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (c[a] == 0) continue;
        r = any ? r + S[ix[a][a]] : S[ix[a][a]];
        any = true;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = a + 1; b < 3; ++b) {
            if (c[a] == 0 || c[b] == 0) continue;
            const R t = R(2) * S[ix[a][b]];
            r = c[a] * c[b] > 0 ? r + t : r - t;
        }
    return r;
}
// acc += c_q,a v (the a-th component of c_q v), only where c_q,a is not zero
template <typename R> __device__ __forceinline__ void cacc(int cq, R &acc, R v)
{
    if (cq > 0) acc += v;
    else if (cq < 0) acc -= v;
}

// State of an interior node from its populations: T (Sec. 3.2), v and u (drag solve in
// FP64, Sec. 3.1), F, p (Sec. 3.1 with omega_0 = 1/3 in the closed forms of App. A), S from
// the non-equilibrium second moment (Eq. ShearEqCom; the D3Q19 equilibrium's second moment
// is eps p I + u u / eps), grad T = <M>^-1 <N> by the Sherman-Morrison form of
// <M> = a I - b u u.  Directions come in opposite pairs (q, q + 1), q odd: the first
// moments take the pair's difference, the second moments its sum.
template <typename R>
__device__ __forceinline__ void macro3(const R *f, const R *g, const K3 &K, const Por<R> &e, Mac<R> &m)
{
    R sg = g[0], s18 = R(0), j[3] = {R(0), R(0), R(0)}, P[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    R h[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int q = 1; q < NQ; q += 2) {
        const R sf = f[q] + f[q + 1], df = f[q] - f[q + 1];
        const R dg = g[q] - g[q + 1];
        sg += g[q] + g[q + 1];
        s18 += sf;
        cacc(CX[q], j[0], df); cacc(CY[q], j[1], df); cacc(CZ[q], j[2], df);
        cacc(CX[q], h[0], dg); cacc(CY[q], h[1], dg); cacc(CZ[q], h[2], dg);
        cacc(CX[q] * CX[q], P[0], sf); cacc(CX[q] * CY[q], P[1], sf); cacc(CX[q] * CZ[q], P[2], sf);
        cacc(CY[q] * CY[q], P[3], sf); cacc(CY[q] * CZ[q], P[4], sf); cacc(CZ[q] * CZ[q], P[5], sf);
    }
    const C3<R> &c = cst3<R>(K);
    const R eps = e.eps, ieps = e.ieps, isig = c.isig, Q = c.Q;
    m.Td = (sg + c.halfQ) * isig;      // sigma T = sum g + Q/2, the rest state sigma T0 taken out
    m.T = c.T0 + m.Td;
    const R G[3] = {c.a[0], c.a[1], c.a[2] + c.gb * m.Td};
    double v[3];
    for (int a = 0; a < 3; ++a) v[a] = double(j[a] + R(0.5) * eps * G[a]);
    const double vm = drag_sqrt<R>(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    const double iden = drag_rcp<R>(e.c0 + drag_sqrt<R>(e.c0 * e.c0 + e.c1 * vm));
    for (int a = 0; a < 3; ++a) m.u[a] = R(v[a] * iden);
    force<R>(K, e, m.u, m.Td, m.F);
    const R uu = m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2];
    const R uF = m.u[0] * m.F[0] + m.u[1] * m.F[1] + m.u[2] * m.F[2];
    // rho0 s_0 = -omega_0 |u|^2 / (2 eps cs^2) = -|u|^2 / (2 eps); tau_f F_0 = -tau_f (1 - 1/(2 tau_f)) u.F / eps
    const R s0 = R(-0.5) * uu * ieps, tF0 = -c.tfh * uF * ieps;
    m.p = R(0.5) * ieps * (s18 + tF0 + s0);            // cs^2 / (eps (1 - omega_0)) = 1 / (2 eps)
    const R ep = eps * m.p;
    const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        const R neq = P[t] - (ia[t] == ib[t] ? ep : R(0)) - m.u[ia[t]] * m.u[ib[t]] * ieps;
        m.S[t] = (neq + R(0.5) * (m.u[ia[t]] * m.F[ib[t]] + m.F[ia[t]] * m.u[ib[t]]) * ieps) * c.Sden;
    }
    R N[3];
    for (int a = 0; a < 3; ++a) N[a] = h[a] - m.T * m.u[a] + R(0.5) * (m.T * m.F[a] + m.u[a] * Q * isig);
    const R am = c.aM0 - R(0.5) * ep;
    const R bm = e.bM;
    const R uN = m.u[0] * N[0] + m.u[1] * N[1] + m.u[2] * N[2];
    const R sm = bm * uN / (am - bm * uu);
    const R iam = R(1) / am;
    for (int a = 0; a < 3; ++a) m.gT[a] = (N[a] + sm * m.u[a]) * iam;
}

// 3 omega_q for an axis and an edge direction with 2 w3a + 8 w3e = 1 exactly in R: the
// first moment of every term 3 omega_q (c_q . v) is then exactly v in the arithmetic
// itself (sum over the lattice of omega c c = cs^2 I), not only up to the rounding of the
// weights, which would scale the momentum and the heat flux by a fixed factor every step.
template <typename R> __device__ __forceinline__ R w3e() { return R(1.0 / 12.0); }
template <typename R> __device__ __forceinline__ R w3a() { return (R(1) - R(8) * w3e<R>()) * R(0.5); }
template <typename R> __device__ __forceinline__ R w3(int q) { return q < 7 ? w3a<R>() : w3e<R>(); }

// Equilibria (Eqs. EQFIN, EQTSHIN, TeEDFEQ) of direction q for pressure term ep = eps p;
// the flow equilibrium as a deviation (f_0^eq - rho0 for q = 0).  Used by the boundary
// scheme and the initialisation; the collision below evaluates the same terms pairwise.
template <typename R>
__device__ __forceinline__ R feq(int q, const K3 &K, const Por<R> &e, R ep, const R *u, const R *S)
{
    const R w = R(W(q));
    const R cu = cdot<R>(q, u);
    const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const R cSc = cScq<R>(q, S);
    const R trS = S[0] + S[3] + S[5];
    const R base = q == 0 ? R(-2) * ep : R(3) * w * ep;      // -(1 - omega_0) eps p / cs^2; omega_q eps p / cs^2
    return base + (q == 0 ? R(0) : w3<R>(q) * cu) + w * R(4.5) * (cu * cu - uu * R(1.0 / 3.0)) * e.ieps
         + w * cst3<R>(K).A15 * (cSc - trS * R(1.0 / 3.0));
}

// The temperature equilibrium as a deviation, g^eq_q - omega_q sigma T0, for T = T0 + Td.
template <typename R>
__device__ __forceinline__ R geq(int q, const K3 &K, const Por<R> &e, R Td, R T, R ep, const R *u, const R *gT)
{
    const R w = R(W(q));
    const R cu = cdot<R>(q, u);
    const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const R cg = cdot<R>(q, gT);
    const R pres = q == 0 ? R(-2) * T * ep : R(3) * w * T * ep;   // varpi_q T eps p / (cs^2 rho0)
    return w * (cst3<R>(K).sig * Td + T * R(4.5) * (cu * cu - uu * R(1.0 / 3.0)) * e.ieps) + pres
         + (q == 0 ? R(0) : w3<R>(q) * (T * cu + cst3<R>(K).sigB3 * cg));
}

// BGK collision with forcing and sources (Eqs. LBEeq, FtermF, TEqColli, Eq:Tforce),
//   f* = f - (f - f^eq) / tau_f + F_q,   g* = g - (g - g^eq) / tau_T + P_q + Q_q.
// Opposite directions (q, q + 1) are updated together from the parts of every term that are
// even and odd in c (as in two dimensions):
//   f*_q = (1 - 1/tau_f) f_q + Ae + Ao,   f*_q+1 = (1 - 1/tau_f) f_q+1 + Ae - Ao,
// Ae = omega [(b0 + 4.5 (c.u)^2 / eps + 1.5 A c.S.c) / tau_f + fF (9 (c.u)(c.F) - 3 u.F) / eps],
// Ao = 3 omega [(c.u) / tau_f + fF c.F], and for the temperature
// Ge = omega [(b1 + 4.5 T (c.u)^2 / eps) / tau_T + fT Q] (b1 with sigma (T - T0): the
// populations are deviations from omega sigma T0),
// Go = 3 omega [s (c.u) + sigma B c.grad T / (3 tau_T) + fT c.(T F + eps p grad T / rho0)].
// The rest direction takes what the other 18 leave of the zeroth moments the moment lists
// fix (App. A; Sec. 3.2): sum_q (f^eq_q / tau_f + F_q) = rho0 / tau_f and
// sum_q (g^eq_q / tau_T + P_q + Q_q) = sigma T / tau_T + (1 - 1/(2 tau_T)) Q, i.e. 0 and
// sigma (T - T0) / tau_T + (1 - 1/(2 tau_T)) Q for the deviations, so that mass and thermal
// energy are conserved by the arithmetic, not only up to the rounding of the lattice
// weights (in FP32 that rounding biases the heat balance by about 1e-8 sigma T / tau_T per
// step).
template <typename R>
__device__ __forceinline__ void collide(R *f, R *g, const Mac<R> &m, const K3 &K, const Por<R> &e)
{
    const C3<R> &c = cst3<R>(K);
    const R ep = e.eps * m.p, ieps = e.ieps;
    const R uu = m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2];
    const R uF = m.u[0] * m.F[0] + m.u[1] * m.F[1] + m.u[2] * m.F[2];
    const R ugT = m.u[0] * m.gT[0] + m.u[1] * m.gT[1] + m.u[2] * m.gT[2];
    const R trS = m.S[0] + m.S[3] + m.S[5];
    const R V[3] = {m.T * m.F[0] + ep * m.gT[0], m.T * m.F[1] + ep * m.gT[1], m.T * m.F[2] + ep * m.gT[2]};
    // per-node coefficients
    const R b0 = R(3) * ep - R(1.5) * uu * ieps - R(0.5) * c.A * trS;
    const R k45 = R(4.5) * ieps, c9 = R(9) * c.fF * ieps, m3b5 = R(-3) * (c.fF * uF * ieps);
    const R b1 = c.sig * m.Td - R(1.5) * m.T * uu * ieps + R(3) * m.T * ep;
    const R T45 = k45 * m.T;
    const R sc = c.itT * m.T + c.fT * ((ieps - c.isig) * ugT + c.Q * c.isig);
    const R bsg = c.itT * c.sigB3;
    R Ef = R(0), Eg = R(0);
#pragma unroll
    for (int q = 1; q < NQ; q += 2) {
        const R w = R(W(q)), w3q = w3<R>(q);
        const R cu = cdot<R>(q, m.u), cF = cdot<R>(q, m.F), cV = cdot<R>(q, V), cg = cdot<R>(q, m.gT);
        const R cSc = cScq<R>(q, m.S), cu2 = cu * cu;
        const R Ae = w * (c.itf * (c.A15 * cSc + (k45 * cu2 + b0)) + (c9 * (cu * cF) + m3b5));
        const R Ao = w3q * (c.itf * cu + c.fF * cF);
        const R Ge = w * (c.itT * (T45 * cu2 + b1) + c.fT * c.Q);
        const R Go = w3q * (sc * cu + (bsg * cg + c.fT * cV));
        f[q] = c.of * f[q] + (Ae + Ao);
        f[q + 1] = c.of * f[q + 1] + (Ae - Ao);
        g[q] = c.og * g[q] + (Ge + Go);
        g[q + 1] = c.og * g[q + 1] + (Ge - Go);
        Ef += Ae;
        Eg += Ge;
    }
    f[0] = c.of * f[0] - R(2) * Ef;
    g[0] = c.og * g[0] + (c.sig * m.Td * c.itT + c.fT * c.Q - R(2) * Eg);
}

// Pre-collision populations and state of node (x, y, z).  Interior: pulled populations
// and their moments.  Wall node: the non-equilibrium extrapolation from the next node
// inward x_f (and T of x_ff on prescribed-gradient walls), whose state is the one the
// scheme assigns (T_b, u_b, p and S of x_f, the boundary grad T).  On an edge or a vertex
// where two or three walls meet, x_f is the inward diagonal neighbour, the wall is at rest,
// an isothermal wall's temperature wins over a prescribed gradient (among isothermal walls
// x first, then y, then z), and each prescribed gradient sets its own normal component of
// grad T, as at the corners in two dimensions.
template <typename S, typename R, bool WALLS = true>
__device__ __forceinline__ void node_state(const S *__restrict__ src, const K3 &K, int x, int y, int z,
                                           R *f, R *g, Mac<R> &m, Por<R> &e)
{
    const size_t plane = (size_t)K.nx * K.ny, k = (size_t)z * plane + (size_t)y * K.nx + x;
    e = por_of<R>(K, k);
    int xw = -1, yw = -1, zw = -1;
    if (WALLS) wall_of(K, x, y, z, xw, yw, zw);
    if (xw < 0 && yw < 0 && zw < 0) {
        pull<S, R>(src, K, x, y, z, f, g);
        macro3<R>(f, g, K, e, m);
        return;
    }
    const int dx = xw == 2 ? 1 : (xw == 3 ? -1 : 0), dz = zw == 0 ? 1 : (zw == 1 ? -1 : 0);
    const int dy = yw == 4 ? 1 : (yw == 5 ? -1 : 0);
    R ff[NQ], gf[NQ];
    pull<S, R>(src, K, x + dx, y + dy, z + dz, ff, gf);
    const Por<R> ef = por_of<R>(K, (size_t)((long long)k + dz * (long long)plane + dy * (long long)K.nx + dx));
    Mac<R> mf;
    macro3<R>(ff, gf, K, ef, mf);
    R Tdb, gb[3] = {mf.gT[0], mf.gT[1], mf.gT[2]};
    const int iso = (xw >= 0 && K.wkind[xw] == 0) ? xw
                  : ((yw >= 0 && K.wkind[yw] == 0) ? yw : ((zw >= 0 && K.wkind[zw] == 0) ? zw : -1));
    if (iso >= 0) {
        Tdb = R(K.wT[iso] - K.T0);
    } else {
        R f2[NQ], g2[NQ];
        pull<S, R>(src, K, x + 2 * dx, y + 2 * dy, z + 2 * dz, f2, g2);
        R sg = R(0);
#pragma unroll
        for (int q = 0; q < NQ; ++q) sg += g2[q];
        const R Tdff = (sg + cst3<R>(K).halfQ) * cst3<R>(K).isig;
        if (xw >= 0) gb[0] = R(dx * K.wdTdn[xw]);
        if (yw >= 0) gb[1] = R(dy * K.wdTdn[yw]);
        if (zw >= 0) gb[2] = R(dz * K.wdTdn[zw]);
        Tdb = (R(4) * mf.Td - Tdff - R(2) * (R(dx) * gb[0] + R(dy) * gb[1] + R(dz) * gb[2])) * R(1.0 / 3.0);
    }
    m.Td = Tdb;
    m.T = cst3<R>(K).T0 + Tdb;
    const int nwall = (xw >= 0) + (yw >= 0) + (zw >= 0);
    const int wu = nwall > 1 ? -1 : (xw >= 0 ? xw : (yw >= 0 ? yw : zw));   // an edge or a vertex is at rest
    for (int a = 0; a < 3; ++a) { m.u[a] = wu < 0 ? R(0) : R(K.wu[wu][a]); m.gT[a] = gb[a]; }
    force<R>(K, e, m.u, m.Td, m.F);
    m.p = mf.p;
    for (int c = 0; c < 6; ++c) m.S[c] = mf.S[c];
    const R epb = e.eps * mf.p, epf = ef.eps * mf.p;   // the wall node's porosity, x_f's pressure
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        f[q] = feq<R>(q, K, e, epb, m.u, mf.S) + (ff[q] - feq<R>(q, K, ef, epf, mf.u, mf.S));
        g[q] = geq<R>(q, K, e, m.Td, m.T, epb, m.u, gb) + (gf[q] - geq<R>(q, K, ef, mf.Td, mf.T, epf, mf.u, mf.gT));
    }
}

__device__ __forceinline__ bool node_xyz(const K3 &K, int &x, int &y, int &z)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K.n) return false;
    x = (int)(k % K.nx);
    y = (int)((k / K.nx) % K.ny);
    z = (int)(k / ((long long)K.nx * K.ny));
    return true;
}

// Post-collision populations (deviations) into the buffer.
template <typename S, typename R>
__device__ __forceinline__ void store(S *__restrict__ dst, const K3 &K, unsigned k, const R *f, const R *g)
{
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        St3<S>::template st<R>(dst + (size_t)q * K.n + k, f[q]);
        St3<S>::template st<R>(dst + (size_t)(NQ + q) * K.n + k, g[q]);
    }
}

constexpr int B3 = 256;

// Extent of the interior along x and z: all nodes of a periodic direction, all but the two
// wall nodes of a walled one.
__host__ __device__ __forceinline__ int inner_x(const K3 &K) { return K.px ? K.nx : K.nx - 2; }
__host__ __device__ __forceinline__ int inner_y(const K3 &K) { return K.py ? K.ny : K.ny - 2; }
__host__ __device__ __forceinline__ int inner_z(const K3 &K) { return K.pz ? K.nz : K.nz - 2; }

// One time step, pull, state, collide, store, in one launch: its first blocks take the
// wall nodes (boundary scheme), the remaining ones the interior nodes (no boundary-scheme
// code).  Run side by side, the short wall blocks no longer add a launch of their own to
// every step.
// Interior node i of interior plane `plane` (32-bit index arithmetic: planes and the grid
// stay below 2^31 nodes, checked on the host).
template <typename S>
__device__ __forceinline__ void k3_interior_node(const S *__restrict__ src, S *__restrict__ dst, const K3 &K,
                                                 unsigned i, int plane)
{
    using R = typename Arith<S>::R;
    const unsigned nxi = (unsigned)inner_x(K), nyi = (unsigned)inner_y(K);
    if (i >= nxi * nyi) return;
    const unsigned yi = i / nxi;
    const int x = (int)(i - yi * nxi) + (K.px ? 0 : 1), y = (int)yi + (K.py ? 0 : 1);
    const int z = plane + (K.pz ? 0 : 1);
    const unsigned k = ((unsigned)z * (unsigned)K.ny + (unsigned)y) * (unsigned)K.nx + (unsigned)x;
    R f[NQ], g[NQ];
    Mac<R> m;
    Por<R> e;
    node_state<S, R, false>(src, K, x, y, z, f, g, m, e);
    collide<R>(f, g, m, K, e);
    store<S, R>(dst, K, k, f, g);
}

// Wall node i: the z wall planes first, then the x wall planes less their z rows, then the
// y wall planes less both.
template <typename S>
__device__ __forceinline__ void k3_wall_node(const S *__restrict__ src, S *__restrict__ dst, const K3 &K,
                                             long long i)
{
    using R = typename Arith<S>::R;
    const long long plane = (long long)K.nx * K.ny, zn = K.pz ? 0 : 2 * plane;
    const long long xside = K.px ? 0 : (long long)K.ny * inner_z(K);
    const long long yside = K.py ? 0 : (long long)inner_x(K) * inner_z(K);
    if (i >= zn + 2 * xside + 2 * yside) return;
    int x, y, z;
    if (i < zn) {
        const long long k = i < plane ? i : (long long)(K.nz - 1) * plane + (i - plane);
        x = (int)(k % K.nx); y = (int)((k / K.nx) % K.ny); z = (int)(k / plane);
    } else if (i < zn + 2 * xside) {
        const long long j = i - zn, r = j % xside;
        x = j < xside ? 0 : K.nx - 1;
        y = (int)(r % K.ny);
        z = (int)(r / K.ny) + (K.pz ? 0 : 1);
    } else {
        const long long j = i - zn - 2 * xside, r = j % yside;
        const int nxi = inner_x(K);
        y = j < yside ? 0 : K.ny - 1;
        x = (int)(r % nxi) + (K.px ? 0 : 1);
        z = (int)(r / nxi) + (K.pz ? 0 : 1);
    }
    const long long k = ((long long)z * K.ny + y) * K.nx + x;
    R f[NQ], g[NQ];
    Mac<R> m;
    Por<R> e;
    node_state<S, R>(src, K, x, y, z, f, g, m, e);
    collide<R>(f, g, m, K, e);
    store<S, R>(dst, K, (unsigned)k, f, g);
}

// Blocks [0, nbw): wall nodes; then nbx blocks per interior plane.  Registers held to the
// interior's own count (FP32/FP16 five waves per SIMD, FP64 three); the wall blocks, 2 %
// of the nodes, absorb any spill.
template <typename S>
__global__ void __launch_bounds__(B3, sizeof(S) == 8 ? 3 : 5)
k3_step(const S *__restrict__ src, S *__restrict__ dst, K3 K, unsigned nbw, unsigned nbx)
{
    const unsigned b = blockIdx.x;
    if (b < nbw) {
        k3_wall_node<S>(src, dst, K, (long long)b * B3 + threadIdx.x);
        return;
    }
    const unsigned bi = b - nbw, plane = bi / nbx, bx = bi - plane * nbx;
    k3_interior_node<S>(src, dst, K, bx * B3 + threadIdx.x, (int)plane);
}

// Initial post-collision populations: the equilibria of the initial fields (S = 0,
// grad T = 0, p = 0), computed in FP64.
template <typename S>
__global__ void __launch_bounds__(B3) k3_init(S *__restrict__ dst, K3 K, const double *T_init, const double *u_init)
{
    int x, y, z;
    if (!node_xyz(K, x, y, z)) return;
    const size_t k = ((size_t)z * K.ny + y) * K.nx + x;
    double T = K.T0;
    int xw, yw, zw;
    wall_of(K, x, y, z, xw, yw, zw);
    if (T_init) T = T_init[k];
    else if (xw >= 0 && K.wkind[xw] == 0) T = K.wT[xw];
    else if (yw >= 0 && K.wkind[yw] == 0) T = K.wT[yw];
    else if (zw >= 0 && K.wkind[zw] == 0) T = K.wT[zw];
    double u[3] = {0.0, 0.0, 0.0};
    if (u_init)
        for (int a = 0; a < 3; ++a) u[a] = u_init[(size_t)a * K.n + k];
    const double S0[6] = {0, 0, 0, 0, 0, 0}, g0[3] = {0, 0, 0};
    const Por<double> e = por_of<double>(K, k);
    double f[NQ], g[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        f[q] = feq<double>(q, K, e, 0.0, u, S0);
        g[q] = geq<double>(q, K, e, T - K.T0, T, 0.0, u, g0);
    }
    store<S, double>(dst, K, (unsigned)k, f, g);
}

// Average Nusselt number of wall w (0: z = 0, 1: z = nz - 1, 2: x = 0, 3: x = nx - 1,
// 4: y = 0, 5: y = ny - 1): -L dT/dn / dT (n = +z, +x or +y along the wall's axis) by the
// one-sided second-order difference at each wall node, averaged over the wall plane, as in
// two dimensions (Eq. AvNuss): a plain mean along each periodic in-plane direction, the
// trapezoid rule along each walled one.  One block; every thread sums a fixed strided subset
// in order, then a fixed-order tree: FP64 results do not depend on the launch.
template <typename S>
__global__ void __launch_bounds__(256) k3_nusselt(const S *__restrict__ src, K3 K, int w, double *out)
{
    using R = typename Arith<S>::R;
    __shared__ double part[256];
    const int ax = w < 2 ? 2 : (w < 4 ? 0 : 1), hi = w & 1;          // normal axis, far wall
    // the in-plane axes: the first is y for x walls and x otherwise, the second y for z walls
    // and z otherwise (selected explicitly, so nothing is indexed at run time)
    const int na = ax == 0 ? K.nx : (ax == 1 ? K.ny : K.nz);
    const int n0 = ax == 0 ? K.ny : K.nx, p0 = ax == 0 ? K.py : K.px;
    const int n1 = ax == 2 ? K.ny : K.nz, p1 = ax == 2 ? K.py : K.pz;
    const long long cells = (long long)n0 * n1;
    double acc = 0.0;
    for (long long c = threadIdx.x; c < cells; c += 256) {
        const int i0 = (int)(c % n0), i1 = (int)(c / n0);
        double T[3];
        for (int d = 0; d < 3; ++d) {
            const int ia = hi ? na - 1 - d : d;
            const int x = ax == 0 ? ia : i0;
            const int y = ax == 1 ? ia : (ax == 0 ? i0 : i1);
            const int z = ax == 2 ? ia : i1;
            R f[NQ], g[NQ];
            Mac<R> m;
            Por<R> p;
            node_state<S, R>(src, K, x, y, z, f, g, m, p);
            T[d] = double(m.T);
        }
        const double d1 = (-3.0 * T[0] + 4.0 * T[1] - T[2]) / 2.0;   // along the inward normal
        double wt = 1.0;
        if (!p0 && (i0 == 0 || i0 == n0 - 1)) wt *= 0.5;
        if (!p1 && (i1 == 0 || i1 == n1 - 1)) wt *= 0.5;
        acc += wt * (-K.L * (hi ? -d1 : d1) / K.dT);
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *out = part[0] / (double(p0 ? n0 : n0 - 1) * double(p1 ? n1 : n1 - 1));
}

struct FieldOut3 { double *p, *u, *T, *S, *gT; };

template <typename S>
__global__ void __launch_bounds__(B3) k3_fields(const S *__restrict__ src, K3 K, FieldOut3 o)
{
    using R = typename Arith<S>::R;
    int x, y, z;
    if (!node_xyz(K, x, y, z)) return;
    R f[NQ], g[NQ];
    Mac<R> m;
    Por<R> e;
    node_state<S, R>(src, K, x, y, z, f, g, m, e);
    const size_t k = ((size_t)z * K.ny + y) * K.nx + x, n = (size_t)K.n;
    if (o.p) o.p[k] = double(m.p);
    if (o.T) o.T[k] = double(m.T);
    for (int a = 0; a < 3; ++a) {
        if (o.u) o.u[a * n + k] = double(m.u[a]);
        if (o.gT) o.gT[a * n + k] = double(m.gT[a]);
    }
    if (o.S)
        for (int c = 0; c < 6; ++c) o.S[c * n + k] = double(m.S[c]);
}

// Pre-collision populations with the rest state added back (f_0 + rho0).
template <typename S>
__global__ void __launch_bounds__(B3) k3_populations(const S *__restrict__ src, K3 K, double *fo, double *go)
{
    using R = typename Arith<S>::R;
    int x, y, z;
    if (!node_xyz(K, x, y, z)) return;
    R f[NQ], g[NQ];
    Mac<R> m;
    Por<R> e;
    node_state<S, R>(src, K, x, y, z, f, g, m, e);
    const size_t k = ((size_t)z * K.ny + y) * K.nx + x;
    for (int q = 0; q < NQ; ++q) {
        if (fo) fo[(size_t)q * K.n + k] = double(f[q]) + (q == 0 ? 1.0 : 0.0);
        if (go) go[(size_t)q * K.n + k] = double(g[q]) + W(q) * K.sigma * K.T0;
    }
}

}  // namespace lbm3

using namespace lbm3;

struct lbm3_ctx {
    K3 K;
    int storage;
    char *buf[2];
    double *result;
    int cur;
    hipStream_t stream;
    int64_t t;
};

namespace {

lbm_status fail3(lbm_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
lbm_status fail3(lbm_status st, const char *fmt, ...)
{
    char msg[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(msg, sizeof(msg), fmt, ap);
    va_end(ap);
    return lbm::set_error(st, msg);
}

size_t elem3(int storage) { return storage == LBM_F64 ? 8 : (storage == LBM_F32 ? 4 : 2); }

// Calls f with a tag naming the storage type of a context.
template <typename S> struct Tag { using type = S; };
template <typename F> void by_storage(int storage, F &&f)
{
    if (storage == LBM_F64) f(Tag<double>{});
    else if (storage == LBM_F32) f(Tag<float>{});
    else f(Tag<__half>{});
}

size_t buffer_bytes(const lbm3_params *p)
{
    const size_t n = (size_t)p->nx * p->ny * p->nz;
    return (2 * NQ * n * elem3(p->storage) + 255) / 256 * 256;
}

constexpr size_t RESULT_BYTES = 256;   // after the two buffers: the reduction's result

// Derived lattice constants, as for two dimensions (Sec. 2, Sec. 3.1, Eq. Therdiff,
// Eq. EQA&B, Eq. ForceEq with the Ergun relation).
lbm_status make_constants(const lbm3_params *p, K3 &K)
{
    if (!p) return fail3(LBM_ERR_INVALID, "params is NULL");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail3(LBM_ERR_INVALID, "grid must be at least 1 x 1 x 1");
    if (!p->periodic_z && p->nz < 4) return fail3(LBM_ERR_INVALID, "walled z needs nz >= 4 (got %d)", p->nz);
    if (!p->periodic_x && p->nx < 4) return fail3(LBM_ERR_INVALID, "walled x needs nx >= 4 (got %d)", p->nx);
    if (!p->periodic_y && p->ny < 4) return fail3(LBM_ERR_INVALID, "walled y needs ny >= 4 (got %d)", p->ny);
    if (p->storage != LBM_F64 && p->storage != LBM_F32 && p->storage != LBM_F16)
        return fail3(LBM_ERR_INVALID, "storage must be LBM_F64, LBM_F32 or LBM_F16");
    if ((double)p->nx * p->ny * p->nz >= 2147483648.0 || (p->periodic_z ? p->nz : p->nz - 2) > 65535)
        return fail3(LBM_ERR_INVALID, "grid too large (at most 2^31 - 1 nodes and 65535 interior z planes)");
    if (!(p->tau_f > 0.5) || !(p->tau_T > 0.5)) return fail3(LBM_ERR_INVALID, "tau_f and tau_T must exceed 1/2");
    if (!(p->eps > 0.0) || !(p->eps <= 1.0) || !(p->sigma > 0.0) || !(p->J > 0.0))
        return fail3(LBM_ERR_INVALID, "eps must lie in (0, 1]; sigma and J must be positive");
    if (p->eps_field && ((uintptr_t)p->eps_field) % 8)
        return fail3(LBM_ERR_INVALID, "eps_field must be 8-byte aligned");
    const double L = p->L > 0 ? p->L : (!p->periodic_x ? p->nx - 1 : (p->periodic_z ? p->nz : p->nz - 1));
    double A = p->A, B = p->B;
    if (std::isnan(A) || std::isnan(B)) {
        if (!(p->Ra > 0) || !(p->Pr > 0)) return fail3(LBM_ERR_INVALID, "A, B from Ma need Ra > 0 and Pr > 0");
        A = p->tau_f - 0.5 - p->J * p->Ma * L * sqrt(3.0 * p->Pr / p->Ra);
        B = p->tau_T - 0.5 - (p->Ma / p->sigma) * L * sqrt(3.0 / (p->Pr * p->Ra));
    }
    const double nu_e = (p->tau_f - A - 0.5) / 3.0, nu = nu_e / p->J;
    const double alpha = p->sigma * (p->tau_T - B - 0.5) / 3.0;
    const double Kp = p->Da * L * L;
    if (!(nu_e > 0)) return fail3(LBM_ERR_INVALID, "nu_e <= 0 (A = %g >= tau_f - 1/2)", A);
    if (!(alpha > 0)) return fail3(LBM_ERR_INVALID, "alpha_e <= 0 (B = %g >= tau_T - 1/2)", B);
    if (!(Kp > 0)) return fail3(LBM_ERR_INVALID, "K = Da L^2 must be positive");
    const double dT = p->T_hot - p->T_cold;
    const double Feps = std::isnan(p->F_eps) ? 1.75 / sqrt(150.0 * p->eps * p->eps * p->eps) : p->F_eps;
    K.nx = p->nx; K.ny = p->ny; K.nz = p->nz; K.px = p->periodic_x ? 1 : 0; K.py = p->periodic_y ? 1 : 0; K.pz = p->periodic_z ? 1 : 0;
    K.n = (long long)p->nx * p->ny * p->nz;
    K.tau_f = p->tau_f; K.tau_T = p->tau_T; K.A = A; K.B = B; K.sigma = p->sigma; K.Q = p->Q; K.eps = p->eps;
    K.T0 = 0.5 * (p->T_hot + p->T_cold);
    K.gbeta = (p->Ra > 0 && dT != 0.0) ? p->Ra * nu * alpha / (dT * L * L * L) : 0.0;
    for (int a = 0; a < 3; ++a) K.a[a] = p->a[a];
    K.c0 = 0.5 * (1.0 + p->eps * 0.5 * nu / Kp);
    K.c1 = p->eps * 0.5 * Feps / sqrt(Kp);
    K.dlin = p->eps * nu / Kp;
    K.dquad = p->eps * Feps / sqrt(Kp);
    K.eps_field = p->eps_field;
    K.L = L;
    K.dT = dT;
    K.nuK = nu / Kp;
    K.isqK = 1.0 / sqrt(Kp);
    K.ergun = std::isnan(p->F_eps) ? 1 : 0;
    K.Feps = K.ergun ? 0.0 : p->F_eps;
    C3<double> &c = K.cd;
    relax_pair(p->tau_f, c.itf, c.of);
    relax_pair(p->tau_T, c.itT, c.og);
    c.fF = 1.0 - 0.5 / p->tau_f;
    c.fT = 1.0 - 0.5 / p->tau_T;
    c.tfh = p->tau_f - 0.5;
    c.sig = p->sigma;
    c.isig = 1.0 / p->sigma;
    c.Q = p->Q;
    c.halfQ = 0.5 * p->Q;
    c.T0 = K.T0;
    c.gb = K.gbeta;
    for (int a = 0; a < 3; ++a) c.a[a] = p->a[a];
    c.Sden = 3.0 / (A - p->tau_f);
    c.aM0 = p->sigma * (B - p->tau_T) / 3.0;
    c.sigB3 = p->sigma * B / 3.0;
    c.A = A;
    c.A15 = 1.5 * A;
    c.eps = p->eps;
    c.ieps = 1.0 / p->eps;
    c.dlin = K.dlin;
    c.dquad = K.dquad;
    c.bM = 0.5 * (1.0 / p->eps - 1.0 / p->sigma);
    C3<float> &cf = K.cf;
    relax_pair(p->tau_f, cf.itf, cf.of);
    relax_pair(p->tau_T, cf.itT, cf.og);
    cf.fF = (float)c.fF; cf.fT = (float)c.fT; cf.tfh = (float)c.tfh; cf.sig = (float)c.sig;
    cf.isig = (float)c.isig; cf.Q = (float)c.Q; cf.halfQ = (float)c.halfQ; cf.T0 = (float)c.T0;
    cf.gb = (float)c.gb;
    for (int a = 0; a < 3; ++a) cf.a[a] = (float)c.a[a];
    cf.Sden = (float)c.Sden; cf.aM0 = (float)c.aM0; cf.sigB3 = (float)c.sigB3; cf.A = (float)c.A; cf.A15 = (float)c.A15;
    cf.eps = (float)c.eps; cf.ieps = (float)c.ieps; cf.dlin = (float)c.dlin; cf.dquad = (float)c.dquad;
    cf.bM = (float)c.bM;
    for (int w = 0; w < 6; ++w) {
        K.wkind[w] = p->wall[w].t_kind == LBM_T_NEUMANN ? 1 : 0;
        for (int a = 0; a < 3; ++a) K.wu[w][a] = p->wall[w].u[a];
        K.wT[w] = p->wall[w].T;
        K.wdTdn[w] = p->wall[w].dTdn;
    }
    return LBM_OK;
}

unsigned blocks_for(long long n) { return (unsigned)((n + B3 - 1) / B3); }

lbm_status launched(const char *what)
{
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LBM_OK : fail3(LBM_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

extern "C" {

size_t lbm3_workspace_bytes(const lbm3_params *params)
{
    K3 K;
    if (make_constants(params, K) != LBM_OK) return 0;
    return 2 * buffer_bytes(params) + RESULT_BYTES;
}

lbm_status lbm3_init(const lbm3_params *params, void *workspace, size_t workspace_bytes, void *hip_stream,
                     lbm3_ctx **out)
{
    if (!out) return fail3(LBM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    K3 K;
    lbm_status st = make_constants(params, K);
    if (st != LBM_OK) return st;
    if (!workspace || ((uintptr_t)workspace) % 256) return fail3(LBM_ERR_INVALID, "workspace must be non-NULL and 256-byte aligned");
    const size_t need = 2 * buffer_bytes(params) + RESULT_BYTES;
    if (workspace_bytes < need) return fail3(LBM_ERR_INVALID, "workspace too small: %zu < %zu bytes", workspace_bytes, need);
    lbm3_ctx *c = new (std::nothrow) lbm3_ctx;
    if (!c) return fail3(LBM_ERR_DEVICE, "out of host memory");
    c->K = K;
    c->storage = params->storage;
    c->buf[0] = static_cast<char *>(workspace);
    c->buf[1] = c->buf[0] + buffer_bytes(params);
    c->result = reinterpret_cast<double *>(c->buf[1] + buffer_bytes(params));
    c->cur = 0;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->t = 0;
    by_storage(c->storage, [&](auto t) {
        using S = typename decltype(t)::type;
        hipLaunchKernelGGL((k3_init<S>), dim3(blocks_for(K.n)), dim3(B3), 0, c->stream,
                           reinterpret_cast<S *>(c->buf[0]), K, params->T_init, params->u_init);
    });
    st = launched("initial populations");
    if (st == LBM_OK) {
        const hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) st = fail3(LBM_ERR_DEVICE, "initial populations: %s", hipGetErrorString(e));
    }
    if (st != LBM_OK) { delete c; return st; }
    *out = c;
    return LBM_OK;
}

lbm_status lbm3_step(lbm3_ctx *c, int64_t nsteps)
{
    if (!c) return fail3(LBM_ERR_INVALID, "ctx is NULL");
    if (nsteps < 0) return fail3(LBM_ERR_INVALID, "nsteps must be >= 0");
    const K3 &K = c->K;
    const long long n_plane = (long long)inner_x(K) * inner_y(K), n_w = K.n - n_plane * inner_z(K);
    const unsigned nbx = n_plane > 0 ? blocks_for(n_plane) : 0, nbw = blocks_for(n_w);
    const long long nb = (long long)nbw + (long long)nbx * (n_plane > 0 ? inner_z(K) : 0);
    if (nb > 0x7fffffff) return fail3(LBM_ERR_INVALID, "grid too large for one launch");
    for (int64_t s = 0; s < nsteps; ++s) {
        by_storage(c->storage, [&](auto t) {
            using S = typename decltype(t)::type;
            const S *src = reinterpret_cast<const S *>(c->buf[c->cur]);
            S *dst = reinterpret_cast<S *>(c->buf[c->cur ^ 1]);
            if (nb > 0)
                hipLaunchKernelGGL((k3_step<S>), dim3((unsigned)nb), dim3(B3), 0, c->stream, src, dst, c->K, nbw,
                                   nbx > 0 ? nbx : 1u);
        });
        c->cur ^= 1;
        c->t += 1;
    }
    return launched("3-D step");
}

lbm_status lbm3_fields(lbm3_ctx *c, double *p, double *u, double *T, double *S, double *gradT)
{
    if (!c) return fail3(LBM_ERR_INVALID, "ctx is NULL");
    const FieldOut3 o{p, u, T, S, gradT};
    by_storage(c->storage, [&](auto t) {
        using S = typename decltype(t)::type;
        hipLaunchKernelGGL((k3_fields<S>), dim3(blocks_for(c->K.n)), dim3(B3), 0, c->stream,
                           reinterpret_cast<const S *>(c->buf[c->cur]), c->K, o);
    });
    return launched("3-D fields");
}

lbm_status lbm3_populations(lbm3_ctx *c, double *f, double *g)
{
    if (!c) return fail3(LBM_ERR_INVALID, "ctx is NULL");
    by_storage(c->storage, [&](auto t) {
        using S = typename decltype(t)::type;
        hipLaunchKernelGGL((k3_populations<S>), dim3(blocks_for(c->K.n)), dim3(B3), 0, c->stream,
                           reinterpret_cast<const S *>(c->buf[c->cur]), c->K, f, g);
    });
    return launched("3-D populations");
}

lbm_status lbm3_nusselt(lbm3_ctx *c, int32_t wall, double *nu_host)
{
    if (!c || !nu_host) return fail3(LBM_ERR_INVALID, "ctx and nu_host must be non-NULL");
    if (wall < 0 || wall > 5)
        return fail3(LBM_ERR_INVALID, "wall must be 0 (z = 0), 1 (z = nz - 1), 2 (x = 0), 3 (x = nx - 1), 4 (y = 0) or 5 (y = ny - 1)");
    if (wall < 2 ? c->K.pz : (wall < 4 ? c->K.px : c->K.py))
        return fail3(LBM_ERR_INVALID, "wall %d does not exist (periodic direction)", (int)wall);
    if (!(c->K.dT != 0.0)) return fail3(LBM_ERR_INVALID, "T_hot - T_cold is zero");
    by_storage(c->storage, [&](auto t) {
        using S = typename decltype(t)::type;
        hipLaunchKernelGGL((k3_nusselt<S>), dim3(1), dim3(256), 0, c->stream,
                           reinterpret_cast<const S *>(c->buf[c->cur]), c->K, (int)wall, c->result);
    });
    lbm_status st = launched("3-D Nusselt number");
    if (st != LBM_OK) return st;
    hipError_t e = hipMemcpyAsync(nu_host, c->result, sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail3(LBM_ERR_DEVICE, "3-D Nusselt number: %s", hipGetErrorString(e));
    return LBM_OK;
}

int32_t lbm3_lattice(int32_t *c)
{
    static const int32_t v[NQ][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
                                     {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1}, {-1, 0, -1},
                                     {1, 0, -1}, {-1, 0, 1}, {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    if (c) memcpy(c, v, sizeof(v));
    return NQ;
}

int64_t lbm3_time(const lbm3_ctx *c) { return c ? c->t : -1; }

void lbm3_destroy(lbm3_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    delete c;
}

}  // extern "C"
