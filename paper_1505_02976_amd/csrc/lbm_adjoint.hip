// Discrete adjoint of the fused step: vector-Jacobian products of one time step for the
// gradient of an average Nusselt number with respect to the porosity of every node.
//
// One step maps the post-collision state s_t to s_{t+1}: node x gathers its pre-collision
// populations pre(x) (streaming; at wall nodes the boundary scheme builds them from the
// reference node x_f and, on prescribed-gradient walls, T at x_ff) and collides them,
// s_{t+1}(x) = C_x(pre(x), eps(x)).  Given lambda_{t+1} = dJ/ds_{t+1} the adjoint step
//   1. evaluates mu(x) = (dC_x/dpre)^T lambda_{t+1}(x) and (dC_x/deps)^T lambda_{t+1}(x) at
//      every node; at wall nodes the derivatives are taken through the boundary scheme,
//      with respect to the reference node's populations, T(x_ff), eps(x_b) and eps(x_f);
//   2. transposes streaming: lambda_t(y, q) is the adjoint of the pre-collision population
//      that s_t(y, q) becomes at y + c_q, i.e. mu(y + c_q, q) plus the contributions of the
//      wall nodes that use y + c_q as their reference node (0 where y + c_q is a wall node
//      or off the grid).  The node kernels scatter mu(z, q) to lambda_t(z - c_q, q); a last
//      kernel adds the wall-reference terms near the walls.
// Off the walls, step 1 is a hand-written reverse-mode product in the storage's arithmetic
// type (node_vjp); at the wall nodes the Jacobian columns come from forward-mode dual
// numbers pushed through the same templated boundary-scheme code as the forward step, one
// column per input.
#include "lbm_kernels.h"

namespace lbm {

constexpr int ADJ_B = 128;
constexpr int ADJ_WB = 64;       // threads per block of the wall-node launch (one pass per wavefront)

__device__ __forceinline__ Cst<Dual> dual_cst(const Cst<double> &c)
{
    Cst<Dual> d;
    d.itf = Dual(c.itf); d.itT = Dual(c.itT); d.of = Dual(c.of); d.og = Dual(c.og);
    d.fF = Dual(c.fF); d.fT = Dual(c.fT); d.tau_f = Dual(c.tau_f); d.A = Dual(c.A);
    d.sigB = Dual(c.sigB); d.sig = Dual(c.sig); d.isig = Dual(c.isig); d.Q = Dual(c.Q);
    d.halfQ = Dual(c.halfQ); d.gb = Dual(c.gb); d.ax = Dual(c.ax); d.ay = Dual(c.ay);
    d.Sden = Dual(c.Sden); d.aM0 = Dual(c.aM0); d.w1 = Dual(c.w1); d.w5 = Dual(c.w5);
    d.w3a = Dual(c.w3a); d.w3d = Dual(c.w3d);
    derive_consts(d);   // products of constants: the FP64 values, derivative 0
    return d;
}

__device__ __forceinline__ void dual_update(Dual *f, Dual *g, const KParams &P, const Cst<Dual> &k,
                                            const EpsC<Dual> &e)
{
    Macro<Dual> m;
    node_macro_full<Dual>(f, g, Dual(P.T0), k, e, m);
    node_collide<Dual>(f, g, m, Dual(P.T0), k, e);
}

// Reverse mode (vector-Jacobian product) of the update of a node off the walls, in the
// arithmetic type R of the storage (FP64 for FP64 storage, FP32 for FP32 and FP16), the
// drag solve in FP64 as in the forward step.  The update is
//   f*_i = (1 - 1/tau_f) f_i + Phi_i(M(f, g), eps),   g*_i = (1 - 1/tau_T) g_i + Psi_i(M, eps),
// with M the moments the node state is built from (sum g, first moments of f and g, the
// sum over i > 0 of f, the second moments of f) and Phi, Psi the equilibrium, forcing and
// source parts of the collision (Eqs. LBEeq, FtermF, TEqColli, Eq:Tforce) of the state of
// Secs. 3.1-3.3 (drag solve, pressure, S, grad T).  Given the adjoints lf, lg of the
// post-collision populations, this returns mf_i = d(lf.f* + lg.g*)/df_i, mg_i, and the
// derivative with respect to the node's porosity.  The forward state is recomputed here
// (same formulas as node_macro, node_gradT and node_collide), then every step is reversed
// in the opposite order; opposite directions (i, i') are reversed together, as the
// collision pairs them.
template <typename R>
__device__ __forceinline__ void node_vjp(const R *f, const R *g, double eps_d, const KParams &P, const R *lf,
                                         const R *lg, R *mf, R *mg, double &geps)
{
    const Cst<R> &k = cst<R>(P);
    const EpsC<R> e = eps_coeffs<R>(P, eps_d);
    // porosity derivatives of the coefficients (Sec. 2: F_eps from the Ergun relation or fixed)
    const double Fe = P.ergun ? 1.75 / sqrt(150.0 * eps_d * eps_d * eps_d) : P.Feps;
    const double dEF = P.ergun ? -0.5 * Fe : Fe;              // d(eps F_eps) / d eps
    // ---- forward ----
    const R sg = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
    const R Td = (sg + k.halfQ) * k.isig;
    const R Gx = k.ax, Gy = k.ay + k.gb * Td;
    const R jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    const R jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
    const double vx = double(jx) + 0.5 * eps_d * double(Gx);
    const double vy = double(jy) + 0.5 * eps_d * double(Gy);
    const double vm = sqrt(vx * vx + vy * vy);
    const double c0 = e.c0, c1 = e.c1;
    const double Rt = sqrt(c0 * c0 + c1 * vm);
    const double iden = 1.0 / (c0 + Rt);
    const R ux = R(vx * iden), uy = R(vy * iden), um = R(vm * iden);
    const R eps = e.eps, ieps = e.ieps;
    const R dl = e.dlin + e.dquad * um;
    const R Fx = eps * Gx - dl * ux, Fy = eps * Gy - dl * uy;
    const R uu = ux * ux + uy * uy, uF = ux * Fx + uy * Fy;
    const R s18 = ((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8]));
    const R cuu = R(-2.0 / 3.0) * ieps, cuF = R(-4.0 / 3.0) * k.fF * k.tau_f * ieps;
    const R X = s18 + cuu * uu + cuF * uF;
    const R p = (R(0.6) * ieps) * X;
    const R ep = eps * p;
    const R qxx = ux * ux - ux * Fx, qyy = uy * uy - uy * Fy, qxy = ux * uy - R(0.5) * (ux * Fy + Fx * uy);
    const R hx = (g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7]);
    const R hy = (g[2] - g[4]) + (g[5] + g[6]) - (g[7] + g[8]);
    const R T = R(P.T0) + Td;
    const R Nx = hx - T * ux + R(0.5) * (T * Fx + ux * k.Q * k.isig);
    const R Ny = hy - T * uy + R(0.5) * (T * Fy + uy * k.Q * k.isig);
    const R a = k.aM0 - R(0.5) * ep;
    const R bM = e.bM;
    const R uN = ux * Nx + uy * Ny;
    const R d = a - bM * uu;
    const R cc = bM * uN / d;
    const R ia = R(1) / a;
    const R gx = (Nx + cc * ux) * ia, gy = (Ny + cc * uy) * ia;
    // collision coefficients (node_collide; the collision is linear in S, whose value the
    // reverse pass does not need)
    const R ugT = ux * gx + uy * gy;
    const R k45 = R(4.5) * ieps, c9 = R(9) * k.fF * ieps;
    const R T45 = k45 * T;
    const R sco = k.itT * T + k.fT * ((ieps - k.isig) * ugT + k.Q * k.isig);

    // ---- reverse ----
    // linear part
#pragma unroll
    for (int i = 0; i < 9; ++i) { mf[i] = k.of * lf[i]; mg[i] = k.og * lg[i]; }
    R a_Td = lg[0] * k.itT * k.sig;
    R a_ux = R(0), a_uy = R(0), a_Fx = R(0), a_Fy = R(0), a_Sxx = R(0), a_Syy = R(0), a_Sxy = R(0);
    R a_gx = R(0), a_gy = R(0), a_vx = R(0), a_vy = R(0);
    R A_k45 = R(0), A_b0 = R(0), A_c9 = R(0), A_m3b5 = R(0), A_T45 = R(0), A_b1 = R(0), A_s = R(0);
    // the four pairs (a, b) with c_b = -c_a: (1,3) (1,0); (2,4) (0,1); (5,7) (1,1); (6,8) (-1,1)
    const int pa[4] = {1, 2, 5, 6}, pb[4] = {3, 4, 7, 8};
    const int pcx[4] = {1, 0, 1, -1}, pcy[4] = {0, 1, 1, 1};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const R cx = R(pcx[t]), cy = R(pcy[t]);
        const R w = t < 2 ? k.w1 : k.w5, w3 = t < 2 ? k.w3a : k.w3d;
        const R sf = lf[pa[t]] + lf[pb[t]] - R(2) * lf[0], df = lf[pa[t]] - lf[pb[t]];
        const R sgm = lg[pa[t]] + lg[pb[t]] - R(2) * lg[0], dg = lg[pa[t]] - lg[pb[t]];
        const R cu = cx * ux + cy * uy, cF = cx * Fx + cy * Fy;
        const R witf = w * k.itf, witT = w * k.itT;
        const R a_cSc = sf * witf * (R(1.5) * k.A);
        const R a_cu = sf * (witf * k45 * R(2) * cu + w * c9 * cF) + df * k.itf * w3
                     + sgm * witT * T45 * R(2) * cu + dg * w3 * sco;
        const R a_cF = sf * w * c9 * cu + df * w3 * k.fF;
        const R a_cg = dg * k.itT * w * k.sigB;
        const R a_cv = dg * w3 * k.fT;
        A_k45 += sf * witf * cu * cu;
        A_b0 += sf * witf;
        A_c9 += sf * w * cu * cF;
        A_m3b5 += sf * w;
        A_T45 += sgm * witT * cu * cu;
        A_b1 += sgm * witT;
        A_s += dg * w3 * cu;
        a_ux += cx * a_cu; a_uy += cy * a_cu;
        a_Fx += cx * a_cF; a_Fy += cy * a_cF;
        a_Sxx += cx * cx * a_cSc; a_Syy += cy * cy * a_cSc; a_Sxy += R(2) * cx * cy * a_cSc;
        a_gx += cx * a_cg; a_gy += cy * a_cg;
        a_vx += cx * a_cv; a_vy += cy * a_cv;
    }
    // per-node coefficients: b0 = 3 ep - 1.5 uu / eps - A trS / 2,
    // b1 = sigma Td - 1.5 T uu / eps + 3 T ep, k45, c9, m3b5 = -3 fF uF / eps, T45, s
    R a_ep = R(3) * A_b0 + R(3) * T * A_b1;
    R a_uu = R(-1.5) * ieps * A_b0 - R(1.5) * T * ieps * A_b1;
    R a_ieps = R(-1.5) * uu * A_b0 - R(1.5) * T * uu * A_b1 + R(4.5) * A_k45 + R(9) * k.fF * A_c9
             - R(3) * k.fF * uF * A_m3b5 + R(4.5) * T * A_T45 + k.fT * ugT * A_s;
    a_Sxx += R(-0.5) * k.A * A_b0;
    a_Syy += R(-0.5) * k.A * A_b0;
    a_Td += k.sig * A_b1;
    R a_T = (R(-1.5) * uu * ieps + R(3) * ep) * A_b1 + k45 * A_T45 + k.itT * A_s;
    R a_uF = R(-3) * k.fF * ieps * A_m3b5;
    const R a_ugT = k.fT * (ieps - k.isig) * A_s;
    // v = T F + eps p grad T
    a_T += Fx * a_vx + Fy * a_vy;
    a_Fx += T * a_vx; a_Fy += T * a_vy;
    a_ep += gx * a_vx + gy * a_vy;
    a_gx += ep * a_vx; a_gy += ep * a_vy;
    // u . grad T
    a_ux += gx * a_ugT; a_uy += gy * a_ugT;
    a_gx += ux * a_ugT; a_gy += uy * a_ugT;
    // grad T = (N + c u) / a, c = b (u . N) / d, d = a - b |u|^2, a = aM0 - eps p / 2
    R a_Nx = a_gx * ia, a_Ny = a_gy * ia;
    const R a_c = (a_gx * ux + a_gy * uy) * ia;
    a_ux += cc * a_gx * ia; a_uy += cc * a_gy * ia;
    R a_a = -(gx * a_gx + gy * a_gy) * ia;
    R a_bM = a_c * uN / d;
    const R a_uN = a_c * bM / d;
    const R a_d = -a_c * cc / d;
    a_a += a_d;
    a_bM += -uu * a_d;
    a_uu += -bM * a_d;
    a_ux += Nx * a_uN; a_uy += Ny * a_uN;
    a_Nx += ux * a_uN; a_Ny += uy * a_uN;
    a_ep += R(-0.5) * a_a;
    // N = h - T u + (T F + u Q / sigma) / 2
    const R a_hx = a_Nx, a_hy = a_Ny;
    a_T += (R(0.5) * Fx - ux) * a_Nx + (R(0.5) * Fy - uy) * a_Ny;
    a_ux += (R(0.5) * k.Q * k.isig - T) * a_Nx;
    a_uy += (R(0.5) * k.Q * k.isig - T) * a_Ny;
    a_Fx += R(0.5) * T * a_Nx; a_Fy += R(0.5) * T * a_Ny;
    a_Td += a_T;
    a_ieps += R(0.5) * a_bM;                           // b = (1/eps - 1/sigma) / 2
    // S (Eq. ShearEqCom)
    const R a_Pxx = k.Sden * a_Sxx, a_Pyy = k.Sden * a_Syy, a_Pxy = k.Sden * a_Sxy;
    a_ep += -k.Sden * (a_Sxx + a_Syy);
    a_ieps += -k.Sden * (qxx * a_Sxx + qyy * a_Syy + qxy * a_Sxy);
    const R sx = -ieps * k.Sden;
    a_ux += sx * ((R(2) * ux - Fx) * a_Sxx + (uy - R(0.5) * Fy) * a_Sxy);
    a_uy += sx * ((R(2) * uy - Fy) * a_Syy + (ux - R(0.5) * Fx) * a_Sxy);
    a_Fx += -sx * (ux * a_Sxx + R(0.5) * uy * a_Sxy);
    a_Fy += -sx * (uy * a_Syy + R(0.5) * ux * a_Sxy);
    // ep = eps p
    R a_p = eps * a_ep;
    double a_eps = double(p * a_ep);
    // p = 0.6 X / eps, X = s18 - (2/3) uu / eps - (4/3) fF tau_f uF / eps
    const R a_X = R(0.6) * ieps * a_p;
    a_ieps += R(0.6) * X * a_p + a_X * (R(-2.0 / 3.0) * uu + R(-4.0 / 3.0) * k.fF * k.tau_f * uF);
    const R a_s18 = a_X;
    a_uu += cuu * a_X;
    a_uF += cuF * a_X;
    a_ux += R(2) * ux * a_uu + Fx * a_uF;
    a_uy += R(2) * uy * a_uu + Fy * a_uF;
    a_Fx += ux * a_uF;
    a_Fy += uy * a_uF;
    // F = eps G - (dlin + dquad |u|) u (Eq. ForceEq)
    a_eps += double(Gx * a_Fx + Gy * a_Fy);
    R a_Gy = eps * a_Fy;
    const R a_dl = -(ux * a_Fx + uy * a_Fy);
    a_ux += -dl * a_Fx; a_uy += -dl * a_Fy;
    const double a_um = double(e.dquad * a_dl);
    a_eps += double(a_dl) * (P.nu_over_K + double(um) * dEF * P.inv_sqrtK);
    // u = v / (c0 + sqrt(c0^2 + c1 |v|)) in FP64 (Sec. 3.1)
    double a_vxd = iden * double(a_ux), a_vyd = iden * double(a_uy), a_vm = iden * a_um;
    const double a_iden = vx * double(a_ux) + vy * double(a_uy) + vm * a_um;
    const double a_den = -iden * iden * a_iden;
    const double a_c0 = a_den * (1.0 + c0 / Rt), a_c1 = a_den * vm / (2.0 * Rt);
    a_vm += a_den * c1 / (2.0 * Rt);
    if (vm > 0.0) { a_vxd += vx / vm * a_vm; a_vyd += vy / vm * a_vm; }   // |v| has derivative 0 at v = 0
    a_eps += 0.25 * P.nu_over_K * a_c0 + 0.5 * P.inv_sqrtK * dEF * a_c1;
    // v = j + eps G / 2
    a_eps += 0.5 * (double(Gx) * a_vxd + double(Gy) * a_vyd);
    a_Gy += R(0.5 * eps_d * a_vyd);
    const R a_jx = R(a_vxd), a_jy = R(a_vyd);
    a_Td += k.gb * a_Gy;
    a_eps += -double(ieps) * double(ieps) * double(a_ieps);
    // moments back to the populations
    const R a_sg = k.isig * a_Td;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const R cx = R(CXd[i]), cy = R(CYd[i]);
        mf[i] += cx * a_jx + cy * a_jy + cx * cx * a_Pxx + cy * cy * a_Pyy + cx * cy * a_Pxy + (i ? a_s18 : R(0));
        mg[i] += a_sg + cx * a_hx + cy * a_hy;
    }
    geps = a_eps;
}

// Steps 1 and 2 at the nodes z off the walls: mu(z) = (dC_z/dpre)^T lambda_{t+1}(z) and the
// porosity derivative by the reverse-mode product above, one thread per node; streaming is
// transposed by scattering, lambda_t(z - c_q, q) = mu(z, q) (each entry has exactly one
// source node z; the wall nodes' part and the wall-reference sums follow in adj_wall_node and
// k_adj_fix).  n: the node.
template <typename S>
__device__ __forceinline__ void adj_interior_node(const S *__restrict__ src, const KParams &P, const AdjBufs &A,
                                                  long long n)
{
    using R = typename Prec<S>::R;
    const long long N = (long long)P.nx * P.ny;
    if (n >= N) return;
    const int x = int(n % P.nx), y = int(n / P.nx);
    if (on_wall(P, x, y)) return;
    R pre[18], lam[18], mu[18];
#pragma unroll
    for (int q = 0; q < 18; ++q) lam[q] = R(A.lam_next[q * N + n]);
    gather<S, R>(src, P, x, y, pre, pre + 9);
    double geps;
    node_vjp<R>(pre, pre + 9, eps_value(P, x, y), P, lam, lam + 9, mu, mu + 9, geps);
    // off the walls x -+ 1 and y -+ 1 stay on the grid except across a periodic edge
    const int xm = x == 0 ? P.nx - 1 : x - 1, xp = x == P.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? P.ny - 1 : y - 1, yp = y == P.ny - 1 ? 0 : y + 1;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int sx = CXd[i] > 0 ? xm : (CXd[i] < 0 ? xp : x);
        const int sy = CYd[i] > 0 ? ym : (CYd[i] < 0 ? yp : y);
        const long long m = (long long)sy * P.nx + sx;
        A.lam[i * N + m] = double(mu[i]);
        A.lam[(9 + i) * N + m] = double(mu[9 + i]);
    }
    A.grad[n] += geps;
}

// Step 1 at the wall nodes (slot s of wall_slot).  A wall node's update depends on its
// reference node's pulled populations ff, gf in two ways only: directly (the boundary
// scheme adds ff - f^eq(x_f) and gf - g^eq(x_f), which the collision scales by
// 1 - 1/tau), and through the nine moments the reference node's state is built from
// (sum_{i>0} f, j, Pxx, Pyy, Pxy of f; sum g and the first moment of g).  Its Jacobian is
// therefore taken by forward-mode dual numbers along nine population directions e_k with
// unit moment k (and zero other moments), plus T(x_ff), eps(x_b) and eps(x_f): 12 passes of
// the same templated boundary-scheme code as the forward step, column j = k for wall slot
// s.  wf[k] receives the adjoint a_k of moment k (the pass's product with lambda
// less its direct part); k_adj_fix rebuilds the adjoint of each reference population from
// them (wall_ref_mu).  Every output has one writer.
constexpr int ADJ_WCOLS = 12;
// e_k over the nine directions (c_0..c_8 as in D2Q9): moments sum_{i>0} f, jx, jy, Pxx,
// Pyy, Pxy of f; then sum g, hx, hy of g
__device__ constexpr double ADJ_EK[9][9] = {
    {0, 0.5, 0.5, 0.5, 0.5, -0.25, -0.25, -0.25, -0.25},   // sum_{i>0} f
    {0, 0.5, 0, -0.5, 0, 0, 0, 0, 0},                      // jx
    {0, 0, 0.5, 0, -0.5, 0, 0, 0, 0},                      // jy
    {0, 0, -0.5, 0, -0.5, 0.25, 0.25, 0.25, 0.25},         // Pxx
    {0, -0.5, 0, -0.5, 0, 0.25, 0.25, 0.25, 0.25},         // Pyy
    {0, 0, 0, 0, 0, 0.25, -0.25, 0.25, -0.25},             // Pxy
    {1, 0, 0, 0, 0, 0, 0, 0, 0},                           // sum g
    {0, 0.5, 0, -0.5, 0, 0, 0, 0, 0},                      // hx
    {0, 0, 0.5, 0, -0.5, 0, 0, 0, 0},                      // hy
};

template <typename S>
__device__ __forceinline__ void adj_wall_node(const S *__restrict__ src, const KParams &P, const AdjBufs &A, int s,
                                              int j)
{
    const long long N = (long long)P.nx * P.ny;
    int x, y;
    if (s >= P.nwall || !wall_slot(P, s, x, y)) return;
    const long long n = (long long)y * P.nx + x;
    double lam[18];
#pragma unroll
    for (int q = 0; q < 18; ++q) lam[q] = A.lam_next[q * N + n];
    const Cst<Dual> k = dual_cst(P.cd);
    const WallInfo w = wall_info(P, x, y);
    const int xf = x + w.dx, yf = y + w.dy;
    double pre[18];
    gather<S, double>(src, P, xf, yf, pre, pre + 9);
    const bool neumann = thermal_dirichlet_wall(P, w) < 0;
    const double Tdff = neumann ? gather_Td<S, double>(src, P, P.cd, x + 2 * w.dx, y + 2 * w.dy) : 0.0;
    const double eb = eps_value(P, x, y), ef = eps_value(P, xf, yf);
    Dual ff[9], gf[9], f[9], g[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        ff[i] = Dual(pre[i], j < 6 ? ADJ_EK[j][i] : 0.0);
        gf[i] = Dual(pre[9 + i], (j >= 6 && j < 9) ? ADJ_EK[j][i] : 0.0);
    }
    const Dual td(Tdff, j == 9 ? 1.0 : 0.0);
    const EpsC<Dual> cb = eps_coeffs<Dual>(P, Dual(eb, j == 10 ? 1.0 : 0.0));
    const EpsC<Dual> cf = eps_coeffs<Dual>(P, Dual(ef, j == 11 ? 1.0 : 0.0));
    Macro<Dual> mb;
    wall_from_ref<Dual>(P, k, x, y, cf, cb, ff, gf, td, f, g, mb);
    node_collide<Dual>(f, g, mb, Dual(P.T0), k, cb);   // the state the boundary scheme assigns
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) acc += lam[i] * f[i].d + lam[9 + i] * g[i].d;
    if (j < 9) {
        // less the direct part (1 - 1/tau) lambda . e_k
        double dir = 0.0;
#pragma unroll
        for (int i = 0; i < 9; ++i) dir += (j < 6 ? P.cd.of * lam[i] : P.cd.og * lam[9 + i]) * ADJ_EK[j][i];
        A.wf[j * N + n] = acc - dir;
    } else if (j == 9) {
        A.wt[n] = acc;
    } else if (j == 10) {
        A.grad[n] += acc;
    } else {
        A.we[n] = acc;
    }
    if (j == 0) {
        // the wall node's own pulled populations are not used (the boundary scheme replaces
        // them): lambda_t(b - c_q, q) = 0; populations of b leaving the grid are dropped:
        // lambda_t(b, q) = 0 where b + c_q is off the grid
#pragma unroll
        for (int q = 0; q < 18; ++q) {
            const int i = q < 9 ? q : q - 9;
            int sx = x - CXd[i], sy = y - CYd[i];
            if (P.px) sx = (sx + P.nx) % P.nx;
            if (P.py) sy = (sy + P.ny) % P.ny;
            if (sx >= 0 && sx < P.nx && sy >= 0 && sy < P.ny) A.lam[q * N + (long long)sy * P.nx + sx] = 0.0;
            int zx = x + CXd[i], zy = y + CYd[i];
            if (P.px) zx = (zx + P.nx) % P.nx;
            if (P.py) zy = (zy + P.ny) % P.ny;
            if (zx < 0 || zx >= P.nx || zy < 0 || zy >= P.ny) A.lam[q * N + n] = 0.0;
        }
    }
}

// Steps 1 and 2 in one launch of 64-thread blocks: blocks [0, 12 nwb) take the wall nodes'
// Jacobian columns (wall slot (b % nwb) * 64 + lane, column b / nwb), the longest work,
// first; the remaining blocks the nodes off the walls.  The two parts write disjoint
// entries (each adjoint entry has one source node; grad and the wall arrays per node), so
// they run side by side.
template <typename S>
__global__ void __launch_bounds__(ADJ_WB)
k_adj_step(const S *__restrict__ src, KParams P, AdjBufs A, int nwb)
{
    const int b = blockIdx.x;
    if (b < nwb * ADJ_WCOLS) {
        adj_wall_node<S>(src, P, A, (b % nwb) * ADJ_WB + (int)threadIdx.x, b / nwb);
        return;
    }
    adj_interior_node<S>(src, P, A, (long long)(b - nwb * ADJ_WCOLS) * ADJ_WB + threadIdx.x);
}

// Adjoint of the wall node b's update with respect to population q of its reference node's
// pulled populations: (1 - 1/tau) lambda_{t+1}(b, q) plus the moment adjoints a_k times the
// moment weights of direction q.
__device__ __forceinline__ double wall_ref_mu(const KParams &P, const AdjBufs &A, long long N, long long b, int q)
{
    const int i = q < 9 ? q : q - 9;
    const double cx = CXd[i], cy = CYd[i];
    if (q < 9)
        return P.cd.of * A.lam_next[q * N + b] + (i ? A.wf[0 * N + b] : 0.0) + cx * A.wf[1 * N + b]
             + cy * A.wf[2 * N + b] + cx * cx * A.wf[3 * N + b] + cy * cy * A.wf[4 * N + b]
             + cx * cy * A.wf[5 * N + b];
    return P.cd.og * A.lam_next[q * N + b] + A.wf[6 * N + b] + cx * A.wf[7 * N + b] + cy * A.wf[8 * N + b];
}

// Sum over the wall nodes b whose reference node at distance dist (1: x_f, 2: x_ff) is
// (zx, zy) of arr[q][b] (arr non-null), or of wall_ref_mu(b, q) (arr null); with
// neumann_only, only prescribed-gradient wall nodes count.
__device__ __forceinline__ double sum_wall_refs(const KParams &P, const AdjBufs &A, const double *arr, long long N,
                                                int q, int zx, int zy, int dist, bool neumann_only)
{
    double s = 0.0;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
        const int dx = CXd[i], dy = CYd[i];
        const int bx = zx - dist * dx, by = zy - dist * dy;
        if (bx < 0 || bx >= P.nx || by < 0 || by >= P.ny || !on_wall(P, bx, by)) continue;
        const WallInfo w = wall_info(P, bx, by);
        if (w.dx != dx || w.dy != dy) continue;
        if (neumann_only && thermal_dirichlet_wall(P, w) >= 0) continue;
        const long long b = (long long)by * P.nx + bx;
        s += arr ? arr[q * N + b] : wall_ref_mu(P, A, N, b, q);
    }
    return s;
}

// The band of nodes within four nodes of a non-periodic wall, enumerated compactly: first
// the rows y < 4 and y >= ny - 4 (walls in y), then the columns x < 4 and x >= nx - 4 (walls
// in x) of the remaining rows.
__host__ __device__ __forceinline__ int band_rows(const KParams &P) { return P.py ? 0 : (P.ny <= 8 ? P.ny : 8); }
__host__ __device__ __forceinline__ int band_cols(const KParams &P) { return P.px ? 0 : (P.nx <= 8 ? P.nx : 8); }
__host__ __device__ __forceinline__ long long band_size(const KParams &P)
{
    return (long long)band_rows(P) * P.nx + (long long)band_cols(P) * (P.ny - band_rows(P));
}
__device__ __forceinline__ void band_node(const KParams &P, long long b, int &x, int &y)
{
    const int nr = band_rows(P);
    if (b < (long long)nr * P.nx) {
        const int r = int(b / P.nx);
        x = int(b % P.nx);
        y = (P.ny <= 8 || r < 4) ? r : P.ny - 8 + r;
    } else {
        const long long j = b - (long long)nr * P.nx;
        const int nc = band_cols(P), c = int(j % nc);
        x = (P.nx <= 8 || c < 4) ? c : P.nx - 8 + c;
        y = int(j / nc) + (nr > 0 ? 4 : 0);
    }
}

// The wall-reference terms of step 2, at the band nodes y (only they can be, or neighbour,
// a reference node x_f or x_ff of a wall node): lambda_t(y, q) gains the wall nodes'
// adjoints with respect to the pulled populations of their reference node z = y + c_q, and
// T(x_ff); for q = 0, eps(y) gains the wall nodes' adjoints with respect to the porosity of
// their reference node y.  One thread per band node and direction (q = blockIdx.y), after
// k_adj_step (both parts).
__global__ void __launch_bounds__(ADJ_B) k_adj_fix(KParams P, AdjBufs A)
{
    const long long N = (long long)P.nx * P.ny;
    const long long b = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= band_size(P)) return;
    int x, y;
    band_node(P, b, x, y);
    const long long n = (long long)y * P.nx + x;
    const int q = blockIdx.y, i = q < 9 ? q : q - 9;
    int zx = x + CXd[i], zy = y + CYd[i];
    if (P.px) zx = (zx + P.nx) % P.nx;
    if (P.py) zy = (zy + P.ny) % P.ny;
    if (zx >= 0 && zx < P.nx && zy >= 0 && zy < P.ny && !on_wall(P, zx, zy)) {
        double v = sum_wall_refs(P, A, nullptr, N, q, zx, zy, 1, false);
        if (q >= 9) v += (1.0 / P.sigma) * sum_wall_refs(P, A, A.wt, N, 0, zx, zy, 2, true);
        A.lam[q * N + n] += v;
    }
    if (q == 0 && !on_wall(P, x, y)) A.grad[n] += sum_wall_refs(P, A, A.we, N, 0, x, y, 1, false);
}

// Seed lambda_N = dJ/ds_N for J depending on T at interior nodes with weights wtj
// (T = T0 + (sum_i g_i + Q/2) / sigma, g_i(z) = s_N(z - c_i, 9 + i)).
__global__ void __launch_bounds__(ADJ_B) k_adj_seed(KParams P, AdjBufs A)
{
    const long long N = (long long)P.nx * P.ny;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const int x = int(n % P.nx), y = int(n / P.nx);
    const double isig = 1.0 / P.sigma;
    for (int q = 0; q < 18; ++q) {
        double v = 0.0;
        if (q >= 9) {
            const int i = q - 9;
            int zx = x + CXd[i], zy = y + CYd[i];
            if (P.px) zx = (zx + P.nx) % P.nx;
            if (P.py) zy = (zy + P.ny) % P.ny;
            if (zx >= 0 && zx < P.nx && zy >= 0 && zy < P.ny && !on_wall(P, zx, zy))
                v = A.wtj[(long long)zy * P.nx + zx] * isig;
        }
        A.lam[q * N + n] = v;
    }
}

template <typename S>
static hipError_t adj_step_t(const void *state, const KParams &P, const AdjBufs &A, hipStream_t st)
{
    const long long N = (long long)P.nx * P.ny;
    const int nwb = (P.nwall + ADJ_WB - 1) / ADJ_WB;
    const long long nb = nwb * ADJ_WCOLS + (N + ADJ_WB - 1) / ADJ_WB;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_adj_step<S>), dim3((unsigned)nb), dim3(ADJ_WB), 0, st, (const S *)state, P, A, nwb);
    if (P.nwall > 0) {
        const long long nband = band_size(P);
        hipLaunchKernelGGL(k_adj_fix, dim3(unsigned((nband + ADJ_B - 1) / ADJ_B), 18), dim3(ADJ_B), 0, st, P, A);
    }
    return hipGetLastError();
}

hipError_t launch_adjoint_step(int storage, const void *state, const KParams &P, const AdjBufs &A,
                               hipStream_t st)
{
    switch (storage) {
    case 0: return adj_step_t<double>(state, P, A, st);
    case 1: return adj_step_t<float>(state, P, A, st);
    case 2: return adj_step_t<__half>(state, P, A, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_adjoint_seed(const KParams &P, const AdjBufs &A, hipStream_t st)
{
    const long long N = (long long)P.nx * P.ny;
    hipLaunchKernelGGL(k_adj_seed, dim3(int((N + ADJ_B - 1) / ADJ_B)), dim3(ADJ_B), 0, st, P, A);
    return hipGetLastError();
}

}  // namespace lbm
