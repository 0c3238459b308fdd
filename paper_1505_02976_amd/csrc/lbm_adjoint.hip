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
//      wall nodes that use y + c_q as their reference node.
// The Jacobian columns come from forward-mode dual numbers pushed through the same
// templated node code as the forward step, one column per input.
#include "lbm_kernels.h"

namespace lbm {

constexpr int ADJ_B = 128;
// The Jacobian columns of a node are split over ADJ_SPLIT blocks (blockIdx.y): column j
// goes to block j % ADJ_SPLIT.  At 256 VGPRs a SIMD holds two wavefronts; one thread per
// node would leave a 256^2 grid with one wavefront per SIMD and its memory latency exposed
// (backward sweep of the 256^2 cavity over 5000 steps: 1.84 s with one thread per node,
// 1.44 / 1.24 / 1.11 s with 2 / 4 / 8 column groups).
constexpr int ADJ_SPLIT = 8;

__device__ __forceinline__ Cst<Dual> dual_cst(const Cst<double> &c)
{
    Cst<Dual> d;
    d.itf = Dual(c.itf); d.itT = Dual(c.itT); d.of = Dual(c.of); d.og = Dual(c.og);
    d.fF = Dual(c.fF); d.fT = Dual(c.fT); d.tau_f = Dual(c.tau_f); d.A = Dual(c.A);
    d.sigB = Dual(c.sigB); d.sig = Dual(c.sig); d.isig = Dual(c.isig); d.Q = Dual(c.Q);
    d.halfQ = Dual(c.halfQ); d.gb = Dual(c.gb); d.ax = Dual(c.ax); d.ay = Dual(c.ay);
    d.Sden = Dual(c.Sden); d.aM0 = Dual(c.aM0); d.w1 = Dual(c.w1); d.w5 = Dual(c.w5);
    d.w3a = Dual(c.w3a); d.w3d = Dual(c.w3d);
    return d;
}

__device__ __forceinline__ void dual_update(Dual *f, Dual *g, const KParams &P, const Cst<Dual> &k,
                                            const EpsC<Dual> &e)
{
    Macro<Dual> m;
    node_macro_full<Dual>(f, g, Dual(P.T0), k, e, m);
    node_collide<Dual>(f, g, m, Dual(P.T0), k, e);
}

// Step 1 at every node, Jacobian columns j = blockIdx.y, blockIdx.y + ADJ_SPLIT, ...  Every
// output (mu[j], grad via column 18 or 19, wt, we, wf[j]) has one writer.
template <typename S>
__global__ void __launch_bounds__(ADJ_B)
k_adj_node(const S *__restrict__ src, KParams P, AdjBufs A)
{
    const long long N = (long long)P.nx * P.ny;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int j0 = blockIdx.y;
    if (n >= N) return;
    const int x = int(n % P.nx), y = int(n / P.nx);
    double lam[18];
#pragma unroll
    for (int q = 0; q < 18; ++q) lam[q] = A.lam_next[q * N + n];
    const Cst<Dual> k = dual_cst(P.cd);
    if (!on_wall(P, x, y)) {
        double pre[18];
        gather<S, double>(src, P, x, y, pre, pre + 9);
        const double eps = eps_value(P, x, y);
#pragma unroll 1
        for (int j = j0; j < 19; j += ADJ_SPLIT) {
            Dual f[9], g[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                f[i] = Dual(pre[i], j == i ? 1.0 : 0.0);
                g[i] = Dual(pre[9 + i], j == 9 + i ? 1.0 : 0.0);
            }
            const EpsC<Dual> e = eps_coeffs<Dual>(P, Dual(eps, j == 18 ? 1.0 : 0.0));
            dual_update(f, g, P, k, e);
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < 9; ++i) acc += lam[i] * f[i].d + lam[9 + i] * g[i].d;
            if (j < 18) A.mu[j * N + n] = acc;
            else A.grad[n] += acc;
        }
    } else {
        const WallInfo w = wall_info(P, x, y);
        const int xf = x + w.dx, yf = y + w.dy;
        double pre[18];
        gather<S, double>(src, P, xf, yf, pre, pre + 9);
        const bool neumann = thermal_dirichlet_wall(P, w) < 0;
        const double Tdff = neumann ? gather_Td<S, double>(src, P, P.cd, x + 2 * w.dx, y + 2 * w.dy) : 0.0;
        const double eb = eps_value(P, x, y), ef = eps_value(P, xf, yf);
#pragma unroll 1
        for (int j = j0; j < 21; j += ADJ_SPLIT) {
            Dual ff[9], gf[9], f[9], g[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                ff[i] = Dual(pre[i], j == i ? 1.0 : 0.0);
                gf[i] = Dual(pre[9 + i], j == 9 + i ? 1.0 : 0.0);
            }
            const Dual td(Tdff, j == 18 ? 1.0 : 0.0);
            const EpsC<Dual> cb = eps_coeffs<Dual>(P, Dual(eb, j == 19 ? 1.0 : 0.0));
            const EpsC<Dual> cf = eps_coeffs<Dual>(P, Dual(ef, j == 20 ? 1.0 : 0.0));
            Macro<Dual> mb;
            wall_from_ref<Dual>(P, k, x, y, cf, cb, ff, gf, td, f, g, mb);
            node_collide<Dual>(f, g, mb, Dual(P.T0), k, cb);   // the state the boundary scheme assigns
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < 9; ++i) acc += lam[i] * f[i].d + lam[9 + i] * g[i].d;
            if (j < 18) A.wf[j * N + n] = acc;
            else if (j == 18) A.wt[n] = acc;
            else if (j == 19) A.grad[n] += acc;
            else A.we[n] = acc;
        }
        if (j0 == 0) {
#pragma unroll
            for (int q = 0; q < 18; ++q) A.mu[q * N + n] = 0.0;   // own gathered values unused
        }
    }
}

// Sum of arr over the wall nodes b whose reference node at distance dist (1: x_f, 2: x_ff)
// is (zx, zy); with neumann_only, only prescribed-gradient wall nodes count.
__device__ __forceinline__ double sum_wall_refs(const KParams &P, const double *arr, long long N, int q,
                                                int zx, int zy, int dist, bool neumann_only)
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
        s += arr[q * N + (long long)by * P.nx + bx];
    }
    return s;
}

// Step 2 at every node y, one direction q = blockIdx.y per thread: lambda_t(y, q), and for
// q = 0 the eps contributions routed through x_f.
__global__ void __launch_bounds__(ADJ_B) k_adj_pull(KParams P, AdjBufs A)
{
    const long long N = (long long)P.nx * P.ny;
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int q = blockIdx.y;
    if (n >= N) return;
    const int x = int(n % P.nx), y = int(n / P.nx);
    const double isig = 1.0 / P.sigma;
    // only nodes within three nodes of a wall can be (or neighbour) a reference node x_f
    // or x_ff of a wall node
    const bool near = (!P.px && (x < 4 || x >= P.nx - 4)) || (!P.py && (y < 4 || y >= P.ny - 4));
    {
        const int i = q < 9 ? q : q - 9;
        int zx = x + CXd[i], zy = y + CYd[i];
        if (P.px) zx = (zx + P.nx) % P.nx;
        if (P.py) zy = (zy + P.ny) % P.ny;
        double v = 0.0;
        if (zx >= 0 && zx < P.nx && zy >= 0 && zy < P.ny && !on_wall(P, zx, zy)) {
            const long long nz = (long long)zy * P.nx + zx;
            v = A.mu[q * N + nz];
            if (near) {
                v += sum_wall_refs(P, A.wf, N, q, zx, zy, 1, false);
                if (q >= 9) v += isig * sum_wall_refs(P, A.wt, N, 0, zx, zy, 2, true);
            }
        }
        A.lam[q * N + n] = v;
    }
    if (q == 0 && near && !on_wall(P, x, y)) A.grad[n] += sum_wall_refs(P, A.we, N, 0, x, y, 1, false);
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
    const int nb = int((N + ADJ_B - 1) / ADJ_B);
    hipLaunchKernelGGL((k_adj_node<S>), dim3(nb, ADJ_SPLIT), dim3(ADJ_B), 0, st, (const S *)state, P, A);
    hipLaunchKernelGGL(k_adj_pull, dim3(nb, 18), dim3(ADJ_B), 0, st, P, A);
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
