// Two time steps per pass over HBM.
//
// A wavefront owns 64 consecutive columns x = X0 - 1 ... X0 + 62 and a band of output rows
// [Y0, Y1).  It walks up the band one row at a time: for row yy it computes the
// post-collision populations of the intermediate step, P1(., yy), exactly as the one-step
// kernels do (pull from the source buffer, boundary scheme at wall nodes, collision), and
// then the final step for row yy - 1 from P1 of rows yy - 2, yy - 1 and yy: the pull in y
// reads the rows kept in registers, the pull in x takes the neighbouring lane's value by
// a wavefront shift.  Lanes 1..62 write their result, so consecutive wavefronts overlap by
// two columns (and bands by two rows of P1), which they compute redundantly.
//
// Only the values a later row needs are kept: from P1(yy - 1) the directions with
// c_y = 0 (0, 1, 3) and c_y = +1 (2, 5, 6), from P1(yy - 2) the directions with c_y = +1;
// directions with c_y = -1 (4, 7, 8) are used as soon as their row is computed.
//
// Nodes on the walls x = 0 and x = nx - 1 take the boundary scheme from the neighbouring
// lanes' pulled populations, as in the one-step kernel.  The walled rows y = 0 and
// y = ny - 1 need the intermediate populations of three more rows for their reference
// nodes, so the pass writes P1 of rows 0-3 and ny-4..ny-1 to a small scratch grid and a
// second launch finishes those two rows.
//
// Every node update is the one-step node code with the same inputs, so two steps here are
// bitwise identical to two one-step launches (FP16 storage rounds P1 to the stored format
// before it is used, as the one-step path does by storing it).
//
// The 62-column outputs are not aligned to cache lines, which costs write bandwidth (a
// copy with such writes runs at 3.3 TB/s against 5.4 aligned); the pass pays off where
// the one-step kernel is furthest from its arithmetic limit, FP64 storage, and is the
// default there only.
#include <vector>

#include "lbm_kernels.h"

namespace lbm {

#ifndef LBM_STEP2_TY
#define LBM_STEP2_TY 8
#endif
constexpr int S2_TY = LBM_STEP2_TY;   // output rows per wavefront

constexpr int S2_OUT = 62;            // output columns per wavefront
constexpr int S2_B = 256;             // threads per block (independent wavefronts)

// The lean instance gathers the next row's populations while it updates the current one
// (one more set of 18 registers); FP64 has no registers to spare for it.
#ifndef LBM_STEP2_PREFETCH
#define LBM_STEP2_PREFETCH 1
#endif
template <typename S> struct S2Prefetch { static constexpr bool v = LBM_STEP2_PREFETCH != 0; };
template <> struct S2Prefetch<double> { static constexpr bool v = false; };

// Wavefront shifts: lane l receives lane l - 1 (from_left) or lane l + 1 (from_right);
// lane 0 (resp. 63) keeps its own value.
__device__ __forceinline__ int dpp_left(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x138, 0xf, 0xf, false); }
__device__ __forceinline__ int dpp_right(int v) { return __builtin_amdgcn_update_dpp(v, v, 0x130, 0xf, 0xf, false); }
__device__ __forceinline__ float from_left(float v) { return __builtin_bit_cast(float, dpp_left(__builtin_bit_cast(int, v))); }
__device__ __forceinline__ float from_right(float v) { return __builtin_bit_cast(float, dpp_right(__builtin_bit_cast(int, v))); }
__device__ __forceinline__ double from_left(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = dpp_left((int)(b & 0xffffffffLL)), hi = dpp_left((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double from_right(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = dpp_right((int)(b & 0xffffffffLL)), hi = dpp_right((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// Value of an intermediate population as the one-step path would read it back.
template <typename S, typename R> __device__ __forceinline__ R as_stored(R v, const KParams &) { return v; }
template <> __device__ __forceinline__ float as_stored<__half, float>(float v, const KParams &P)
{
    return __builtin_fmaf(__half2float(__float2half(v * P.hscale)), P.hinv, 0.0f);
}

// Post-collision populations of node (x, y) one step after src (the one-step node code).
template <typename S, typename R>
__device__ __forceinline__ void p1_node(const S *__restrict__ src, const KParams &P, int x, int y, R *f, R *g)
{
    if (on_wall(P, x, y))
        wall_populations<S, R>(src, P, make_cst<R>(P), x, y, f, g);
    else
        gather<S, R>(src, P, x, y, f, g);
    node_update<R, typename Prec<S>::M>(f, g, P, x, y);
}

// Whether the wavefront (column chunk cxi, row band cyi) touches no wall node, no node
// whose intermediate state goes to the scratch grid and no row outside the grid: then it
// runs the lean instance of the kernel, without the boundary-scheme code.
__host__ __device__ __forceinline__ bool s2_lean(const KParams &P, int cxi, int cyi)
{
    const int X0 = min(cxi * S2_OUT, P.nx - S2_OUT);
    const int Y0 = cyi * S2_TY, Y1 = min(Y0 + S2_TY, P.ny);
    const bool xin = P.px || (X0 - 1 >= 1 && X0 + S2_OUT <= P.nx - 2);
    const bool yin = P.py || (Y0 - 1 >= 4 && Y1 <= P.ny - 5);
    return xin && yin;
}

// One wavefront's walk: column chunk cxi, row band cyi.
template <typename S, bool FULL>
__device__ __forceinline__ void march2(const S *__restrict__ src, S *__restrict__ dst, S *__restrict__ scr,
                                       const KParams &P, const KParams &Pm, int cxi, int cyi, int lane)
{
    using R = typename Prec<S>::R;
    const int X0 = min(cxi * S2_OUT, P.nx - S2_OUT);
    int x = X0 - 1 + lane;                               // X0 < 0 when nx < 62
    bool xok = true;
    if (P.px) x = ((x % P.nx) + P.nx) % P.nx;
    else xok = x >= 0 && x < P.nx;
    const bool xout = lane >= 1 && lane <= S2_OUT && xok;
    const bool vwall = xok && !P.px && (x == 0 || x == P.nx - 1);
    const int Y0 = cyi * S2_TY, Y1 = min(Y0 + S2_TY, P.ny);

    // kept values: U2 = (2,5,6) of P1(yy-2), U1 = (2,5,6) and C1 = (0,1,3) of P1(yy-1),
    // already shifted in x to where the final step pulls them
    R fU2[3], gU2[3], fU1[3], gU1[3], fC1[3], gC1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) fU2[k] = gU2[k] = fU1[k] = gU1[k] = fC1[k] = gC1[k] = R(0);

    constexpr bool PF = !FULL && S2Prefetch<S>::v;
    R nf[9], ng[9];                                      // next row, gathered ahead
    if constexpr (PF) gather<S, R>(src, P, x, P.py ? (Y0 - 1 + P.ny) % P.ny : Y0 - 1, nf, ng);

    for (int yy = Y0 - 1; yy <= Y1; ++yy) {
        int yr = yy;
        bool yok = true;
        if (P.py) yr = (yy + P.ny) % P.ny;
        else yok = yy >= 0 && yy < P.ny;
        R f[9], g[9];
        if (!FULL) {
            if constexpr (PF) {
#pragma unroll
                for (int i = 0; i < 9; ++i) { f[i] = nf[i]; g[i] = ng[i]; }
                if (yy < Y1) gather<S, R>(src, P, x, P.py ? (yy + 1) % P.ny : yy + 1, nf, ng);
            } else {
                gather<S, R>(src, P, x, yr, f, g);
            }
            node_update<R, typename Prec<S>::M>(f, g, P, x, yr);
#pragma unroll
            for (int i = 0; i < 9; ++i) { f[i] = as_stored<S, R>(f[i], P); g[i] = as_stored<S, R>(g[i], P); }
        } else if (xok && yok) {
            p1_node<S, R>(src, P, x, yr, f, g);
#pragma unroll
            for (int i = 0; i < 9; ++i) { f[i] = as_stored<S, R>(f[i], P); g[i] = as_stored<S, R>(g[i], P); }
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) f[i] = g[i] = R(0);
        }
        // intermediate rows the walled rows' boundary scheme needs (scratch rows 0-3, 4-7)
        if (FULL && !P.py && yok && xok && (yr <= 3 || yr >= P.ny - 4)) {
            const int ym = yr <= 3 ? yr : yr - (P.ny - 8);
            store_node<S, R>(scr, Pm, x, ym, f, g);
        }
        // shift in x: directions with c_x = +1 (1, 5, 8) come from the left neighbour,
        // c_x = -1 (3, 6, 7) from the right one
        f[1] = from_left(f[1]); g[1] = from_left(g[1]);
        f[5] = from_left(f[5]); g[5] = from_left(g[5]);
        f[8] = from_left(f[8]); g[8] = from_left(g[8]);
        f[3] = from_right(f[3]); g[3] = from_right(g[3]);
        f[6] = from_right(f[6]); g[6] = from_right(g[6]);
        f[7] = from_right(f[7]); g[7] = from_right(g[7]);

        const int o = yy - 1;                            // output row of this iteration
        int orow = o;
        bool oout = o >= Y0 && o < Y1;
        if (P.py) orow = (o + P.ny) % P.ny;
        else oout = oout && o >= 1 && o <= P.ny - 2;     // walled rows: second launch
        if (oout) {                                      // wavefront-uniform
            // pre-collision populations of (x, orow) at the final step
            R pf[9], pg[9];
            pf[0] = fC1[0]; pg[0] = gC1[0];
            pf[1] = fC1[1]; pg[1] = gC1[1];
            pf[3] = fC1[2]; pg[3] = gC1[2];
            pf[2] = fU2[0]; pg[2] = gU2[0];
            pf[5] = fU2[1]; pg[5] = gU2[1];
            pf[6] = fU2[2]; pg[6] = gU2[2];
            pf[4] = f[4]; pg[4] = g[4];
            pf[7] = f[7]; pg[7] = g[7];
            pf[8] = f[8]; pg[8] = g[8];
            if (FULL && __ballot(vwall && xout)) {       // wavefront-uniform
                const Cst<R> &c = make_cst<R>(P);
                R sg = R(0);
#pragma unroll
                for (int i = 0; i < 9; ++i) sg += pg[i];
                const R Td_own = (sg + c.halfQ) * c.isig;
                const int dx = (x == 0) ? 1 : -1;
                const int s1 = vwall ? lane + dx : lane, s2 = vwall ? lane + 2 * dx : lane;
                R ff[9], gf[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) { ff[i] = __shfl(pf[i], s1); gf[i] = __shfl(pg[i], s1); }
                const R Tdff = __shfl(Td_own, s2);
                if (vwall && xout) {
                    const R Tn = thermal_dirichlet_wall(P, wall_info(P, x, orow)) < 0 ? Tdff : R(0);
                    wall_from_ref<R>(P, c, x, orow, eps_at<R>(P, x + dx, orow), eps_at<R>(P, x, orow),
                                     ff, gf, Tn, pf, pg);
                }
            }
            if (xout) {
                node_update<R, typename Prec<S>::M>(pf, pg, P, x, orow);
                store_node<S, R>(dst, P, x, orow, pf, pg);
            }
        }
        // advance the kept values by one row
#pragma unroll
        for (int k = 0; k < 3; ++k) { fU2[k] = fU1[k]; gU2[k] = gU1[k]; }
        fU1[0] = f[2]; gU1[0] = g[2];
        fU1[1] = f[5]; gU1[1] = g[5];
        fU1[2] = f[6]; gU1[2] = g[6];
        fC1[0] = f[0]; gC1[0] = g[0];
        fC1[1] = f[1]; gC1[1] = g[1];
        fC1[2] = f[3]; gC1[2] = g[3];
    }
}

template <typename S, bool FULL>
__global__ void __launch_bounds__(S2_B)
k_step2(const S *__restrict__ src, S *__restrict__ dst, S *__restrict__ scr, KParams P, KParams Pm,
        int ncx, int ncy)
{
    const int wave = blockIdx.x * (S2_B / 64) + (threadIdx.x >> 6);
    if (wave >= ncx * ncy) return;                       // wavefront-uniform
    const int cxi = wave % ncx, cyi = wave / ncx;
    if (s2_lean(P, cxi, cyi) == FULL) return;            // the other instance's wavefront
    march2<S, FULL>(src, dst, scr, P, Pm, cxi, cyi, threadIdx.x & 63);
}

// Batched: item (problem, wavefront index); the host sorts the wavefronts of every problem
// into the lean and the full item lists.
template <typename S, bool FULL>
__global__ void __launch_bounds__(S2_B)
k_batch_step2(const BatchProblem *__restrict__ probs, const int2 *__restrict__ items, int nitems, int parity)
{
    const int wi = blockIdx.x * (S2_B / 64) + (threadIdx.x >> 6);
    if (wi >= nitems) return;                            // wavefront-uniform
    const int2 it = items[wi];
    const BatchProblem &B = probs[it.x];
    const int ncx = (B.P.nx + S2_OUT - 1) / S2_OUT;
    march2<S, FULL>(static_cast<const S *>(B.buf[parity]), static_cast<S *>(B.buf[parity ^ 1]),
                    static_cast<S *>(B.scr), B.P, B.Pm, it.y % ncx, it.y / ncx, threadIdx.x & 63);
}

// Final step of the walled rows y = 0 and y = ny - 1 from the intermediate rows in the
// scratch grid (rows 0-3 hold y = 0..3, rows 4-7 hold y = ny-4..ny-1).
template <typename S>
__device__ __forceinline__ void rows2_node(const S *__restrict__ scr, S *__restrict__ dst, const KParams &P,
                                           const KParams &Pm, int s)
{
    using M = typename Prec<S>::M;
    if (s >= 2 * P.nx) return;
    const int x = s % P.nx;
    const bool top = s >= P.nx;
    const int y = top ? P.ny - 1 : 0, ym = top ? 7 : 0;
    const WallInfo w = wall_info(P, x, y);
    const Cst<M> &k = make_cst<M>(P);
    M ff[9], gf[9], f[9], g[9];
    gather<S, M>(scr, Pm, x + w.dx, ym + w.dy, ff, gf);
    M Tdff = M(0);
    if (thermal_dirichlet_wall(P, w) < 0) Tdff = gather_Td<S, M>(scr, Pm, k, x + 2 * w.dx, ym + 2 * w.dy);
    wall_from_ref<M>(P, k, x, y, eps_at<M>(P, x + w.dx, y + w.dy), eps_at<M>(P, x, y), ff, gf, Tdff, f, g);
    node_update<M, M>(f, g, P, x, y);
    store_node<S, M>(dst, P, x, y, f, g);
}

template <typename S>
__global__ void __launch_bounds__(64)
k_step2_rows(const S *__restrict__ scr, S *__restrict__ dst, KParams P, KParams Pm)
{
    rows2_node<S>(scr, dst, P, Pm, blockIdx.x * blockDim.x + threadIdx.x);
}

// Batched: item (problem, block of 64 walled-row nodes).
template <typename S>
__global__ void __launch_bounds__(64)
k_batch_step2_rows(const BatchProblem *__restrict__ probs, const int2 *__restrict__ items, int parity)
{
    const int2 it = items[blockIdx.x];
    const BatchProblem &B = probs[it.x];
    rows2_node<S>(static_cast<const S *>(B.scr), static_cast<S *>(B.buf[parity ^ 1]), B.P, B.Pm,
                  it.y * 64 + threadIdx.x);
}

template <typename S, bool FULL>
static hipError_t step2_main_t(const void *src, void *dst, void *scr, const KParams &P, const KParams &Pm,
                               hipStream_t st)
{
    const int ncx = (P.nx + S2_OUT - 1) / S2_OUT;
    const int ncy = (P.ny + S2_TY - 1) / S2_TY;
    const long long waves = (long long)ncx * ncy;
    const int blocks = (int)((waves + S2_B / 64 - 1) / (S2_B / 64));
    hipLaunchKernelGGL((k_step2<S, FULL>), dim3(blocks), dim3(S2_B), 0, st, (const S *)src, (S *)dst, (S *)scr,
                       P, Pm, ncx, ncy);
    return hipGetLastError();
}

template <typename S>
static hipError_t step2_rows_t(void *dst, const void *scr, const KParams &P, const KParams &Pm, hipStream_t st)
{
    if (!P.py)
        hipLaunchKernelGGL((k_step2_rows<S>), dim3((2 * P.nx + 63) / 64), dim3(64), 0, st, (const S *)scr, (S *)dst,
                           P, Pm);
    return hipGetLastError();
}

// nx >= 4 (a wall column needs its two inner neighbours), ny >= 8 (the scratch grid holds
// rows 0-3 and ny-4..ny-1 without overlap).  Grids narrower than a wavefront start their
// only column chunk left of x = 0 (those lanes idle, or wrapped when x is periodic).
bool step2_supported(const KParams &P) { return P.nx >= 4 && P.ny >= 8; }

long long step2_nodes(const KParams &P) { return (long long)P.nx * (P.py ? P.ny : P.ny - 2); }

// Output nodes of the lean launch (column chunks and row bands away from walls).
long long step2_lean_nodes(const KParams &P)
{
    const int ncx = (P.nx + S2_OUT - 1) / S2_OUT;
    const int ncy = (P.ny + S2_TY - 1) / S2_TY;
    long long n = 0;
    for (int cy = 0; cy < ncy; ++cy)
        for (int cx = 0; cx < ncx; ++cx)
            if (s2_lean(P, cx, cy)) {
                const int Y0 = cy * S2_TY, Y1 = min(Y0 + S2_TY, P.ny);
                n += (long long)S2_OUT * (Y1 - Y0);
            }
    return n;
}

hipError_t launch_step2_main(int storage, bool full, const void *src, void *dst, void *scr, const KParams &P,
                             const KParams &Pm, hipStream_t st)
{
    if (!step2_supported(P)) return hipErrorInvalidValue;
    switch (storage) {
    case 0: return full ? step2_main_t<double, true>(src, dst, scr, P, Pm, st)
                        : step2_main_t<double, false>(src, dst, scr, P, Pm, st);
    case 1: return full ? step2_main_t<float, true>(src, dst, scr, P, Pm, st)
                        : step2_main_t<float, false>(src, dst, scr, P, Pm, st);
    case 2: return full ? step2_main_t<__half, true>(src, dst, scr, P, Pm, st)
                        : step2_main_t<__half, false>(src, dst, scr, P, Pm, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step2_rows(int storage, void *dst, const void *scr, const KParams &P, const KParams &Pm,
                             hipStream_t st)
{
    switch (storage) {
    case 0: return step2_rows_t<double>(dst, scr, P, Pm, st);
    case 1: return step2_rows_t<float>(dst, scr, P, Pm, st);
    case 2: return step2_rows_t<__half>(dst, scr, P, Pm, st);
    default: return hipErrorInvalidValue;
    }
}

// Wavefront indices (cyi * ncx + cxi) of a problem's lean and full wavefronts, and its
// number of walled-row blocks of 64 nodes.
void step2_wave_lists(const KParams &P, std::vector<int> &lean, std::vector<int> &full, int &row_blocks)
{
    const int ncx = (P.nx + S2_OUT - 1) / S2_OUT;
    const int ncy = (P.ny + S2_TY - 1) / S2_TY;
    lean.clear();
    full.clear();
    for (int cy = 0; cy < ncy; ++cy)
        for (int cx = 0; cx < ncx; ++cx) (s2_lean(P, cx, cy) ? lean : full).push_back(cy * ncx + cx);
    row_blocks = P.py ? 0 : (2 * P.nx + 63) / 64;
}

template <typename S>
static hipError_t batch_step2_t(const BatchProblem *probs, const int2 *lean, int nlean, const int2 *full,
                                int nfull, const int2 *rows, int nrows, int parity, hipStream_t st)
{
    constexpr int W = S2_B / 64;
    if (nlean > 0)
        hipLaunchKernelGGL((k_batch_step2<S, false>), dim3((nlean + W - 1) / W), dim3(S2_B), 0, st, probs, lean,
                           nlean, parity);
    if (nfull > 0)
        hipLaunchKernelGGL((k_batch_step2<S, true>), dim3((nfull + W - 1) / W), dim3(S2_B), 0, st, probs, full,
                           nfull, parity);
    if (nrows > 0)
        hipLaunchKernelGGL((k_batch_step2_rows<S>), dim3(nrows), dim3(64), 0, st, probs, rows, parity);
    return hipGetLastError();
}

hipError_t launch_batch_step2(int storage, const BatchProblem *probs, const int2 *lean, int nlean,
                              const int2 *full, int nfull, const int2 *rows, int nrows, int parity, hipStream_t st)
{
    switch (storage) {
    case 0: return batch_step2_t<double>(probs, lean, nlean, full, nfull, rows, nrows, parity, st);
    case 1: return batch_step2_t<float>(probs, lean, nlean, full, nfull, rows, nrows, parity, st);
    case 2: return batch_step2_t<__half>(probs, lean, nlean, full, nfull, rows, nrows, parity, st);
    default: return hipErrorInvalidValue;
    }
}

Batch2Kernels batch2_kernels(int storage)
{
    Batch2Kernels k;
    switch (storage) {
    case 0: k.lean = (const void *)k_batch_step2<double, false>; k.full = (const void *)k_batch_step2<double, true>;
            k.rows = (const void *)k_batch_step2_rows<double>; break;
    case 1: k.lean = (const void *)k_batch_step2<float, false>; k.full = (const void *)k_batch_step2<float, true>;
            k.rows = (const void *)k_batch_step2_rows<float>; break;
    default: k.lean = (const void *)k_batch_step2<__half, false>; k.full = (const void *)k_batch_step2<__half, true>;
             k.rows = (const void *)k_batch_step2_rows<__half>; break;
    }
    k.threads = S2_B;
    k.waves_per_block = S2_B / 64;
    return k;
}

}  // namespace lbm
