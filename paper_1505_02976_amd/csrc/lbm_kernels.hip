// HIP kernels of the fused collide-stream step (pull scheme, structure-of-arrays) and of
// the auxiliary passes (initialisation, macroscopic fields, residual, Nusselt number,
// state conversion) for the modified lattice-BGK porous thermal model.
//
// Layout in device memory: one population buffer holds rows of tiles of TileOf<S>
// consecutive nodes, each tile its 18 directions (f_0..f_8, g_0..g_8) contiguously,
// [y][x / T][q][x % T].  A step reads buffer src and writes buffer dst; node (x, y) pulls
// f_i from (x - c_i) and stores its post-collision populations at (x, y), so no two threads
// write the same element and no thread reads what another thread writes in the same launch.
#include "lbm_kernels.h"

namespace lbm {

constexpr int BULK_BX = 256;
constexpr int WALL_B = 64;
constexpr int RED_B = 256;

// ---------------------------------------------------------------------------------
// Initialisation: post-collision populations before the first step are the equilibria
// of the initial fields with S = 0 and grad T = 0.
// ---------------------------------------------------------------------------------
template <typename S, typename R>
__global__ void __launch_bounds__(BULK_BX)
k_init(S *__restrict__ dst, KParams P, const double *__restrict__ T_init,
       const double *__restrict__ p_init, const double *__restrict__ ux_init,
       const double *__restrict__ uy_init)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= P.nx) return;
    const long long n = (long long)y * P.nx + x;
    const Cst<R> &k = make_cst<R>(P);
    const EpsC<R> e = eps_at<R>(P, x, y);
    double T = P.T0;
    if (T_init) {
        T = T_init[n];
    } else {
        const WallInfo w = wall_info(P, x, y);
        if (w.xw >= 0 && P.wall_kind[w.xw] == 0) T = P.wall_T[w.xw];
        else if (w.yw >= 0 && P.wall_kind[w.yw] == 0) T = P.wall_T[w.yw];
    }
    const R p = p_init ? R(p_init[n]) : R(0);
    const R ux = ux_init ? R(ux_init[n]) : R(0);
    const R uy = uy_init ? R(uy_init[n]) : R(0);
    const R Td = R(T - P.T0);
    const R Tf = R(T);
    const R ep = e.eps * p;
    R f[9], g[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        f[i] = feq_i<R>(i, ep, ux, uy, e.ieps, R(0), R(0), R(0), k.A);
        g[i] = geq_i<R>(i, Td, Tf, ux, uy, e.ieps, ep, R(0), R(0), k);
    }
    store_node<S, R>(dst, P, x, y, f, g);
}

// ---------------------------------------------------------------------------------
// Fused step, bulk nodes: gather -> moments -> S, grad T -> equilibria -> collide -> store
//
// A block of BX threads covers a segment of (BX / 64) * WS * NPT consecutive nodes of one
// row, WS = Wspan (columns per wavefront: 64, or the tile width when tiles are narrower,
// so that a wavefront stores whole tile segments); lane l of wavefront w handles nodes
// w WS + l + k (BX / 64) WS, k < NPT, so every load instruction stays coalesced and each
// thread has NPT nodes' loads in flight before it computes.
// ---------------------------------------------------------------------------------
// Nodes per thread: two for FP16 (more loads in flight per thread), one otherwise.
template <typename S> struct Npt;
template <> struct Npt<double> { static constexpr int v = 1; };
template <> struct Npt<float> { static constexpr int v = 1; };
template <> struct Npt<__half> { static constexpr int v = 2; };

// Columns covered by one node slot of a block of BX threads, and by the whole block.
template <typename S, int BX> __host__ __device__ constexpr int slot_span() { return (BX / 64) * Wspan<S>::v; }
template <typename S, int BX> __host__ __device__ constexpr int block_span() { return slot_span<S, BX>() * Npt<S>::v; }

// One row segment of the bulk update: nodes x = xbeg + (tid / 64) WS + tid % 64 +
// k (BX / 64) WS (k < NPT) with x < xend, of row y (tid: the thread's index among the BX
// threads of the segment).
//
// Nodes on the walls x = 0 and x = nx - 1 (outside the walled rows) are updated here too:
// the lanes of a wavefront hold consecutive x, so the reference node x_f = x -+ 1 of a
// wall node (and x_ff = x -+ 2 on prescribed-gradient walls) normally sits in the
// neighbouring lane, whose streamed populations are taken by cross-lane shuffles; only
// when it falls in another wavefront is it gathered from memory.  Only wavefronts that
// contain such a node take this branch.
template <typename S, bool WALLS, int BX, int NPT = Npt<S>::v>
__device__ __forceinline__ void bulk_tile(const S *__restrict__ src, S *__restrict__ dst,
                                          const KParams &P, int y, int xbeg, int xend,
                                          int tid)
{
    constexpr int WS = Wspan<S>::v, SPAN = slot_span<S, BX>();
    using RC = typename Prec<S>::R;
    const int wl = tid & 63;
    const bool lane_on = wl < WS;
    const int x0 = xbeg + (tid >> 6) * WS + wl;
    if (!P.py && (y == 0 || y == P.ny - 1)) return;
    RC f[NPT][9], g[NPT][9];
    bool act[NPT], vw[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int x = x0 + k * SPAN;
        vw[k] = WALLS && lane_on && x < xend && !P.px && (x == 0 || x == P.nx - 1);
        act[k] = lane_on && x < xend && !vw[k];
        if (act[k]) gather<S, RC>(src, P, x, y, f[k], g[k]);
    }
    if (WALLS && !P.px) {
        const Cst<RC> &c = make_cst<RC>(P);
        const int lane = __lane_id();
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            if (!__ballot(vw[k])) continue;               // wavefront-uniform
            const int x = x0 + k * SPAN;
            const int dx = (x == 0) ? 1 : -1;
            RC sg = RC(0);
#pragma unroll
            for (int i = 0; i < 9; ++i) sg += g[k][i];
            const RC Td_own = (sg + c.halfQ) * c.isig;
            const int l1 = lane + dx, l2 = lane + 2 * dx;
            const bool in1 = vw[k] && l1 >= 0 && l1 < WS;
            const bool in2 = vw[k] && l2 >= 0 && l2 < WS;
            const int s1 = in1 ? l1 : lane, s2 = in2 ? l2 : lane;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                f[k][i] = __shfl(f[k][i], s1);
                g[k][i] = __shfl(g[k][i], s1);
            }
            RC Tdff = __shfl(Td_own, s2);
            if (vw[k]) {
                if (!in1) gather<S, RC>(src, P, x + dx, y, f[k], g[k]);
                if (!in2 && thermal_dirichlet_wall(P, wall_info(P, x, y)) < 0)
                    Tdff = gather_Td<S, RC>(src, P, c, x + 2 * dx, y);
                Macro<RC> mb;
                wall_from_ref<RC>(P, c, x, y, eps_at<RC>(P, x + dx, y), eps_at<RC>(P, x, y),
                                  f[k], g[k], Tdff, f[k], g[k], mb);
                wall_collide<RC>(f[k], g[k], mb, P, x, y);
                store_node<S, RC>(dst, P, x, y, f[k], g[k]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        if (!act[k]) continue;
        const int x = x0 + k * SPAN;
        node_update<RC, typename Prec<S>::M>(f[k], g[k], P, x, y);
        store_node<S, RC>(dst, P, x, y, f[k], g[k]);
    }
}

// One node of the walled rows y = 0 and y = ny - 1 (slot s < nwall_rows): boundary scheme
// -> collision with the state it assigns -> store.
template <typename S>
__device__ __forceinline__ void wall_node(const S *__restrict__ src, S *__restrict__ dst,
                                          const KParams &P, int s)
{
    int x, y;
    if (s >= P.nwall_rows || !wall_slot(P, s, x, y)) return;
    using M = typename Prec<S>::M;
    M f[9], g[9];
    Macro<M> mb;
    wall_populations<S, M>(src, P, make_cst<M>(P), x, y, f, g, mb);
    wall_collide<M>(f, g, mb, P, x, y);
    store_node<S, M>(dst, P, x, y, f, g);
}

// Columns of the interior launch: [xa, xb) of every non-walled row, no node of the walls
// x = 0, x = nx - 1.  The edge launch covers the rest of those rows in segments of one
// wavefront with one node per lane (Wspan nodes): [0, xa) and [xb, nx) -- a single segment
// at each end when the row is at least two segments long, else the whole row -- and the
// walled rows.  One node per lane keeps the edge instance's register count low and leaves
// fewer nodes to its slower wall-aware code.
constexpr int EDGE_BX = 64;

struct Cols { int xa, xb, nseg, span_e; bool split; };

template <typename S> __host__ __device__ __forceinline__ Cols step_cols(const KParams &P)
{
    Cols c;
    c.span_e = slot_span<S, EDGE_BX>();
    c.split = !P.px && P.nx >= 2 * c.span_e;
    if (P.px) { c.xa = 0; c.xb = P.nx; c.nseg = 0; }
    else if (c.split) { c.xa = c.span_e; c.xb = P.nx - c.span_e; c.nseg = 2; }
    else { c.xa = c.xb = P.nx; c.nseg = (P.nx + c.span_e - 1) / c.span_e; }
    return c;
}

__host__ __device__ __forceinline__ int rows_begin(const KParams &P) { return P.py ? 0 : 1; }
__host__ __device__ __forceinline__ int rows_count(const KParams &P) { return P.py ? P.ny : P.ny - 2; }

template <typename S> __host__ __device__ __forceinline__ int interior_segments(const KParams &P)
{
    const Cols c = step_cols<S>(P);
    const int span = block_span<S, BULK_BX>();
    return (c.xb - c.xa + span - 1) / span;
}

template <typename S, typename R>
__global__ void __launch_bounds__(BULK_BX)
k_step_bulk(const S *__restrict__ src, S *__restrict__ dst, KParams P, int nseg)
{
    const Cols c = step_cols<S>(P);
    const int r = blockIdx.x / nseg, s = blockIdx.x - r * nseg;
    bulk_tile<S, false, BULK_BX>(src, dst, P, rows_begin(P) + r, c.xa + s * block_span<S, BULK_BX>(), c.xb,
                                 threadIdx.x);
}

// Work item `item` of the wall-side update (one wavefront): items [0, ne) are the edge
// segments (row by row), the remaining ones blocks of EDGE_BX walled-row nodes.
template <typename S>
__device__ __forceinline__ void edge_item(const S *__restrict__ src, S *__restrict__ dst, const KParams &P,
                                          int item, int ne, int lane)
{
    if (item >= ne) {
        wall_node<S>(src, dst, P, (item - ne) * EDGE_BX + lane);
        return;
    }
    const Cols c = step_cols<S>(P);
    const int r = item / c.nseg, s = item - r * c.nseg;
    int xbeg, xend;
    if (c.split) {
        xbeg = (s == 0) ? 0 : c.xb;
        xend = (s == 0) ? c.xa : P.nx;
    } else {
        xbeg = s * c.span_e;
        xend = min(P.nx, xbeg + c.span_e);
    }
    bulk_tile<S, true, EDGE_BX, 1>(src, dst, P, rows_begin(P) + r, xbeg, xend, lane);
}

template <typename S, typename R>
__global__ void __launch_bounds__(EDGE_BX)
k_step_edge(const S *__restrict__ src, S *__restrict__ dst, KParams P, int ne)
{
    edge_item<S>(src, dst, P, blockIdx.x, ne, threadIdx.x);
}

// ---------------------------------------------------------------------------------
// Batched step over many problems: block b works on item items[b] = (problem, tile) of
// the bulk update, or (problem, wall block) of the wall update.  parity selects which
// of each problem's two buffers is the source.
// ---------------------------------------------------------------------------------
// Candidate block widths of the batched update (picked per batch by timing them).
constexpr int BATCH_WIDTHS[3] = {64, 128, 256};
constexpr int CHECK_BX = 64;

template <typename S, bool WALLS, int BX>
__global__ void __launch_bounds__(BX)
k_batch_bulk(const BatchProblem *__restrict__ probs, const int2 *__restrict__ items, int parity)
{
    const int2 it = items[blockIdx.x];
    const BatchProblem &B = probs[it.x];
    const int y = it.y / B.tiles_x;
    const int xbeg = (it.y - y * B.tiles_x) * block_span<S, BX>();
    bulk_tile<S, WALLS, BX>(static_cast<const S *>(B.buf[parity]),
                            static_cast<S *>(B.buf[parity ^ 1]), B.P, y, xbeg, B.P.nx, threadIdx.x);
}

template <typename S>
__global__ void __launch_bounds__(WALL_B)
k_batch_wall(const BatchProblem *__restrict__ probs, const int2 *__restrict__ items, int parity)
{
    const int2 it = items[blockIdx.x];
    const BatchProblem &B = probs[it.x];
    wall_node<S>(static_cast<const S *>(B.buf[parity]), static_cast<S *>(B.buf[parity ^ 1]), B.P,
                 it.y * WALL_B + threadIdx.x);
}

// Non-finite check of each problem's current populations (one flag per problem; a block
// that finds a bad value stores 1, stores of the same value from several blocks are
// harmless).
// Items are (problem, segment) with segments of CHECK_BX * NPT nodes of a row.
template <typename S>
__global__ void __launch_bounds__(CHECK_BX)
k_batch_check(const BatchProblem *__restrict__ probs, const int2 *__restrict__ items, int parity,
              int *flags)
{
    const int2 it = items[blockIdx.x];
    const BatchProblem &B = probs[it.x];
    const KParams &P = B.P;
    constexpr int NPT = Npt<S>::v;
    const S *src = static_cast<const S *>(B.buf[parity]);
    const int tx = (P.nx + CHECK_BX * NPT - 1) / (CHECK_BX * NPT);
    const int y = it.y / tx;
    const int x0 = (it.y - y * tx) * (CHECK_BX * NPT) + threadIdx.x;
    bool bad = false;
    for (int k = 0; k < NPT; ++k) {
        const int x = x0 + k * CHECK_BX;
        if (x >= P.nx) continue;
        for (int q = 0; q < 18; ++q)
            bad |= !isfinite(float(Store<S>::ld(src + pidx<S>(P, q, x, y), 1.0f)));
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) flags[it.x] = 1;
}

// ---------------------------------------------------------------------------------
// Macroscopic fields at the current time (same node code as the step, no collision)
// ---------------------------------------------------------------------------------
struct FieldOut {
    void *ptr[9];   // p, ux, uy, T, Sxx, Sxy, Syy, dTdx, dTdy
    int f32;
};

template <typename R>
__device__ __forceinline__ void write_fields(const FieldOut &o, const KParams &P, int x, int y,
                                             const Macro<R> &m)
{
    const long long n = (long long)y * P.nx + x;
    const double v[9] = {double(m.p), double(m.ux), double(m.uy), P.T0 + double(m.Td),
                         double(m.Sxx), double(m.Sxy), double(m.Syy), double(m.gx),
                         double(m.gy)};
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        if (!o.ptr[q]) continue;
        if (o.f32) static_cast<float *>(o.ptr[q])[n] = float(v[q]);
        else static_cast<double *>(o.ptr[q])[n] = v[q];
    }
}

template <typename S, typename R>
__global__ void __launch_bounds__(BULK_BX)
k_fields_bulk(const S *__restrict__ src, KParams P, FieldOut o)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= P.nx || on_wall(P, x, y)) return;
    using M = typename Prec<S>::M;
    M f[9], g[9];
    gather<S, M>(src, P, x, y, f, g);
    Macro<M> m;
    node_macro_full<M>(f, g, M(P.T0), make_cst<M>(P), eps_at<M>(P, x, y), m);
    write_fields<M>(o, P, x, y, m);
}

template <typename S, typename R>
__global__ void __launch_bounds__(WALL_B)
k_fields_wall(const S *__restrict__ src, KParams P, FieldOut o)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    int x, y;
    if (s >= P.nwall || !wall_slot(P, s, x, y)) return;
    using M = typename Prec<S>::M;
    M f[9], g[9];
    Macro<M> mb;   // a wall node's fields are the state the boundary scheme assigns
    wall_populations<S, M>(src, P, make_cst<M>(P), x, y, f, g, mb);
    write_fields<M>(o, P, x, y, mb);
}

// ---------------------------------------------------------------------------------
// Residual against a snapshot (FP64, fixed-order reduction) and non-finite detection.
// Each block writes 5 partial sums: |du|_2, |u|_2, |dT|, |T|, count of non-finite.
// ---------------------------------------------------------------------------------
__device__ __forceinline__ void block_sum5(double v[5], double *out)
{
    __shared__ double sm[5][RED_B];
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 5; ++q) sm[q][t] = v[q];
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (t < s) {
#pragma unroll
            for (int q = 0; q < 5; ++q) sm[q][t] += sm[q][t + s];
        }
        __syncthreads();
    }
    if (t < 5) out[t] = sm[t][0];
}

template <typename R>
__device__ __forceinline__ void resid_node(const KParams &P, int x, int y, const R *f, const R *g,
                                           const Macro<R> &m, double *snap, double v[5])
{
    const long long n = (long long)y * P.nx + x;
    const long long N = (long long)P.nx * P.ny;
    bool bad = false;
#pragma unroll
    for (int i = 0; i < 9; ++i) bad |= !isfinite(double(f[i])) || !isfinite(double(g[i]));
    const double ux = double(m.ux), uy = double(m.uy), T = P.T0 + double(m.Td);
    bad |= !isfinite(ux) || !isfinite(uy) || !isfinite(T);
    const double dux = ux - snap[n], duy = uy - snap[N + n];
    v[0] = sqrt(dux * dux + duy * duy);
    v[1] = sqrt(ux * ux + uy * uy);
    v[2] = fabs(T - snap[2 * N + n]);
    v[3] = fabs(T);
    v[4] = bad ? 1.0 : 0.0;
    snap[n] = ux;
    snap[N + n] = uy;
    snap[2 * N + n] = T;
}

template <typename S, typename R>
__global__ void __launch_bounds__(RED_B)
k_resid_bulk(const S *__restrict__ src, KParams P, double *snap, double *partial)
{
    // 1-D over nodes so that every block has a fixed slot in the partial array
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double v[5] = {0, 0, 0, 0, 0};
    if (idx < (long long)P.nx * P.ny) {
        const int x = int(idx % P.nx), y = int(idx / P.nx);
        if (!on_wall(P, x, y)) {
            using M = typename Prec<S>::M;
            M f[9], g[9];
            gather<S, M>(src, P, x, y, f, g);
            Macro<M> m;
            node_macro_full<M>(f, g, M(P.T0), make_cst<M>(P), eps_at<M>(P, x, y), m);
            resid_node<M>(P, x, y, f, g, m, snap, v);
        }
    }
    block_sum5(v, partial + 5 * (long long)blockIdx.x);
}

template <typename S, typename R>
__global__ void __launch_bounds__(RED_B)
k_resid_wall(const S *__restrict__ src, KParams P, double *snap, double *partial)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    double v[5] = {0, 0, 0, 0, 0};
    int x, y;
    if (s < P.nwall && wall_slot(P, s, x, y)) {
        using M = typename Prec<S>::M;
        M f[9], g[9];
        Macro<M> mb;
        wall_populations<S, M>(src, P, make_cst<M>(P), x, y, f, g, mb);
        resid_node<M>(P, x, y, f, g, mb, snap, v);
    }
    block_sum5(v, partial + 5 * (long long)blockIdx.x);
}

// Sums nparts partial 5-vectors in a fixed order (one block).
__global__ void __launch_bounds__(RED_B) k_sum_partials(const double *partial, int nparts, double *out)
{
    double v[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nparts; b += blockDim.x)
#pragma unroll
        for (int q = 0; q < 5; ++q) v[q] += partial[5 * (long long)b + q];
    block_sum5(v, out);
}

// ---------------------------------------------------------------------------------
// Nusselt number (Eq. AvNuss): T on the three node layers next to a wall, one-sided
// second-order derivative, trapezoid rule; FP64, fixed-order reduction in one block.
// ---------------------------------------------------------------------------------
template <typename S, typename R>
__device__ __forceinline__ double node_Td_interior(const S *__restrict__ src, const KParams &P,
                                                   const Cst<R> &k, int x, int y)
{
    R f[9], g[9];
    gather<S, R>(src, P, x, y, f, g);
    R sg = R(0);
#pragma unroll
    for (int i = 0; i < 9; ++i) sg += g[i];
    return double((sg + k.halfQ) * k.isig);
}

template <typename S, typename R>
__device__ __forceinline__ double node_Td(const S *__restrict__ src, const KParams &P,
                                          const Cst<R> &k, int x, int y)
{
    if (!on_wall(P, x, y)) return node_Td_interior<S, R>(src, P, k, x, y);
    // wall node: the boundary scheme sets T(x_b) = T_b exactly (sum of g^eq is sigma T)
    const WallInfo w = wall_info(P, x, y);
    int dir = -1;
    if (w.xw >= 0 && P.wall_kind[w.xw] == 0) dir = w.xw;
    else if (w.yw >= 0 && P.wall_kind[w.yw] == 0) dir = w.yw;
    if (dir >= 0) return P.wall_T[dir] - P.T0;
    const double Tdf = node_Td_interior<S, R>(src, P, k, x + w.dx, y + w.dy);
    const double Tdff = node_Td_interior<S, R>(src, P, k, x + 2 * w.dx, y + 2 * w.dy);
    double dn = 0.0;
    if (w.xw >= 0) dn += P.wall_dTdn[w.xw];
    if (w.yw >= 0) dn += P.wall_dTdn[w.yw];
    return (4.0 * Tdf - Tdff - 2.0 * dn) / 3.0;
}

template <typename S, typename R>
__global__ void __launch_bounds__(RED_B)
k_nusselt(const S *__restrict__ src, KParams P, int wall, double L, double dT, double *out)
{
    using M = typename Prec<S>::M;
    const Cst<M> &k = make_cst<M>(P);
    const int along = (wall < 2) ? P.ny : P.nx;
    double acc = 0.0;
    for (int j = threadIdx.x; j < along; j += blockDim.x) {
        double t0, t1, t2, sgn;
        if (wall == 0) { t0 = node_Td<S, M>(src, P, k, 0, j); t1 = node_Td<S, M>(src, P, k, 1, j); t2 = node_Td<S, M>(src, P, k, 2, j); sgn = 1.0; }
        else if (wall == 1) { t0 = node_Td<S, M>(src, P, k, P.nx - 1, j); t1 = node_Td<S, M>(src, P, k, P.nx - 2, j); t2 = node_Td<S, M>(src, P, k, P.nx - 3, j); sgn = -1.0; }
        else if (wall == 2) { t0 = node_Td<S, M>(src, P, k, j, 0); t1 = node_Td<S, M>(src, P, k, j, 1); t2 = node_Td<S, M>(src, P, k, j, 2); sgn = 1.0; }
        else { t0 = node_Td<S, M>(src, P, k, j, P.ny - 1); t1 = node_Td<S, M>(src, P, k, j, P.ny - 2); t2 = node_Td<S, M>(src, P, k, j, P.ny - 3); sgn = -1.0; }
        const double d = sgn * (-3.0 * t0 + 4.0 * t1 - t2) * 0.5;
        const double nu = -L * d / dT;
        acc += (j == 0 || j == along - 1) ? 0.5 * nu : nu;
    }
    double v[5] = {acc, 0, 0, 0, 0};
    __shared__ double res[5];
    block_sum5(v, res);
    if (threadIdx.x == 0) out[0] = res[0] / double(along - 1);
}

// ---------------------------------------------------------------------------------
// State conversion: stored deviations <-> raw FP64 populations [2][9][ny][nx]
// ---------------------------------------------------------------------------------
template <typename S>
__global__ void __launch_bounds__(BULK_BX)
k_get_state(const S *__restrict__ src, KParams P, double *__restrict__ out)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= P.nx) return;
    const long long N = (long long)P.nx * P.ny, n = (long long)y * P.nx + x;
    for (int q = 0; q < 18; ++q) {
        double v = double(Store<S>::ld(src + pidx<S>(P, q, x, y), P.hinv));
        if (q == 0) v += 1.0;
        if (q >= 9) v += Wd(q - 9) * P.sigma * P.T0;
        out[q * N + n] = v;
    }
}

template <typename S>
__global__ void __launch_bounds__(BULK_BX)
k_set_state(S *__restrict__ dst, KParams P, const double *__restrict__ in)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= P.nx) return;
    const long long N = (long long)P.nx * P.ny, n = (long long)y * P.nx + x;
    for (int q = 0; q < 18; ++q) {
        double v = in[q * N + n];
        if (q == 0) v -= 1.0;
        if (q >= 9) v -= Wd(q - 9) * P.sigma * P.T0;
        Store<S>::st(dst + pidx<S>(P, q, x, y), decltype(Store<S>::ld(dst, 0.f))(v), P.hscale);
    }
}

// ---------------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------------
static dim3 bulk_grid(const KParams &P) { return dim3((P.nx + BULK_BX - 1) / BULK_BX, P.ny); }
static int wall_blocks(const KParams &P, int b) { return (P.nwall + b - 1) / b; }

template <typename S, typename R>
static hipError_t launch_init_t(void *dst, const KParams &P, const double *T, const double *p,
                                const double *ux, const double *uy, hipStream_t st)
{
    hipLaunchKernelGGL((k_init<S, R>), bulk_grid(P), dim3(BULK_BX), 0, st, (S *)dst, P, T, p, ux, uy);
    return hipGetLastError();
}

template <typename S, typename R>
static void launch_interior(const void *src, void *dst, const KParams &P, hipStream_t st)
{
    const int nseg = interior_segments<S>(P);
    const int n = nseg * rows_count(P);
    if (n > 0)
        hipLaunchKernelGGL((k_step_bulk<S, R>), dim3(n), dim3(BULK_BX), 0, st, (const S *)src, (S *)dst, P, nseg);
}

template <typename S, typename R>
static void launch_edges(const void *src, void *dst, const KParams &P, hipStream_t st)
{
    const int ne = step_cols<S>(P).nseg * rows_count(P);
    const int nw = (P.nwall_rows + EDGE_BX - 1) / EDGE_BX;
    if (ne + nw > 0)
        hipLaunchKernelGGL((k_step_edge<S, R>), dim3(ne + nw), dim3(EDGE_BX), 0, st, (const S *)src, (S *)dst, P, ne);
}

template <typename S, typename R>
static hipError_t launch_step_t(const void *src, void *dst, const KParams &P, hipStream_t st)
{
    launch_interior<S, R>(src, dst, P, st);
    launch_edges<S, R>(src, dst, P, st);
    return hipGetLastError();
}

template <typename S, typename R>
static hipError_t launch_step_bulk_t(const void *src, void *dst, const KParams &P, hipStream_t st)
{
    launch_interior<S, R>(src, dst, P, st);
    return hipGetLastError();
}

template <typename S, typename R>
static hipError_t launch_step_wall_t(const void *src, void *dst, const KParams &P, hipStream_t st)
{
    launch_edges<S, R>(src, dst, P, st);
    return hipGetLastError();
}

template <typename S, typename R>
static hipError_t launch_fields_t(const void *src, const KParams &P, void *const out[9], int f32,
                                  hipStream_t st)
{
    FieldOut o;
    for (int q = 0; q < 9; ++q) o.ptr[q] = out[q];
    o.f32 = f32;
    hipLaunchKernelGGL((k_fields_bulk<S, R>), bulk_grid(P), dim3(BULK_BX), 0, st, (const S *)src, P, o);
    if (P.nwall > 0)
        hipLaunchKernelGGL((k_fields_wall<S, R>), dim3(wall_blocks(P, WALL_B)), dim3(WALL_B), 0, st,
                           (const S *)src, P, o);
    return hipGetLastError();
}

template <typename S, typename R>
static hipError_t launch_resid_t(const void *src, const KParams &P, double *snap, double *partial,
                                 double *out, hipStream_t st)
{
    const long long N = (long long)P.nx * P.ny;
    const int nb = int((N + RED_B - 1) / RED_B);
    const int nw = P.nwall > 0 ? wall_blocks(P, RED_B) : 0;
    hipLaunchKernelGGL((k_resid_bulk<S, R>), dim3(nb), dim3(RED_B), 0, st, (const S *)src, P, snap, partial);
    if (nw > 0)
        hipLaunchKernelGGL((k_resid_wall<S, R>), dim3(nw), dim3(RED_B), 0, st, (const S *)src, P, snap,
                           partial + 5 * (long long)nb);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(RED_B), 0, st, (const double *)partial, nb + nw, out);
    return hipGetLastError();
}

template <typename S, typename R>
static hipError_t launch_nusselt_t(const void *src, const KParams &P, int wall, double L, double dT,
                                   double *out, hipStream_t st)
{
    hipLaunchKernelGGL((k_nusselt<S, R>), dim3(1), dim3(RED_B), 0, st, (const S *)src, P, wall, L, dT, out);
    return hipGetLastError();
}

// Non-finite detector: *flag |= 1 if any population of a node of the grid is NaN or
// infinite (padding columns of the last tile are not read).
template <typename S>
__global__ void __launch_bounds__(BULK_BX) k_check(const S *__restrict__ src, KParams P, int *__restrict__ flag)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= P.nx) return;
    bool bad = false;
    for (int q = 0; q < 18; ++q) {
        const float v = float(Store<S>::ld(src + pidx<S>(P, q, x, y), P.hinv));
        bad = bad || !__builtin_isfinite(v);
    }
    if (bad) atomicOr(flag, 1);
}

template <typename S>
static hipError_t launch_check_t(const void *buf, const KParams &P, int *flag, hipStream_t st)
{
    hipLaunchKernelGGL((k_check<S>), bulk_grid(P), dim3(BULK_BX), 0, st, (const S *)buf, P, flag);
    return hipGetLastError();
}

template <typename S>
static hipError_t launch_state_t(void *buf, const KParams &P, double *io, bool get, hipStream_t st)
{
    if (get) hipLaunchKernelGGL((k_get_state<S>), bulk_grid(P), dim3(BULK_BX), 0, st, (const S *)buf, P, io);
    else hipLaunchKernelGGL((k_set_state<S>), bulk_grid(P), dim3(BULK_BX), 0, st, (S *)buf, P, (const double *)io);
    return hipGetLastError();
}

#define LBM_DISPATCH(storage, CALL_F64, CALL_F32, CALL_F16)   \
    switch (storage) {                                         \
    case 0: return CALL_F64;                                   \
    case 1: return CALL_F32;                                   \
    case 2: return CALL_F16;                                   \
    default: return hipErrorInvalidValue;                      \
    }

hipError_t launch_init(int storage, void *dst, const KParams &P, const double *T, const double *p,
                       const double *ux, const double *uy, hipStream_t st)
{
    LBM_DISPATCH(storage, (launch_init_t<double, double>(dst, P, T, p, ux, uy, st)),
                 (launch_init_t<float, float>(dst, P, T, p, ux, uy, st)),
                 (launch_init_t<__half, float>(dst, P, T, p, ux, uy, st)))
}

hipError_t launch_step(int storage, const void *src, void *dst, const KParams &P, hipStream_t st)
{
    LBM_DISPATCH(storage, (launch_step_t<double, double>(src, dst, P, st)),
                 (launch_step_t<float, float>(src, dst, P, st)),
                 (launch_step_t<__half, float>(src, dst, P, st)))
}

hipError_t launch_step_bulk(int storage, const void *src, void *dst, const KParams &P, hipStream_t st)
{
    LBM_DISPATCH(storage, (launch_step_bulk_t<double, double>(src, dst, P, st)),
                 (launch_step_bulk_t<float, float>(src, dst, P, st)),
                 (launch_step_bulk_t<__half, float>(src, dst, P, st)))
}

hipError_t launch_step_wall(int storage, const void *src, void *dst, const KParams &P, hipStream_t st)
{
    LBM_DISPATCH(storage, (launch_step_wall_t<double, double>(src, dst, P, st)),
                 (launch_step_wall_t<float, float>(src, dst, P, st)),
                 (launch_step_wall_t<__half, float>(src, dst, P, st)))
}

hipError_t launch_fields(int storage, const void *src, const KParams &P, void *const out[9], int f32,
                         hipStream_t st)
{
    LBM_DISPATCH(storage, (launch_fields_t<double, double>(src, P, out, f32, st)),
                 (launch_fields_t<float, float>(src, P, out, f32, st)),
                 (launch_fields_t<__half, float>(src, P, out, f32, st)))
}

hipError_t launch_residual(int storage, const void *src, const KParams &P, double *snap,
                           double *partial, double *out, hipStream_t st)
{
    LBM_DISPATCH(storage, (launch_resid_t<double, double>(src, P, snap, partial, out, st)),
                 (launch_resid_t<float, float>(src, P, snap, partial, out, st)),
                 (launch_resid_t<__half, float>(src, P, snap, partial, out, st)))
}

hipError_t launch_nusselt(int storage, const void *src, const KParams &P, int wall, double L,
                          double dT, double *out, hipStream_t st)
{
    LBM_DISPATCH(storage, (launch_nusselt_t<double, double>(src, P, wall, L, dT, out, st)),
                 (launch_nusselt_t<float, float>(src, P, wall, L, dT, out, st)),
                 (launch_nusselt_t<__half, float>(src, P, wall, L, dT, out, st)))
}

hipError_t launch_check(int storage, const void *buf, const KParams &P, int *flag, hipStream_t st)
{
    LBM_DISPATCH(storage, (launch_check_t<double>(buf, P, flag, st)), (launch_check_t<float>(buf, P, flag, st)),
                 (launch_check_t<__half>(buf, P, flag, st)))
}

hipError_t launch_state(int storage, void *buf, const KParams &P, double *io, bool get, hipStream_t st)
{
    LBM_DISPATCH(storage, (launch_state_t<double>(buf, P, io, get, st)),
                 (launch_state_t<float>(buf, P, io, get, st)),
                 (launch_state_t<__half>(buf, P, io, get, st)))
}

template <typename S, int BX>
static hipError_t batch_step_w(const BatchProblem *probs, const int2 *bulk_items, int nbulk,
                               const int2 *edge_items, int nedge, const int2 *wall_items, int nwall,
                               int parity, hipStream_t st)
{
    if (nbulk > 0)
        hipLaunchKernelGGL((k_batch_bulk<S, false, BX>), dim3(nbulk), dim3(BX), 0, st, probs, bulk_items, parity);
    if (nedge > 0)
        hipLaunchKernelGGL((k_batch_bulk<S, true, BX>), dim3(nedge), dim3(BX), 0, st, probs, edge_items, parity);
    if (nwall > 0)
        hipLaunchKernelGGL((k_batch_wall<S>), dim3(nwall), dim3(WALL_B), 0, st, probs, wall_items, parity);
    return hipGetLastError();
}

template <typename S>
static hipError_t batch_step_t(int bx, const BatchProblem *probs, const int2 *bulk_items, int nbulk,
                               const int2 *edge_items, int nedge, const int2 *wall_items, int nwall,
                               int parity, hipStream_t st)
{
    switch (bx) {
    case 64: return batch_step_w<S, 64>(probs, bulk_items, nbulk, edge_items, nedge, wall_items, nwall, parity, st);
    case 128: return batch_step_w<S, 128>(probs, bulk_items, nbulk, edge_items, nedge, wall_items, nwall, parity, st);
    case 256: return batch_step_w<S, 256>(probs, bulk_items, nbulk, edge_items, nedge, wall_items, nwall, parity, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_step(int storage, int bx, const BatchProblem *probs, const int2 *bulk_items, int nbulk,
                             const int2 *edge_items, int nedge, const int2 *wall_items, int nwall,
                             int parity, hipStream_t st)
{
    LBM_DISPATCH(storage,
                 (batch_step_t<double>(bx, probs, bulk_items, nbulk, edge_items, nedge, wall_items, nwall, parity, st)),
                 (batch_step_t<float>(bx, probs, bulk_items, nbulk, edge_items, nedge, wall_items, nwall, parity, st)),
                 (batch_step_t<__half>(bx, probs, bulk_items, nbulk, edge_items, nedge, wall_items, nwall, parity, st)))
}

template <typename S, int BX>
static void batch_kernels_w(BatchKernels &k)
{
    k.bulk = (const void *)k_batch_bulk<S, false, BX>;
    k.edge = (const void *)k_batch_bulk<S, true, BX>;
    k.wall = (const void *)k_batch_wall<S>;
    k.bulk_threads = BX;
    k.wall_threads = WALL_B;
}

template <typename S>
static bool batch_kernels_t(int bx, BatchKernels &k)
{
    switch (bx) {
    case 64: batch_kernels_w<S, 64>(k); return true;
    case 128: batch_kernels_w<S, 128>(k); return true;
    case 256: batch_kernels_w<S, 256>(k); return true;
    default: return false;
    }
}

bool batch_kernels(int storage, int bx, BatchKernels &k)
{
    switch (storage) {
    case 0: return batch_kernels_t<double>(bx, k);
    case 1: return batch_kernels_t<float>(bx, k);
    case 2: return batch_kernels_t<__half>(bx, k);
    default: return false;
    }
}

int batch_width(int i) { return (i >= 0 && i < 3) ? BATCH_WIDTHS[i] : 0; }

template <typename S>
static hipError_t batch_check_t(const BatchProblem *probs, const int2 *items, int n, int parity,
                                int *flags, hipStream_t st)
{
    if (n > 0)
        hipLaunchKernelGGL((k_batch_check<S>), dim3(n), dim3(CHECK_BX), 0, st, probs, items, parity, flags);
    return hipGetLastError();
}

hipError_t launch_batch_check(int storage, const BatchProblem *probs, const int2 *items, int n,
                              int parity, int *flags, hipStream_t st)
{
    LBM_DISPATCH(storage, (batch_check_t<double>(probs, items, n, parity, flags, st)),
                 (batch_check_t<float>(probs, items, n, parity, flags, st)),
                 (batch_check_t<__half>(probs, items, n, parity, flags, st)))
}

static int npt_of(int storage)
{
    return storage == 0 ? Npt<double>::v : (storage == 1 ? Npt<float>::v : Npt<__half>::v);
}

static int wspan_of(int storage)
{
    return storage == 0 ? Wspan<double>::v : (storage == 1 ? Wspan<float>::v : Wspan<__half>::v);
}

int batch_tiles_x(int storage, const KParams &P, int bx)
{
    const int span = (bx / 64) * wspan_of(storage) * npt_of(storage);
    return (P.nx + span - 1) / span;
}

int batch_check_tiles_x(int storage, const KParams &P)
{
    const int span = CHECK_BX * npt_of(storage);
    return (P.nx + span - 1) / span;
}

int wall_block_size() { return WALL_B; }

template <typename S> static long long interior_nodes_t(const KParams &P)
{
    const Cols c = step_cols<S>(P);
    return (long long)(c.xb - c.xa) * rows_count(P);
}

long long interior_nodes(int storage, const KParams &P)
{
    return storage == 0 ? interior_nodes_t<double>(P)
                        : (storage == 1 ? interior_nodes_t<float>(P) : interior_nodes_t<__half>(P));
}

long long residual_partials(const KParams &P)
{
    const long long N = (long long)P.nx * P.ny;
    return (N + RED_B - 1) / RED_B + (P.nwall + RED_B - 1) / RED_B;
}

}  // namespace lbm
