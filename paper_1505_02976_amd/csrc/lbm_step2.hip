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
// Three instances of the walk, by what lies in a wavefront's reach: lean (no wall, no
// boundary-scheme code), xwall (the vertical walls x = 0, x = nx - 1 only: the wall
// column's intermediate rows are computed before the walk, one lane per row, and its final
// rows after it, from values the reference lanes leave in LDS) and full (everything else:
// the boundary scheme inline, with the wall node taking its reference node's pulled
// populations from the neighbouring lanes, as in the one-step kernel).  The walled rows
// y = 0 and y = ny - 1 need the intermediate populations of three more rows for their
// reference nodes, so the full instance, which runs the bands of rows 0-3 and ny-4..ny-1,
// writes P1 of those rows to a small scratch grid and a last launch finishes the two
// walled rows.  A pass is two launches over wavefront lists built on the host: the main
// one (xwall and lean wavefronts, the instance chosen per wavefront) and the full one, then
// the walled rows.
//
// Every node update is the one-step node code with the same inputs, so two steps here are
// bitwise identical to two one-step launches (FP16 storage rounds P1 to the stored format
// before it is used, as the one-step path does by storing it).
//
// FP32 and FP64 storage use tiles of 62 columns, so every wavefront's 62 outputs fill one
// tile segment per direction (unaligned 62-lane writes into wider tiles ran at 3.3 TB/s
// against 5.4 aligned).  Each pass reads about 1.3 times the populations it writes (the two
// halo columns and the two halo rows of intermediate state are recomputed) and issues
// about 2.3 node updates per output node, so it sits near both the memory and the vector
// issue limit; it pays off against one step per pass for FP32 and FP64 storage, not for
// FP16, whose one-step kernel is already bound by vector issue.
#include <vector>

#include "lbm_kernels.h"

namespace lbm {

constexpr int S2_TY = 8;              // output rows per wavefront

constexpr int S2_OUT = 62;            // output columns per wavefront
constexpr int S2_B = 256;             // threads per block (independent wavefronts)
static_assert(S2_B / 64 == STEP2_WAVES_PER_BLOCK, "wavefronts per block");

// The lean instance gathers the next row's populations while it updates the current one
// (one more set of 18 registers).  For FP64 it fits (253 VGPRs, two wavefronts per SIMD as
// without it) but measured 2.4 % slower, so FP64 gathers each row when it needs it.
template <typename S> struct S2Prefetch { static constexpr bool v = true; };
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
template <typename S, typename R, bool PRE>
__device__ __forceinline__ void p1_node(const S *__restrict__ src, const KParams &P, int x, int y, R *f, R *g)
{
    if (on_wall(P, x, y)) {
        Macro<R> mb;
        wall_populations<S, R, PRE>(src, P, make_cst<R>(P), x, y, f, g, mb);
        wall_collide<R, PRE>(f, g, mb, P, x, y);
    } else {
        gather<S, R>(src, P, x, y, f, g);
        node_update<R, typename Prec<S>::M, PRE>(f, g, P, x, y);
    }
}

// Instance that runs the wavefront of column chunk cxi and row band cyi: lean (no wall
// node, no node whose intermediate state goes to the scratch grid, no row outside the
// grid: no boundary-scheme code), xwall (walls x = 0 or x = nx - 1 only: the wall column's
// intermediate rows are computed lane-parallel before the walk and its final rows after
// it), full (everything else).
// First output column of column chunk cxi.  Walls in x: chunks start on the 62-column
// tiles, so that their loads and stores fill whole tile segments; the last one may reach
// past x = nx - 1 (those lanes idle) and starts at least three columns before the wall, so
// that the wall node's reference nodes x_f, x_ff are output lanes.  Periodic x: the last
// chunk ends at x = nx - 1 (it may overlap its neighbour; grids narrower than 62 wrap).
__host__ __device__ __forceinline__ int s2_x0(const KParams &P, int cxi)
{
    return P.px ? min(cxi * S2_OUT, P.nx - S2_OUT) : min(cxi * S2_OUT, P.nx - 3);
}

// Row bands.  Periodic y: bands of S2_TY rows from y = 0 (the last one may be shorter).
// Walls in y: band 0 holds rows 0-3 and the last band rows ny-4..ny-1, both for the full
// instance (the walled rows, and the intermediate rows their boundary scheme reads from the
// scratch grid); between them bands of S2_TY rows from y = 4, the last one ending at ny - 4
// (their halo rows 3 and ny - 4 are recomputed but not written to the scratch grid).
__host__ __device__ __forceinline__ int s2_nbands(const KParams &P)
{
    return P.py ? (P.ny + S2_TY - 1) / S2_TY : 2 + (P.ny - 8 + S2_TY - 1) / S2_TY;
}

__host__ __device__ __forceinline__ void s2_band(const KParams &P, int cyi, int &Y0, int &Y1)
{
    if (P.py) {
        Y0 = cyi * S2_TY;
        Y1 = min(Y0 + S2_TY, P.ny);
    } else if (cyi == 0) {
        Y0 = 0;
        Y1 = 4;
    } else if (cyi == s2_nbands(P) - 1) {
        Y0 = P.ny - 4;
        Y1 = P.ny;
    } else {
        Y0 = 4 + (cyi - 1) * S2_TY;
        Y1 = min(Y0 + S2_TY, P.ny - 4);
    }
}

__host__ __device__ __forceinline__ int s2_kind(const KParams &P, int cxi, int cyi)
{
    const int X0 = s2_x0(P, cxi);
    const bool xin = P.px || (X0 - 1 >= 1 && X0 + S2_OUT <= P.nx - 2);
    const bool yin = P.py || (cyi > 0 && cyi < s2_nbands(P) - 1);
    return yin ? (xin ? STEP2_LEAN : STEP2_XWALL) : STEP2_FULL;
}

// LDS of one xwall wavefront: intermediate populations of the (up to two) wall columns for
// the band's S2_TY + 2 intermediate rows, then per output row the pulled populations of
// the wall node's reference node x_f and Td of x_ff.
static_assert(2 * (S2_TY + 2) <= 64, "xwall: one lane per intermediate row of each wall column");
constexpr int S2_LDS_P1 = 2 * (S2_TY + 2) * 18;
constexpr int S2_LDS = S2_LDS_P1 + 2 * S2_TY * 19;

// LDS writes of some lanes made visible to the other lanes of the wavefront.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wavefront's walk: column chunk cxi, row band cyi.  lds: S2_LDS values of the
// wavefront's own (xwall instance only).  PRIO: the wavefront raises its issue priority
// while it issues the next row's loads (lean and xwall instances with the row gathered
// ahead), so that they leave before the arithmetic of the other wavefronts on its SIMD.
// The single-grid launch takes it (FP32 on the 4096^2 cavity: 533 against 536 us); the
// batched one ran 0.4 % slower with it, and FP16's one-step kernel, bound by vector
// issue, 5 % slower with the same around its gathers.
template <typename S, int MODE, bool PRE, bool PRIO = false>
__device__ __forceinline__ void march2(const S *__restrict__ src, S *__restrict__ dst, S *__restrict__ scr,
                                       const KParams &P, const KParams &Pm, int cxi, int cyi, int lane,
                                       typename Prec<S>::R *lds)
{
    using R = typename Prec<S>::R;
    using M = typename Prec<S>::M;
    constexpr bool FULL = MODE == STEP2_FULL, XW = MODE == STEP2_XWALL;
    const int X0 = s2_x0(P, cxi);
    int x = X0 - 1 + lane;                               // X0 < 0 when x is periodic, nx < 62
    bool xok = true;
    if (P.px) x = ((x % P.nx) + P.nx) % P.nx;
    else xok = x >= 0 && x < P.nx;
    const bool xout = lane >= 1 && lane <= S2_OUT && xok;
    const bool vwall = xok && !P.px && (x == 0 || x == P.nx - 1);
    int Y0, Y1;
    s2_band(P, cyi, Y0, Y1);
    // xwall: lanes outside the grid compute on the nearest column (results unused); wl[0],
    // wl[1] = lanes of the columns x = 0 and x = nx - 1, -1 when not in this wavefront
    const int xs = XW ? min(max(x, 0), P.nx - 1) : x;
    const int wl0 = XW && X0 <= 1 ? 1 - X0 : -1;
    const int wl1 = XW && P.nx - X0 <= 63 ? P.nx - X0 : -1;
    R *const P1w = lds, *const REF = lds + S2_LDS_P1;
    if constexpr (XW) {
        // intermediate populations of the wall nodes for rows Y0 - 1 .. Y1, one per lane
        const int side = lane / (S2_TY + 2), r = lane % (S2_TY + 2);
        const int wl = side == 0 ? wl0 : wl1;
        const int yy = Y0 - 1 + r;
        if (side < 2 && wl >= 0 && yy <= Y1) {
            const int yr = P.py ? (yy + P.ny) % P.ny : yy;
            R f[9], g[9];
            p1_node<S, R, PRE>(src, P, side == 0 ? 0 : P.nx - 1, yr, f, g);
            R *q = P1w + (side * (S2_TY + 2) + r) * 18;
#pragma unroll
            for (int i = 0; i < 9; ++i) { q[i] = as_stored<S, R>(f[i], P); q[9 + i] = as_stored<S, R>(g[i], P); }
        }
        wave_sync();
    }

    // kept values: U2 = (2,5,6) of P1(yy-2), U1 = (2,5,6) and C1 = (0,1,3) of P1(yy-1),
    // already shifted in x to where the final step pulls them
    R fU2[3], gU2[3], fU1[3], gU1[3], fC1[3], gC1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) fU2[k] = gU2[k] = fU1[k] = gU1[k] = fC1[k] = gC1[k] = R(0);

    constexpr bool PF = !FULL && S2Prefetch<S>::v;   // lean and xwall
    R nf[9], ng[9];                                      // next row, gathered ahead
    if constexpr (PF) gather<S, R>(src, P, xs, P.py ? (Y0 - 1 + P.ny) % P.ny : Y0 - 1, nf, ng);

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
                if constexpr (PRIO) __builtin_amdgcn_s_setprio(3);
                if (yy < Y1) gather<S, R>(src, P, xs, P.py ? (yy + 1) % P.ny : yy + 1, nf, ng);
                if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
            } else {
                gather<S, R>(src, P, xs, yr, f, g);
            }
            node_update<R, M, PRE>(f, g, P, xs, yr);
#pragma unroll
            for (int i = 0; i < 9; ++i) { f[i] = as_stored<S, R>(f[i], P); g[i] = as_stored<S, R>(g[i], P); }
            if (XW && (lane == wl0 || lane == wl1)) {
                const R *q = P1w + ((lane == wl0 ? 0 : 1) * (S2_TY + 2) + (yy - (Y0 - 1))) * 18;
#pragma unroll
                for (int i = 0; i < 9; ++i) { f[i] = q[i]; g[i] = q[9 + i]; }
            }
        } else if (xok && yok) {
            p1_node<S, R, PRE>(src, P, x, yr, f, g);
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
                    Macro<R> mb;
                    wall_from_ref<R, PRE>(P, c, x, orow, eps_at<R>(P, x + dx, orow), eps_at<R>(P, x, orow),
                                     ff, gf, Tn, pf, pg, mb);
                    wall_collide<R, PRE>(pf, pg, mb, P, x, orow);
                    store_node<S, R>(dst, P, x, orow, pf, pg);
                }
            }
            if constexpr (XW) {
                // what the deferred update of the wall node needs: the pulled populations of
                // its reference node x_f and Td of x_ff (as the full instance takes them)
                const int r = o - Y0;
#pragma unroll
                for (int side = 0; side < 2; ++side) {
                    const int wl = side == 0 ? wl0 : wl1, dx = side == 0 ? 1 : -1;
                    if (wl < 1 || wl > S2_OUT) continue;                  // wavefront-uniform
                    R *q = REF + (side * S2_TY + r) * 19;
                    if (lane == wl + dx) {
#pragma unroll
                        for (int i = 0; i < 9; ++i) { q[i] = pf[i]; q[9 + i] = pg[i]; }
                    }
                    if (lane == wl + 2 * dx) {
                        const Cst<R> &c = make_cst<R>(P);
                        R sg = R(0);
#pragma unroll
                        for (int i = 0; i < 9; ++i) sg += pg[i];
                        q[18] = (sg + c.halfQ) * c.isig;
                    }
                }
            }
            if (xout && !((XW || FULL) && vwall)) {     // wall nodes: above, or after the walk
                node_update<R, M, PRE>(pf, pg, P, x, orow);
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
    if constexpr (XW) {
        // final step of the wall nodes of the output rows, one per lane
        wave_sync();
        const int side = lane / S2_TY, r = lane % S2_TY;
        const int wl = side == 0 ? wl0 : wl1;
        const int o = Y0 + r;
        if (side < 2 && wl >= 1 && wl <= S2_OUT && o < Y1) {
            const int orow = P.py ? (o + P.ny) % P.ny : o;
            const int xw = side == 0 ? 0 : P.nx - 1, dx = side == 0 ? 1 : -1;
            const R *q = REF + (side * S2_TY + r) * 19;
            R ff[9], gf[9], pf[9], pg[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) { ff[i] = q[i]; gf[i] = q[9 + i]; }
            const Cst<R> &c = make_cst<R>(P);
            const R Tn = thermal_dirichlet_wall(P, wall_info(P, xw, orow)) < 0 ? q[18] : R(0);
            Macro<R> mb;
            wall_from_ref<R, PRE>(P, c, xw, orow, eps_at<R>(P, xw + dx, orow), eps_at<R>(P, xw, orow), ff, gf, Tn,
                             pf, pg, mb);
            wall_collide<R, PRE>(pf, pg, mb, P, xw, orow);
            store_node<S, R>(dst, P, xw, orow, pf, pg);
        }
    }
}

// Logical block of dispatched block b out of nb: blocks are dealt round-robin to the eight
// XCDs, each with its own L2; this hands every XCD one contiguous range of logical blocks,
// so that the neighbouring wavefronts whose halo columns and rows overlap share an L2.
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    constexpr int X = 8;
    const int per = nb / X, rem = nb % X;
    const int x = b % X, i = b / X;
    return x * per + min(x, rem) + i;
}

// One wavefront's walk with the instance chosen at run time: the main launch runs the lean
// and the xwall wavefronts (both about 135 VGPRs), the full launch the full ones.
// w: wavefront index cyi * ncx + cxi.  PRE: the collision's constant products read from
// the parameter block, or formed once per wavefront in vector registers (node_k).  The
// main launches take the second form: for FP32 the single-grid one holds 137 VGPRs with
// it and 179 with the first, and the batched one, though it holds 113 VGPRs with the first
// form against 131, ran 1.7 % slower with it.  The full launches take the first (FP32:
// 152 VGPRs against 170).
template <typename S, int LAUNCH, bool PRE, bool PRIO = false>
__device__ __forceinline__ void march2_any(const S *__restrict__ src, S *__restrict__ dst, S *__restrict__ scr,
                                           const KParams &P, const KParams &Pm, int w, int ncx, int lane,
                                           typename Prec<S>::R *lds)
{
    const int cxi = w % ncx, cyi = w / ncx;
    if constexpr (LAUNCH == STEP2_FULL)
        march2<S, STEP2_FULL, PRE>(src, dst, scr, P, Pm, cxi, cyi, lane, lds);
    else if (s2_kind(P, cxi, cyi) == STEP2_XWALL)     // wavefront-uniform
        march2<S, STEP2_XWALL, PRE, PRIO>(src, dst, scr, P, Pm, cxi, cyi, lane, lds);
    else
        march2<S, STEP2_LEAN, PRE, PRIO>(src, dst, scr, P, Pm, cxi, cyi, lane, lds);
}

// items: wavefront indices cyi * ncx + cxi of this launch (the main launch lists the xwall
// wavefronts first, so that they start beside the first lean ones rather than at the tail).
// The FP64 full launch is held to two waves per SIMD (at most 256 registers; it needs 236):
// it runs beside the main launch, whose FP64 waves take 217 of a SIMD's 512 registers per
// lane, and a full wave of more than 295 would wait for a SIMD with no main wave on it.
template <typename S, int LAUNCH>
__global__ void __launch_bounds__(S2_B, (LAUNCH == STEP2_FULL && sizeof(S) == 8) ? 2 : 1)
k_step2(const S *__restrict__ src, S *__restrict__ dst, S *__restrict__ scr, KParams P, KParams Pm,
        const int *__restrict__ items, int nitems, int ncx)
{
    using R = typename Prec<S>::R;
    __shared__ R lds[S2_B / 64][LAUNCH == STEP2_FULL ? 1 : S2_LDS];
    const int wi = xcd_block(blockIdx.x, gridDim.x) * (S2_B / 64) + (threadIdx.x >> 6);
    if (wi >= nitems) return;                            // wavefront-uniform
    march2_any<S, LAUNCH, LAUNCH == STEP2_FULL, true>(src, dst, scr, P, Pm, items[wi], ncx, threadIdx.x & 63,
                                                     lds[threadIdx.x >> 6]);
}

// Batched: item (problem, wavefront index); one item list per launch.  The block holds
// blockDim.x / 64 (1, 2 or 4) independent wavefronts, chosen by the batch autotuner; the
// main launch's LDS (S2_LDS values per wavefront) is dynamic shared memory.
template <typename S, int LAUNCH>
__global__ void __launch_bounds__(S2_B)
k_batch_step2(const BatchProblem *__restrict__ probs, const int2 *__restrict__ items, int nitems, int parity)
{
    using R = typename Prec<S>::R;
    extern __shared__ __align__(16) unsigned char s2_lds[];
    // the item, and with it the problem's parameters, are wavefront-uniform: reading them
    // through wavefront-uniform indices keeps them in scalar registers (scalar loads)
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wi = __builtin_amdgcn_readfirstlane(xcd_block(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + wave);
    if (wi >= nitems) return;
    const int2 it = items[wi];
    const int pk = __builtin_amdgcn_readfirstlane(it.x), w = __builtin_amdgcn_readfirstlane(it.y);
    const BatchProblem &B = probs[pk];
    const int ncx = (B.P.nx + S2_OUT - 1) / S2_OUT;
    R *lds = LAUNCH == STEP2_FULL ? nullptr : reinterpret_cast<R *>(s2_lds) + wave * S2_LDS;
    march2_any<S, LAUNCH, LAUNCH == STEP2_FULL>(static_cast<const S *>(B.buf[parity]), static_cast<S *>(B.buf[parity ^ 1]),
                          static_cast<S *>(B.scr), B.P, B.Pm, w, ncx, threadIdx.x & 63, lds);
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
    Macro<M> mb;
    wall_from_ref<M>(P, k, x, y, eps_at<M>(P, x + w.dx, y + w.dy), eps_at<M>(P, x, y), ff, gf, Tdff, f, g, mb);
    wall_collide<M>(f, g, mb, P, x, y);
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

template <typename S, int LAUNCH>
static hipError_t step2_main_t(const void *src, void *dst, void *scr, const KParams &P, const KParams &Pm,
                               const int *items, int nitems, hipStream_t st)
{
    const int ncx = (P.nx + S2_OUT - 1) / S2_OUT;
    const int blocks = (nitems + S2_B / 64 - 1) / (S2_B / 64);
    if (nitems > 0)
        hipLaunchKernelGGL((k_step2<S, LAUNCH>), dim3(blocks), dim3(S2_B), 0, st, (const S *)src, (S *)dst, (S *)scr,
                           P, Pm, items, nitems, ncx);
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
// rows 0-3 and ny-4..ny-1 without overlap).  Grids narrower than a wavefront have one
// column chunk: from x = 0 with lanes past the wall x = nx - 1 idle, or, periodic in x,
// starting left of x = 0 with the lanes wrapped.
bool step2_supported(const KParams &P)
{
    return P.nx >= 4 && P.ny >= 8 && (long long)((P.nx + S2_OUT - 1) / S2_OUT) * s2_nbands(P) <= 0x7fffffff;
}


int step2_waves(const KParams &P)
{
    return ((P.nx + S2_OUT - 1) / S2_OUT) * s2_nbands(P);
}

// Wavefront indices of the xwall, lean and full instances (the main launch runs the first
// two); the number of walled-row blocks of 64 nodes; the output nodes of the main launch.
void step2_lists(const KParams &P, std::vector<int> &xwall, std::vector<int> &lean, std::vector<int> &full,
                 int &row_blocks, long long &main_nodes)
{
    const int ncx = (P.nx + S2_OUT - 1) / S2_OUT;
    const int ncy = s2_nbands(P);
    xwall.clear();
    lean.clear();
    full.clear();
    main_nodes = 0;
    for (int cy = 0; cy < ncy; ++cy)
        for (int cx = 0; cx < ncx; ++cx) {
            const int w = cy * ncx + cx, kind = s2_kind(P, cx, cy);
            if (kind == STEP2_FULL) {
                full.push_back(w);
                continue;
            }
            (kind == STEP2_XWALL ? xwall : lean).push_back(w);
            const int X0 = s2_x0(P, cx);
            int Y0, Y1;
            s2_band(P, cy, Y0, Y1);
            int cols = 0;
            for (int l = 1; l <= S2_OUT; ++l) cols += P.px || (X0 - 1 + l >= 0 && X0 - 1 + l < P.nx);
            main_nodes += (long long)cols * (Y1 - Y0);
        }
    row_blocks = P.py ? 0 : (2 * P.nx + 63) / 64;
}

template <typename S>
static hipError_t step2_main_s(int launch, const void *src, void *dst, void *scr, const KParams &P,
                               const KParams &Pm, const int *items, int nitems, hipStream_t st)
{
    if (launch == STEP2_FULL) return step2_main_t<S, STEP2_FULL>(src, dst, scr, P, Pm, items, nitems, st);
    return step2_main_t<S, STEP2_MAIN>(src, dst, scr, P, Pm, items, nitems, st);
}

hipError_t launch_step2_main(int storage, int launch, const void *src, void *dst, void *scr, const KParams &P,
                             const KParams &Pm, const int *items, int nitems, hipStream_t st)
{
    if (!step2_supported(P)) return hipErrorInvalidValue;
    switch (storage) {
    case 0: return step2_main_s<double>(launch, src, dst, scr, P, Pm, items, nitems, st);
    case 1: return step2_main_s<float>(launch, src, dst, scr, P, Pm, items, nitems, st);
    case 2: return step2_main_s<__half>(launch, src, dst, scr, P, Pm, items, nitems, st);
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

// The side stream's launches are issued first, so that their wavefronts are dispatched
// beside the main launch's first ones rather than after its last ones.
template <typename S>
static hipError_t batch_step2_t(const BatchProblem *probs, const int2 *const *items, const int *nitems,
                                const int2 *rows, int nrows, int parity, int main_waves, hipStream_t st_main,
                                hipStream_t st_side)
{
    using R = typename Prec<S>::R;
    constexpr int W = S2_B / 64;
    if (main_waves < 1 || main_waves > W) return hipErrorInvalidValue;
    if (nitems[STEP2_FULL] > 0)
        hipLaunchKernelGGL((k_batch_step2<S, STEP2_FULL>), dim3((nitems[STEP2_FULL] + W - 1) / W), dim3(S2_B), 0,
                           st_side, probs, items[STEP2_FULL], nitems[STEP2_FULL], parity);
    if (nrows > 0)   // after the full launch, whose scratch rows it reads
        hipLaunchKernelGGL((k_batch_step2_rows<S>), dim3(nrows), dim3(64), 0, st_side, probs, rows, parity);
    if (nitems[STEP2_MAIN] > 0)
        hipLaunchKernelGGL((k_batch_step2<S, STEP2_MAIN>), dim3((nitems[STEP2_MAIN] + main_waves - 1) / main_waves),
                           dim3(64 * main_waves), (size_t)main_waves * S2_LDS * sizeof(R), st_main,
                           probs, items[STEP2_MAIN], nitems[STEP2_MAIN], parity);
    return hipGetLastError();
}

hipError_t launch_batch_step2(int storage, const BatchProblem *probs, const int2 *const *items, const int *nitems,
                              const int2 *rows, int nrows, int parity, int main_waves, hipStream_t st_main,
                              hipStream_t st_side)
{
    switch (storage) {
    case 0: return batch_step2_t<double>(probs, items, nitems, rows, nrows, parity, main_waves, st_main, st_side);
    case 1: return batch_step2_t<float>(probs, items, nitems, rows, nrows, parity, main_waves, st_main, st_side);
    case 2: return batch_step2_t<__half>(probs, items, nitems, rows, nrows, parity, main_waves, st_main, st_side);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace lbm
