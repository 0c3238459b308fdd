// Launchers of the HIP kernels (host side).  storage: 0 = FP64, 1 = FP32, 2 = FP16.
#pragma once

#include <algorithm>
#include <vector>

#include "lbm_device.h"

namespace lbm {

// One problem of a batch: its kernel parameters and its two population buffers.
struct BatchProblem {
    KParams P;
    KParams Pm;      // the eight-row scratch grid of the two-step pass
    void *buf[2];
    void *scr;
    int tiles_x;
};

// Instances of the two-step pass: lean (no wall in reach), full, xwall (walls x = 0 and
// x = nx - 1 only).  Launches: main (the xwall and lean wavefronts) and full.
enum : int { STEP2_LEAN = 0, STEP2_FULL = 1, STEP2_XWALL = 2 };
enum : int { STEP2_MAIN = 0, STEP2_LAUNCHES = 2 };

// Device buffers of the adjoint sweep (FP64, [18][ny][nx] for the 18-component arrays).
struct AdjBufs {
    const double *lam_next;   // adjoint of s_{t+1}
    double *lam;              // adjoint of s_t (output)
    double *wf;               // wall nodes: adjoint of the reference node's populations
    double *wt;               // wall nodes: adjoint of T at x_ff
    double *we;               // wall nodes: adjoint of eps at the reference node
    double *grad;             // dJ/deps, accumulated
    const double *wtj;        // dJ/dT at interior nodes (seed)
};

struct BatchKernels {
    const void *bulk, *edge, *wall;
    int bulk_threads, wall_threads;
};

hipError_t launch_init(int storage, void *dst, const KParams &P, const double *T, const double *p,
                       const double *ux, const double *uy, hipStream_t st);
hipError_t launch_step(int storage, const void *src, void *dst, const KParams &P, hipStream_t st);
// The launches of one step separately: interior tiles; edge tiles and walled rows.
hipError_t launch_step_bulk(int storage, const void *src, void *dst, const KParams &P, hipStream_t st);
hipError_t launch_step_wall(int storage, const void *src, void *dst, const KParams &P, hipStream_t st);
hipError_t launch_fields(int storage, const void *src, const KParams &P, void *const out[9], int f32,
                         hipStream_t st);
hipError_t launch_residual(int storage, const void *src, const KParams &P, double *snap,
                           double *partial, double *out, hipStream_t st);
hipError_t launch_nusselt(int storage, const void *src, const KParams &P, int wall, double L,
                          double dT, double *out, hipStream_t st);
hipError_t launch_state(int storage, void *buf, const KParams &P, double *io, bool get, hipStream_t st);
// *flag |= 1 if some population of the grid is NaN or infinite (flag cleared by the caller).
hipError_t launch_check(int storage, const void *buf, const KParams &P, int *flag, hipStream_t st);
long long residual_partials(const KParams &P);

// Two time steps per pass: the main launch (lean and xwall wavefronts) and the full launch
// (together every node outside the walled rows y = 0, y = ny - 1; the full one also writes
// the intermediate populations of rows 0-3 and ny-4..ny-1 to the eight-row scratch grid
// described by Pm), then the walled rows from the scratch grid.  Each launch reads its
// wavefront indices from a device list built by step2_lists.
bool step2_supported(const KParams &P);
int step2_waves(const KParams &P);   // wavefronts of both launches together
void step2_lists(const KParams &P, std::vector<int> &xwall, std::vector<int> &lean, std::vector<int> &full,
                 int &row_blocks, long long &main_nodes);

// The two-step kernels run STEP2_WAVES_PER_BLOCK independent wavefronts per block.  The
// hardware deals consecutive blocks round-robin to the eight XCDs; the kernels map
// dispatched block b to a logical block so that XCD x runs the x-th contiguous range of
// logical blocks (first block of that range below), whose wavefronts share that XCD's L2.
constexpr int STEP2_WAVES_PER_BLOCK = 4;
inline int xcd_range_start(int x, int nblocks)
{
    const int per = nblocks / 8, rem = nblocks % 8;
    return x * per + std::min(x, rem);
}

// Item list of a launch of heavy and light wavefronts in which every XCD's range starts
// with its proportional share of the heavy ones (so that no XCD gets more work than the
// others, and the heavy wavefronts are not left for the end).
template <typename T>
std::vector<T> xcd_balanced(const std::vector<T> &heavy, const std::vector<T> &light)
{
    const long long H = (long long)heavy.size(), n = H + (long long)light.size();
    std::vector<T> out;
    out.reserve(n);
    if (n == 0) return out;
    const int nb = (int)((n + STEP2_WAVES_PER_BLOCK - 1) / STEP2_WAVES_PER_BLOCK);
    size_t ih = 0, il = 0;
    for (int x = 0; x < 8; ++x) {
        const long long w0 = std::min(n, (long long)STEP2_WAVES_PER_BLOCK * xcd_range_start(x, nb));
        const long long w1 = std::min(n, (long long)STEP2_WAVES_PER_BLOCK * xcd_range_start(x + 1, nb));
        const size_t h1 = (size_t)(H * w1 / n);
        for (long long w = w0; w < w1; ++w) out.push_back(ih < h1 ? heavy[ih++] : light[il++]);
    }
    return out;
}
hipError_t launch_step2_main(int storage, int launch, const void *src, void *dst, void *scr, const KParams &P,
                             const KParams &Pm, const int *items, int nitems, hipStream_t st);
hipError_t launch_step2_rows(int storage, void *dst, const void *scr, const KParams &P, const KParams &Pm,
                             hipStream_t st);

// Batched two-step passes: items[l] (problem, wavefront index) for launch l, nitems[l] of
// them; rows: (problem, block of 64 walled-row nodes); main_waves: wavefronts per block of
// the main launch (1, 2 or 4).  The full launch and then the walled rows go to st_side, the
// main launch to st_main; the caller orders the two streams (they may be the same one).
hipError_t launch_batch_step2(int storage, const BatchProblem *probs, const int2 *const *items, const int *nitems,
                              const int2 *rows, int nrows, int parity, int main_waves, hipStream_t st_main,
                              hipStream_t st_side);

// Adjoint sweep.
hipError_t launch_adjoint_step(int storage, const void *state, const KParams &P, const AdjBufs &A,
                               hipStream_t st);
hipError_t launch_adjoint_seed(const KParams &P, const AdjBufs &A, hipStream_t st);

// Batched stepping: items are (problem, tile) / (problem, wall block) pairs.
// bx: block width of the batched update, one of batch_width(0..2).
hipError_t launch_batch_step(int storage, int bx, const BatchProblem *probs, const int2 *bulk_items, int nbulk,
                             const int2 *edge_items, int nedge, const int2 *wall_items, int nwall,
                             int parity, hipStream_t st);
hipError_t launch_batch_check(int storage, const BatchProblem *probs, const int2 *items, int n,
                              int parity, int *flags, hipStream_t st);
bool batch_kernels(int storage, int bx, BatchKernels &k);
int batch_width(int i);
int batch_tiles_x(int storage, const KParams &P, int bx);
int batch_check_tiles_x(int storage, const KParams &P);
int wall_block_size();
// Nodes updated by the interior-tile launch of one step (single-problem path).
long long interior_nodes(int storage, const KParams &P);

// The device-resident scratch array of the entry point that allocates nothing (one per
// device, LBM_STATIC_SCRATCH_BYTES of include/lbm.h, 256-byte aligned, held until the
// process ends).  static_scratch_setup looks up the address on `device`, which must be
// current; it runs once per device (later calls return the first result).  static_scratch
// returns the address, or NULL before a successful setup on that device.
hipError_t static_scratch_setup(int device);
void *static_scratch(int device);

}  // namespace lbm
