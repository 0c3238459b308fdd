// C interface (include/lbm.h): parameter validation and mapping, workspace layout,
// context bookkeeping and dispatch to the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_error.h"
#include "lbm_kernels.h"

namespace {

thread_local char g_err[512] = "";

lbm_status fail(lbm_status st, const char *fmt, ...)
{
    // formatted into a local buffer first: callers may pass the previous message as an argument
    char msg[sizeof(g_err)];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(msg, sizeof(msg), fmt, ap);
    va_end(ap);
    memcpy(g_err, msg, sizeof(g_err));
    return st;
}

lbm_status hip_fail(hipError_t e, const char *what)
{
    return fail(LBM_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

// The message lbm_last_error reports, for the three-dimensional entry points.
lbm_status lbm::set_error(lbm_status st, const char *msg) { return fail(st, "%s", msg); }

namespace {

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t elem_size(int storage) { return storage == LBM_F64 ? 8 : (storage == LBM_F32 ? 4 : 2); }

// Mapping of Sec. 2, Sec. 3.1, Eq. Therdiff and Eq. EQA&B (see lbm_params in lbm.h).
lbm_status derive(const lbm_params *p, lbm_derived *d)
{
    if (!p) return fail(LBM_ERR_INVALID, "params is NULL");
    if (p->nx < 1 || p->ny < 1) return fail(LBM_ERR_INVALID, "nx, ny must be >= 1");
    if (p->storage < LBM_F64 || p->storage > LBM_F16) return fail(LBM_ERR_INVALID, "unknown storage %d", p->storage);
    for (int ax = 0; ax < 2; ++ax) {
        const int periodic = ax == 0 ? p->periodic_x : p->periodic_y;
        const int n = ax == 0 ? p->nx : p->ny;
        if (periodic) continue;
        const bool neumann = p->wall[2 * ax].t_kind == LBM_T_NEUMANN || p->wall[2 * ax + 1].t_kind == LBM_T_NEUMANN;
        const int need = neumann ? 4 : 3;
        if (n < need) return fail(LBM_ERR_INVALID, "walled direction %c needs >= %d nodes", ax ? 'y' : 'x', need);
        for (int k = 2 * ax; k < 2 * ax + 2; ++k)
            if (p->wall[k].t_kind != LBM_T_DIRICHLET && p->wall[k].t_kind != LBM_T_NEUMANN)
                return fail(LBM_ERR_INVALID, "wall %d: unknown thermal kind", k);
    }
    if (!(p->tau_f > 0.5) || !(p->tau_T > 0.5)) return fail(LBM_ERR_INVALID, "tau_f and tau_T must exceed 1/2");
    if (!(p->sigma > 0) || !(p->J > 0)) return fail(LBM_ERR_INVALID, "sigma and J must be positive");
    if (!(p->eps > 0 && p->eps <= 1)) return fail(LBM_ERR_INVALID, "eps must lie in (0, 1]");
    if (!(p->Da > 0)) return fail(LBM_ERR_INVALID, "Da must be positive (inf allowed)");
    if (!std::isfinite(p->Q) || !std::isfinite(p->ax) || !std::isfinite(p->ay))
        return fail(LBM_ERR_INVALID, "Q, ax, ay must be finite");

    if (p->L > 0) d->L = p->L;
    else if (!p->periodic_x) d->L = p->nx - 1;
    else if (!p->periodic_y) d->L = p->ny - 1;
    else d->L = p->nx;
    d->T0 = 0.5 * (p->T_hot + p->T_cold);
    d->dT = p->T_hot - p->T_cold;
    if (std::isnan(p->A) || std::isnan(p->B)) {
        if (!(p->Ra > 0) || !(p->Pr > 0) || !(p->Ma > 0))
            return fail(LBM_ERR_INVALID, "A, B from Ma need Ra > 0, Pr > 0, Ma > 0");
        d->A = p->tau_f - 0.5 - p->J * p->Ma * d->L * std::sqrt(3.0 * p->Pr / p->Ra);
        d->B = p->tau_T - 0.5 - (p->Ma / p->sigma) * d->L * std::sqrt(3.0 / (p->Pr * p->Ra));
    } else {
        d->A = p->A;
        d->B = p->B;
    }
    d->nu_e = (p->tau_f - d->A - 0.5) / 3.0;
    d->nu = d->nu_e / p->J;
    d->alpha_e = p->sigma * (p->tau_T - d->B - 0.5) / 3.0;
    if (!(d->nu_e > 0)) return fail(LBM_ERR_INVALID, "nu_e <= 0 (A = %g >= tau_f - 1/2)", d->A);
    if (!(d->alpha_e > 0)) return fail(LBM_ERR_INVALID, "alpha_e <= 0 (B = %g >= tau_T - 1/2)", d->B);
    d->gbeta = (p->Ra > 0 && d->dT != 0.0) ? p->Ra * d->nu * d->alpha_e / (d->dT * d->L * d->L * d->L) : 0.0;
    d->K = p->Da * d->L * d->L;
    if (!std::isnan(p->F_eps) && !(p->F_eps >= 0)) return fail(LBM_ERR_INVALID, "F_eps must be >= 0 or NaN");
    return LBM_OK;
}

struct Layout {
    int ntx;              // tiles per row
    size_t pop_bytes;     // one population buffer
    size_t off_a, off_b, off_eps, off_snap, off_part, off_scalar, off_scr, off_items, total;
    long long nparts;
};

// Populations in rows of tiles (TileOf in lbm_device.h), the last tile of a row padded.
Layout layout(const lbm_params *p, const lbm::KParams &kp)
{
    Layout L;
    const size_t es = elem_size(p->storage);
    const int tile = lbm::tile_of_storage(p->storage);
    L.ntx = (p->nx + tile - 1) / tile;
    L.pop_bytes = align_up((size_t)p->ny * L.ntx * 18 * tile * es, 256);
    const size_t N = (size_t)p->nx * p->ny;
    L.nparts = lbm::residual_partials(kp) + 1;
    size_t o = 0;
    L.off_a = o; o += L.pop_bytes;
    L.off_b = o; o += L.pop_bytes;
    L.off_eps = o; o += align_up(p->eps_field ? N * 8 : 0, 256);
    L.off_snap = o; o += align_up(3 * N * 8, 256);
    L.off_part = o; o += align_up((size_t)L.nparts * 5 * 8, 256);
    L.off_scalar = o; o += 256;
    // eight rows of intermediate populations for the two-step pass (walled rows)
    L.off_scr = o; o += align_up((size_t)8 * L.ntx * 18 * tile * es, 256);
    // wavefront lists of the two-step pass's launches
    L.off_items = o; o += align_up(lbm::step2_supported(kp) ? (size_t)lbm::step2_waves(kp) * sizeof(int) : 0, 256);
    L.total = o;
    return L;
}

void fill_kparams(const lbm_params *p, const lbm_derived &d, lbm::KParams &k)
{
    std::memset(&k, 0, sizeof(k));
    k.nx = p->nx; k.ny = p->ny; k.px = p->periodic_x ? 1 : 0; k.py = p->periodic_y ? 1 : 0;
    k.nwall = 2 * p->nx + 2 * p->ny;
    if (k.px && k.py) k.nwall = 0;
    k.nwall_rows = k.py ? 0 : 2 * p->nx;
    k.tau_f = p->tau_f; k.tau_T = p->tau_T; k.A = d.A; k.B = d.B; k.sigma = p->sigma; k.Q = p->Q;
    k.gbeta = d.gbeta; k.T0 = d.T0; k.ax = p->ax; k.ay = p->ay;
    const bool kinf = std::isinf(d.K);
    k.nu_over_K = kinf ? 0.0 : d.nu / d.K;
    k.inv_sqrtK = kinf ? 0.0 : 1.0 / std::sqrt(d.K);
    k.ergun = std::isnan(p->F_eps) ? 1 : 0;
    k.Feps = k.ergun ? 0.0 : p->F_eps;
    k.field = p->eps_field ? 1 : 0;
    k.eps = p->eps;
    const double Fe = k.ergun ? 1.75 / std::sqrt(150.0 * p->eps * p->eps * p->eps) : k.Feps;
    k.c0 = 0.5 * (1.0 + 0.5 * p->eps * k.nu_over_K);
    k.c1 = 0.5 * p->eps * Fe * k.inv_sqrtK;
    k.dlin = p->eps * k.nu_over_K;
    k.dquad = p->eps * Fe * k.inv_sqrtK;
    for (int w = 0; w < 4; ++w) {
        k.wall_ux[w] = p->wall[w].ux; k.wall_uy[w] = p->wall[w].uy;
        k.wall_T[w] = p->wall[w].T; k.wall_dTdn[w] = p->wall[w].dTdn;
        k.wall_kind[w] = p->wall[w].t_kind;
    }
    k.hscale = p->storage == LBM_F16 ? 256.0f : 1.0f;
    k.hinv = 1.0f / k.hscale;

    lbm::Cst<double> &c = k.cd;
    lbm::relax_pair(p->tau_f, c.itf, c.of);
    lbm::relax_pair(p->tau_T, c.itT, c.og);
    c.fF = 1.0 - 0.5 / p->tau_f;
    c.fT = 1.0 - 0.5 / p->tau_T;
    c.tau_f = p->tau_f;
    c.A = d.A;
    c.sigB = p->sigma * d.B;
    c.sig = p->sigma;
    c.isig = 1.0 / p->sigma;
    c.Q = p->Q;
    c.halfQ = 0.5 * p->Q;
    c.gb = d.gbeta;
    c.ax = p->ax;
    c.ay = p->ay;
    c.Sden = 3.0 / (d.A - p->tau_f);
    c.aM0 = p->sigma * (d.B - p->tau_T) / 3.0;
    c.w1 = 1.0 / 9.0;
    c.w5 = 1.0 / 36.0;
    c.w3a = 1.0 / 3.0;
    c.w3d = (1.0 - 2.0 * c.w3a) / 4.0;
    lbm::Cst<float> &cf = k.cf;
    lbm::relax_pair(p->tau_f, cf.itf, cf.of);
    lbm::relax_pair(p->tau_T, cf.itT, cf.og);
    cf.fF = (float)c.fF; cf.fT = (float)c.fT; cf.tau_f = (float)c.tau_f; cf.A = (float)c.A;
    cf.sigB = (float)c.sigB; cf.sig = (float)c.sig; cf.isig = (float)c.isig; cf.Q = (float)c.Q;
    cf.halfQ = (float)c.halfQ; cf.gb = (float)c.gb; cf.ax = (float)c.ax; cf.ay = (float)c.ay;
    cf.Sden = (float)c.Sden; cf.aM0 = (float)c.aM0;
    cf.w1 = (float)c.w1; cf.w5 = (float)c.w5;
    cf.w3a = 1.0f / 3.0f;
    cf.w3d = (1.0f - 2.0f * cf.w3a) / 4.0f;   // 2 w3a + 4 w3d == 1 exactly in FP32
    lbm::derive_consts(c);
    lbm::derive_consts(cf);
    k.ed.eps = p->eps;
    k.ed.ieps = 1.0 / p->eps;
    k.ed.dlin = k.dlin;
    k.ed.dquad = k.dquad;
    k.ed.bM = 0.5 * (1.0 / p->eps - 1.0 / p->sigma);
    k.ef.eps = (float)k.ed.eps; k.ef.ieps = (float)k.ed.ieps; k.ef.dlin = (float)k.ed.dlin;
    k.ef.dquad = (float)k.ed.dquad; k.ef.bM = (float)k.ed.bM;
}

}  // namespace

// HIP events of one bracketed pass of lbm_step_timed (i: main launch, e: the rest).
struct StepEvents { hipEvent_t i0, i1, e0, e1; };

struct lbm_ctx {
    lbm_params prm;
    lbm_derived d;
    lbm::KParams kp;
    Layout lay;
    char *ws;
    hipStream_t stream;
    int64_t t;
    int have_snap;
    int device;
    int in_batch;
    int cur;             // buffer holding the current populations (0: a, 1: b)
    int fuse;            // time steps per pass over the populations (1 or 2)
    int64_t check_every; // lbm_step checks for non-finite populations at multiples of this time (0: never)
    lbm::KParams kpm;    // parameters of the eight-row scratch grid of the two-step pass
    int n_main2, n_full2;       // wavefronts of the two-step pass's main and full launches
    long long main_nodes2;      // output nodes of the main launch
    // Second stream of the two-step pass: the wavefronts next to walls (few, long) run
    // there beside the lean launch; events order each launch after both of the previous pass.
    hipStream_t side;
    hipEvent_t ev_join, ev_main, ev_side;
    // lbm_step_timed's events, created by its first call and kept, so that a timed region
    // that starts with a call does not also time the host creating them
    std::vector<StepEvents> tev;
};

static void *cur_buf(lbm_ctx *c) { return c->ws + (c->cur ? c->lay.off_b : c->lay.off_a); }
static void *next_buf(lbm_ctx *c) { return c->ws + (c->cur ? c->lay.off_a : c->lay.off_b); }

extern "C" {

const char *lbm_last_error(void) { return g_err; }

lbm_status lbm_derive(const lbm_params *params, lbm_derived *out)
{
    if (!out) return fail(LBM_ERR_INVALID, "out is NULL");
    return derive(params, out);
}

size_t lbm_workspace_bytes(const lbm_params *params)
{
    lbm_derived d;
    if (derive(params, &d) != LBM_OK) return 0;
    lbm::KParams kp;
    fill_kparams(params, d, kp);
    return layout(params, kp).total;
}

static lbm_status init_ctx(const lbm_params *params, void *workspace, size_t workspace_bytes,
                           void *hip_stream, lbm_ctx **out)
{
    if (!out) return fail(LBM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    lbm_derived d;
    lbm_status st = derive(params, &d);
    if (st != LBM_OK) return st;
    if (!workspace) return fail(LBM_ERR_INVALID, "workspace is NULL");
    if (((uintptr_t)workspace) % 256) return fail(LBM_ERR_INVALID, "workspace must be 256-byte aligned");
    lbm::KParams kp;
    fill_kparams(params, d, kp);
    const Layout lay = layout(params, kp);
    if (workspace_bytes < lay.total)
        return fail(LBM_ERR_INVALID, "workspace too small: %zu < %zu bytes", workspace_bytes, lay.total);
    kp.ntx = lay.ntx;

    lbm_ctx *c = new (std::nothrow) lbm_ctx;
    if (!c) return fail(LBM_ERR_DEVICE, "out of host memory");
    c->prm = *params;
    c->prm.eps_field = c->prm.T_init = c->prm.p_init = c->prm.ux_init = c->prm.uy_init = nullptr;
    c->d = d;
    c->lay = lay;
    c->ws = static_cast<char *>(workspace);
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->t = 0;
    c->have_snap = 0;
    c->in_batch = 0;
    c->cur = 0;
    c->check_every = 0;
    c->side = nullptr;
    c->ev_join = c->ev_main = c->ev_side = nullptr;
    if (hipGetDevice(&c->device) != hipSuccess) c->device = -1;
    // the address of this device's static scratch array (lbm_residual_noalloc), once per
    // device; a failure here surfaces only in that entry point
    if (c->device >= 0) (void)lbm::static_scratch_setup(c->device);

    hipError_t e;
    if (params->eps_field) {
        double *eps = reinterpret_cast<double *>(c->ws + lay.off_eps);
        e = hipMemcpyAsync(eps, params->eps_field, (size_t)params->nx * params->ny * 8,
                           hipMemcpyDeviceToDevice, c->stream);
        if (e != hipSuccess) { delete c; return hip_fail(e, "copy of eps_field"); }
        kp.eps_field = eps;
    }
    c->kp = kp;
    c->kpm = kp;
    c->kpm.ny = 8;
    c->kpm.py = 0;
    // two-step passes by default where they are faster: FP32 and FP64 storage, whose tiles
    // match the two-step wavefronts (see lbm_step2.hip)
    c->fuse = (params->storage != LBM_F16 && lbm::step2_supported(kp)) ? 2 : 1;
    c->n_main2 = c->n_full2 = 0;
    c->main_nodes2 = 0;
    if (lbm::step2_supported(kp)) {
        std::vector<int> xw, lean, fullv;
        int rb = 0;
        lbm::step2_lists(kp, xw, lean, fullv, rb, c->main_nodes2);
        std::vector<int> mainv = lbm::xcd_balanced(xw, lean);
        c->n_main2 = (int)mainv.size();
        c->n_full2 = (int)fullv.size();
        mainv.insert(mainv.end(), fullv.begin(), fullv.end());
        e = hipMemcpyAsync(c->ws + lay.off_items, mainv.data(), mainv.size() * sizeof(int), hipMemcpyHostToDevice,
                           c->stream);
        // the host list is released on return
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) { delete c; return hip_fail(e, "two-step wavefront lists"); }
    }
    e = hipMemsetAsync(c->ws + lay.off_b, 0, lay.pop_bytes, c->stream);
    if (e == hipSuccess)
        e = lbm::launch_init(params->storage, cur_buf(c), c->kp, params->T_init, params->p_init,
                             params->ux_init, params->uy_init, c->stream);
    if (e != hipSuccess) { delete c; return hip_fail(e, "initialisation"); }
    *out = c;
    return LBM_OK;
}

lbm_status lbm_init(const lbm_params *params, void *workspace, size_t workspace_bytes,
                    void *hip_stream, lbm_ctx **out)
{
    return init_ctx(params, workspace, workspace_bytes, hip_stream, out);
}

namespace {

// Timing events of one launch group: i0 .. i1 around the main launch, e0 .. e1 around the
// rest (on the side stream for two-step passes).
static void destroy_step_events(std::vector<StepEvents> &ev)
{
    for (auto &x : ev) {
        if (x.i0) (void)hipEventDestroy(x.i0);
        if (x.i1) (void)hipEventDestroy(x.i1);
        if (x.e0) (void)hipEventDestroy(x.e0);
        if (x.e1) (void)hipEventDestroy(x.e1);
    }
    ev.clear();
}

hipError_t ensure_side(lbm_ctx *c)
{
    if (c->side) return hipSuccess;
    hipError_t e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_main, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_side, hipEventDisableTiming);
    return e;
}

// npass two-step passes.  The main launch (lean and xwall wavefronts) goes to the context's
// stream; the full launch and the walled rows (which read the scratch rows the full launch
// writes) go to the side stream; pass p's main launch waits for the side stream's pass
// p - 1, its full launch for the main launch of pass p - 1 (both read the source and write
// disjoint nodes of the destination).  Every wait names an event recorded earlier in
// host order; the side stream first waits for the caller's stream and the caller's stream
// finally waits for the side stream, so the call is ordered like launches on the caller's
// stream.
hipError_t run_passes(lbm_ctx *c, int64_t npass, const StepEvents *tev, int every, int64_t gi0)
{
    const int sto = c->prm.storage;
    void *scr = c->ws + c->lay.off_scr;
    const int *items = reinterpret_cast<const int *>(c->ws + c->lay.off_items);
    hipError_t e = ensure_side(c);
    hipStream_t side = c->side;
    if (e == hipSuccess) e = hipEventRecord(c->ev_join, c->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(side, c->ev_join, 0);
    for (int64_t p = 0; p < npass && e == hipSuccess; ++p) {
        void *src = cur_buf(c), *dst = next_buf(c);
        const int64_t gi = gi0 + p;
        const StepEvents *t = (tev && gi % every == 0) ? tev + gi / every : nullptr;
        if (p > 0) {
            e = hipStreamWaitEvent(c->stream, c->ev_side, 0);
            if (e == hipSuccess) e = hipStreamWaitEvent(side, c->ev_main, 0);
        }
        // the side stream's launches are issued first so that their few wavefronts are
        // dispatched beside the main launch's first ones rather than after its last ones
        if (e == hipSuccess && t) e = hipEventRecord(t->e0, side);
        if (e == hipSuccess)
            e = lbm::launch_step2_main(sto, lbm::STEP2_FULL, src, dst, scr, c->kp, c->kpm, items + c->n_main2,
                                       c->n_full2, side);
        if (e == hipSuccess) e = lbm::launch_step2_rows(sto, dst, scr, c->kp, c->kpm, side);
        if (e == hipSuccess && t) e = hipEventRecord(t->e1, side);
        if (e == hipSuccess) e = hipEventRecord(c->ev_side, side);
        if (e == hipSuccess && t) e = hipEventRecord(t->i0, c->stream);
        if (e == hipSuccess)
            e = lbm::launch_step2_main(sto, lbm::STEP2_MAIN, src, dst, scr, c->kp, c->kpm, items, c->n_main2,
                                       c->stream);
        if (e == hipSuccess && t) e = hipEventRecord(t->i1, c->stream);
        if (e == hipSuccess) e = hipEventRecord(c->ev_main, c->stream);
        if (e == hipSuccess) {
            c->t += 2;
            c->cur ^= 1;
        }
    }
    if (e == hipSuccess && npass > 0) e = hipStreamWaitEvent(c->stream, c->ev_side, 0);
    return e;
}

// nsteps steps on the context's stream.  One step: the interior launch, then the launch of
// the columns next to the walls x = 0, x = nx - 1 and of the walled rows.  With fuse = 2,
// pairs of steps run as two-step passes (run_passes), a last odd step as one step.  With
// tev, every `every`-th launch group (g = 0, every, 2 every, ...) is bracketed by
// tev[g / every].  Returns the number of launch groups in *groups.
hipError_t run_steps(lbm_ctx *c, int64_t nsteps, const StepEvents *tev, int every, int64_t *groups)
{
    hipError_t e = hipSuccess;
    const int sto = c->prm.storage;
    int64_t s = 0, gi = 0;
    if (c->fuse == 2 && nsteps >= 2) {
        const int64_t npass = nsteps / 2;
        e = run_passes(c, npass, tev, every, 0);
        s = 2 * npass;
        gi = npass;
    }
    while (s < nsteps && e == hipSuccess) {
        void *src = cur_buf(c), *dst = next_buf(c);
        const StepEvents *t = (tev && gi % every == 0) ? tev + gi / every : nullptr;
        if (t) e = hipEventRecord(t->i0, c->stream);
        if (e == hipSuccess) e = lbm::launch_step_bulk(sto, src, dst, c->kp, c->stream);
        if (e == hipSuccess && t) e = hipEventRecord(t->i1, c->stream);
        if (e == hipSuccess && t) e = hipEventRecord(t->e0, c->stream);
        if (e == hipSuccess) e = lbm::launch_step_wall(sto, src, dst, c->kp, c->stream);
        if (e == hipSuccess && t) e = hipEventRecord(t->e1, c->stream);
        if (e == hipSuccess) {
            c->t += 1;
            s += 1;
            c->cur ^= 1;
            ++gi;
        }
    }
    if (groups) *groups = gi;
    return e;
}

}  // namespace

// Non-finite check of the current populations (synchronizes).
static lbm_status check_state(lbm_ctx *c)
{
    int *flag = reinterpret_cast<int *>(c->ws + c->lay.off_scalar + 192);
    int h = 0;
    hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), c->stream);
    if (e == hipSuccess) e = lbm::launch_check(c->prm.storage, cur_buf(c), c->kp, flag, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "non-finite check");
    if (h) return fail(LBM_ERR_NONFINITE, "populations hold non-finite values at time %lld", (long long)c->t);
    return LBM_OK;
}

lbm_status lbm_step(lbm_ctx *c, int64_t nsteps)
{
    if (!c) return fail(LBM_ERR_INVALID, "ctx is NULL");
    if (c->in_batch) return fail(LBM_ERR_INVALID, "problem belongs to a batch: use lbm_batch_step");
    if (nsteps < 0) return fail(LBM_ERR_INVALID, "nsteps < 0");
    if (nsteps == 0) return LBM_OK;
    if (c->check_every <= 0) {
        hipError_t e = run_steps(c, nsteps, nullptr, 1, nullptr);
        if (e != hipSuccess) return hip_fail(e, "step launch");
        return LBM_OK;
    }
    // chunks that end on multiples of check_every, each followed by the check
    int64_t left = nsteps;
    while (left > 0) {
        const int64_t to_check = c->check_every - c->t % c->check_every;
        const int64_t n = left < to_check ? left : to_check;
        hipError_t e = run_steps(c, n, nullptr, 1, nullptr);
        if (e != hipSuccess) return hip_fail(e, "step launch");
        left -= n;
        if (c->t % c->check_every == 0) {
            const lbm_status st = check_state(c);
            if (st != LBM_OK) return st;
        }
    }
    return LBM_OK;
}

lbm_status lbm_set_check_interval(lbm_ctx *c, int64_t every)
{
    if (!c) return fail(LBM_ERR_INVALID, "ctx is NULL");
    if (every < 0) return fail(LBM_ERR_INVALID, "every must be >= 0");
    c->check_every = every;
    return LBM_OK;
}

lbm_status lbm_step_timed(lbm_ctx *c, int64_t nsteps, int32_t every, double *main_ms, double *rest_ms,
                          int64_t *main_nodes, int32_t *steps_per_launch)
{
    if (!c) return fail(LBM_ERR_INVALID, "ctx is NULL");
    if (c->in_batch) return fail(LBM_ERR_INVALID, "problem belongs to a batch: use lbm_batch_step");
    if (nsteps < c->fuse) return fail(LBM_ERR_INVALID, "nsteps < %d", c->fuse);
    if (every < 1) return fail(LBM_ERR_INVALID, "every < 1");
    // events are read back in groups so that the stream is not drained after every step
    constexpr int GROUP = 32;
    hipError_t e = hipSuccess;
    if (c->tev.empty()) {
        c->tev.assign(GROUP, StepEvents{nullptr, nullptr, nullptr, nullptr});
        for (int k = 0; k < GROUP && e == hipSuccess; ++k) {
            e = hipEventCreate(&c->tev[k].i0);
            if (e == hipSuccess) e = hipEventCreate(&c->tev[k].i1);
            if (e == hipSuccess) e = hipEventCreate(&c->tev[k].e0);
            if (e == hipSuccess) e = hipEventCreate(&c->tev[k].e1);
        }
        if (e != hipSuccess) {
            destroy_step_events(c->tev);
            return hip_fail(e, "timing events");
        }
    }
    std::vector<StepEvents> &ev = c->tev;
    double tb = 0.0, tw = 0.0;
    int64_t done = 0, sampled = 0;
    // only whole passes are timed; a leftover single step runs untimed at the end
    const int64_t timed = nsteps - nsteps % c->fuse;
    const int64_t chunk = (int64_t)GROUP * every * c->fuse;
    while (done < timed && e == hipSuccess) {
        const int64_t nb = (timed - done) < chunk ? (timed - done) : chunk;
        int64_t groups = 0;
        e = run_steps(c, nb, ev.data(), every, &groups);
        const int ns = (int)((groups + every - 1) / every);
        if (e == hipSuccess) e = hipEventSynchronize(ev[ns - 1].e1);
        if (e == hipSuccess) e = hipEventSynchronize(ev[ns - 1].i1);
        for (int s = 0; s < ns && e == hipSuccess; ++s) {
            float a = 0.f, b = 0.f;
            e = hipEventElapsedTime(&a, ev[s].i0, ev[s].i1);
            if (e == hipSuccess) e = hipEventElapsedTime(&b, ev[s].e0, ev[s].e1);
            tb += a;
            tw += b;
        }
        sampled += ns;
        done += nb;
    }
    if (e == hipSuccess && nsteps > timed) e = run_steps(c, nsteps - timed, nullptr, 1, nullptr);
    if (e != hipSuccess) return hip_fail(e, "timed step");
    if (main_ms) *main_ms = tb / (double)sampled;
    if (rest_ms) *rest_ms = tw / (double)sampled;
    if (main_nodes)
        *main_nodes = c->fuse == 2 ? c->main_nodes2 : lbm::interior_nodes(c->prm.storage, c->kp);
    if (steps_per_launch) *steps_per_launch = c->fuse;
    return LBM_OK;
}

lbm_status lbm_set_fusion(lbm_ctx *c, int32_t steps_per_pass)
{
    if (!c) return fail(LBM_ERR_INVALID, "ctx is NULL");
    if (steps_per_pass != 1 && steps_per_pass != 2) return fail(LBM_ERR_INVALID, "steps_per_pass must be 1 or 2");
    if (steps_per_pass == 2 && !lbm::step2_supported(c->kp))
        return fail(LBM_ERR_UNSUPPORTED, "two-step passes need nx >= 4 and ny >= 8");
    c->fuse = steps_per_pass;
    return LBM_OK;
}

int32_t lbm_fusion(const lbm_ctx *c) { return c ? c->fuse : 0; }

int64_t lbm_time(const lbm_ctx *c) { return c ? c->t : -1; }

static lbm_status fields(lbm_ctx *c, int32_t out_dtype, void *const out[9])
{
    if (!c) return fail(LBM_ERR_INVALID, "ctx is NULL");
    if (out_dtype != 0 && out_dtype != 1) return fail(LBM_ERR_INVALID, "out_dtype must be 0 (FP64) or 1 (FP32)");
    hipError_t e = lbm::launch_fields(c->prm.storage, cur_buf(c), c->kp, out, out_dtype, c->stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "fields launch");
}

lbm_status lbm_moments(lbm_ctx *c, int32_t out_dtype, void *p, void *ux, void *uy, void *T)
{
    void *const o[9] = {p, ux, uy, T, nullptr, nullptr, nullptr, nullptr, nullptr};
    return fields(c, out_dtype, o);
}

lbm_status lbm_gradients(lbm_ctx *c, int32_t out_dtype, void *Sxx, void *Sxy, void *Syy,
                         void *dTdx, void *dTdy)
{
    void *const o[9] = {nullptr, nullptr, nullptr, nullptr, Sxx, Sxy, Syy, dTdx, dTdy};
    return fields(c, out_dtype, o);
}

static lbm_status check_nusselt_wall(const lbm_ctx *c, int32_t wall)
{
    if (wall < 0 || wall > 3) return fail(LBM_ERR_INVALID, "wall must be 0..3");
    const bool xwall = wall < 2;
    if ((xwall && c->prm.periodic_x) || (!xwall && c->prm.periodic_y))
        return fail(LBM_ERR_INVALID, "wall %d does not exist (periodic direction)", wall);
    if ((xwall ? c->prm.nx : c->prm.ny) < 3) return fail(LBM_ERR_INVALID, "need 3 node layers");
    if (c->d.dT == 0.0) return fail(LBM_ERR_INVALID, "T_hot == T_cold");
    return LBM_OK;
}

lbm_status lbm_nusselt(lbm_ctx *c, int32_t wall, double *nu_host)
{
    if (!c) return fail(LBM_ERR_INVALID, "ctx is NULL");
    if (!nu_host) return fail(LBM_ERR_INVALID, "nu_host is NULL");
    const lbm_status chk = check_nusselt_wall(c, wall);
    if (chk != LBM_OK) return chk;
    double *dev = reinterpret_cast<double *>(c->ws + c->lay.off_scalar);
    hipError_t e = lbm::launch_nusselt(c->prm.storage, cur_buf(c), c->kp, wall, c->d.L, c->d.dT, dev, c->stream);
    if (e != hipSuccess) return hip_fail(e, "nusselt launch");
    e = hipMemcpyAsync(nu_host, dev, sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "nusselt");
    if (!std::isfinite(*nu_host)) return fail(LBM_ERR_NONFINITE, "Nusselt number is not finite");
    return LBM_OK;
}

// The residual of Sec. 4 with the reduction's partial sums in `part` (residual_partials x 5
// doubles) and its five totals in `res`.
static lbm_status residual_into(lbm_ctx *c, double *part, double *res, double *r_u, double *r_T)
{
    double *snap = reinterpret_cast<double *>(c->ws + c->lay.off_snap);
    hipError_t e = lbm::launch_residual(c->prm.storage, cur_buf(c), c->kp, snap, part, res, c->stream);
    if (e != hipSuccess) return hip_fail(e, "residual launch");
    double h[5];
    e = hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "residual");
    const bool first = !c->have_snap;
    c->have_snap = 1;
    if (h[4] != 0.0) return fail(LBM_ERR_NONFINITE, "%.0f nodes hold non-finite values", h[4]);
    if (first) { *r_u = -1.0; *r_T = -1.0; return LBM_OK; }
    *r_u = h[1] > 0 ? h[0] / h[1] : (h[0] > 0 ? INFINITY : 0.0);
    *r_T = h[3] > 0 ? h[2] / h[3] : (h[2] > 0 ? INFINITY : 0.0);
    return LBM_OK;
}

lbm_status lbm_residual(lbm_ctx *c, double *r_u, double *r_T)
{
    if (!c) return fail(LBM_ERR_INVALID, "ctx is NULL");
    if (!r_u || !r_T) return fail(LBM_ERR_INVALID, "outputs are NULL");
    double *part = reinterpret_cast<double *>(c->ws + c->lay.off_part);
    double *res = reinterpret_cast<double *>(c->ws + c->lay.off_scalar) + 8;
    return residual_into(c, part, res, r_u, r_T);
}

lbm_status lbm_residual_noalloc(lbm_ctx *c, double *r_u, double *r_T)
{
    if (!c) return fail(LBM_ERR_INVALID, "ctx is NULL");
    if (!r_u || !r_T) return fail(LBM_ERR_INVALID, "outputs are NULL");
    const long long np = lbm::residual_partials(c->kp);
    if (256 + (size_t)np * 5 * sizeof(double) > LBM_STATIC_SCRATCH_BYTES)
        return fail(LBM_ERR_INVALID,
                    "grid of %lld nodes needs %lld partial sums (%zu bytes with the totals); the static scratch "
                    "holds %zu bytes", (long long)c->prm.nx * c->prm.ny, np,
                    (size_t)256 + (size_t)np * 5 * sizeof(double), (size_t)LBM_STATIC_SCRATCH_BYTES);
    char *scr = static_cast<char *>(lbm::static_scratch(c->device));
    if (!scr) {
        const hipError_t e = c->device >= 0 ? lbm::static_scratch_setup(c->device) : hipErrorInvalidDevice;
        return hip_fail(e == hipSuccess ? hipErrorInvalidSymbol : e, "static scratch of this device");
    }
    // totals in the first 256 bytes, partial sums after them; every slot is written before
    // it is read, so nothing needs clearing between calls
    return residual_into(c, reinterpret_cast<double *>(scr + 256), reinterpret_cast<double *>(scr), r_u, r_T);
}

lbm_status lbm_get_state(lbm_ctx *c, double *dst)
{
    if (!c || !dst) return fail(LBM_ERR_INVALID, "NULL argument");
    hipError_t e = lbm::launch_state(c->prm.storage, cur_buf(c), c->kp, dst, true, c->stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "get_state");
}

lbm_status lbm_set_state(lbm_ctx *c, const double *src)
{
    if (!c || !src) return fail(LBM_ERR_INVALID, "NULL argument");
    hipError_t e = lbm::launch_state(c->prm.storage, cur_buf(c), c->kp, const_cast<double *>(src), false, c->stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "set_state");
}

static void release_ctx(lbm_ctx *c)
{
    if (c->side) {
        (void)hipStreamSynchronize(c->side);
        (void)hipStreamDestroy(c->side);
    }
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->ev_main) (void)hipEventDestroy(c->ev_main);
    if (c->ev_side) (void)hipEventDestroy(c->ev_side);
    destroy_step_events(c->tev);
    delete c;
}

void lbm_destroy(lbm_ctx *c)
{
    if (!c || c->in_batch) return;
    release_ctx(c);
}

// ---------------------------------------------------------------------------------
// Adjoint
// ---------------------------------------------------------------------------------
struct lbm_adjoint {
    lbm_ctx *ctx;
    int wall;
    int64_t nsteps, K, nck;
    char *ws;
    size_t pop;
    size_t off_ck, off_seg, off_lam0, off_lam1, off_wf, off_wt, off_we, off_wtj;
    double J;
};

namespace {

struct AdjLayout {
    int64_t K, nck;
    size_t off_ck, off_seg, off_lam0, off_lam1, off_wf, off_wt, off_we, off_wtj, total;
};

AdjLayout adj_layout(const lbm_ctx *c, int64_t nsteps)
{
    AdjLayout L;
    int64_t K = (int64_t)std::ceil(std::sqrt((double)nsteps));
    if (K < 1) K = 1;
    L.K = K;
    L.nck = (nsteps + K - 1) / K;
    const size_t N = (size_t)c->prm.nx * c->prm.ny;
    const size_t pop = c->lay.pop_bytes;
    size_t o = 0;
    L.off_ck = o; o += (size_t)L.nck * pop;
    L.off_seg = o; o += (size_t)K * pop;
    L.off_lam0 = o; o += align_up(18 * N * 8, 256);
    L.off_lam1 = o; o += align_up(18 * N * 8, 256);
    L.off_wf = o; o += align_up(18 * N * 8, 256);
    L.off_wt = o; o += align_up(N * 8, 256);
    L.off_we = o; o += align_up(N * 8, 256);
    L.off_wtj = o; o += align_up(N * 8, 256);
    L.total = o;
    return L;
}

// Host copy of the device wall classification.
void host_wall(const lbm_ctx *c, int x, int y, int &xw, int &yw, int &dx, int &dy)
{
    const lbm_params &p = c->prm;
    xw = -1; yw = -1;
    if (!p.periodic_x) { if (x == 0) xw = 0; else if (x == p.nx - 1) xw = 1; }
    if (!p.periodic_y) { if (y == 0) yw = 2; else if (y == p.ny - 1) yw = 3; }
    dx = xw == 0 ? 1 : (xw == 1 ? -1 : 0);
    dy = yw == 2 ? 1 : (yw == 3 ? -1 : 0);
}

// dJ/dT at interior nodes for J = average Nusselt number of `wall` (same definition as
// lbm_nusselt), T at wall nodes expressed through their reference nodes.
void nusselt_weights(const lbm_ctx *c, int wall, double scale, std::vector<double> &w)
{
    const int nx = c->prm.nx, ny = c->prm.ny;
    w.assign((size_t)nx * ny, 0.0);
    const int along = wall < 2 ? ny : nx;
    const double sgn = (wall == 0 || wall == 2) ? 1.0 : -1.0;
    const double cf[3] = {-3.0, 4.0, -1.0};
    auto add = [&](int x, int y, double v) {
        int xw, yw, dx, dy;
        host_wall(c, x, y, xw, yw, dx, dy);
        if (xw < 0 && yw < 0) { w[(size_t)y * nx + x] += v; return; }
        const bool dir = (xw >= 0 && c->prm.wall[xw].t_kind == LBM_T_DIRICHLET) ||
                         (yw >= 0 && c->prm.wall[yw].t_kind == LBM_T_DIRICHLET);
        if (dir) return;   // T fixed at an isothermal wall
        w[(size_t)(y + dy) * nx + (x + dx)] += v * 4.0 / 3.0;
        w[(size_t)(y + 2 * dy) * nx + (x + 2 * dx)] -= v / 3.0;
    };
    for (int j = 0; j < along; ++j) {
        const double wtr = (j == 0 || j == along - 1) ? 0.5 : 1.0;
        const double base = scale * wtr / (along - 1) * (-c->d.L / c->d.dT) * sgn * 0.5;
        for (int k = 0; k < 3; ++k) {
            int x, y;
            if (wall == 0) { x = k; y = j; }
            else if (wall == 1) { x = nx - 1 - k; y = j; }
            else if (wall == 2) { x = j; y = k; }
            else { x = j; y = ny - 1 - k; }
            add(x, y, base * cf[k]);
        }
    }
}

}  // namespace

size_t lbm_adjoint_workspace_bytes(const lbm_ctx *c, int64_t nsteps)
{
    if (!c || nsteps < 1) return 0;
    return adj_layout(c, nsteps).total;
}

lbm_status lbm_adjoint_forward(lbm_ctx *c, int32_t wall, int64_t nsteps, void *workspace,
                               size_t workspace_bytes, lbm_adjoint **out, double *nu_host)
{
    if (!c || !out || !nu_host) return fail(LBM_ERR_INVALID, "NULL argument");
    *out = nullptr;
    if (c->in_batch) return fail(LBM_ERR_INVALID, "problem belongs to a batch");
    if (nsteps < 1) return fail(LBM_ERR_INVALID, "nsteps must be >= 1");
    const lbm_status chk = check_nusselt_wall(c, wall);
    if (chk != LBM_OK) return chk;
    const AdjLayout L = adj_layout(c, nsteps);
    if (!workspace || ((uintptr_t)workspace) % 256) return fail(LBM_ERR_INVALID, "workspace must be non-NULL and 256-byte aligned");
    if (workspace_bytes < L.total) return fail(LBM_ERR_INVALID, "workspace too small: %zu < %zu bytes", workspace_bytes, L.total);
    char *ws = static_cast<char *>(workspace);
    hipError_t e = hipSuccess;
    for (int64_t s = 0; s < nsteps && e == hipSuccess; ++s) {
        if (s % L.K == 0)
            e = hipMemcpyAsync(ws + L.off_ck + (size_t)(s / L.K) * c->lay.pop_bytes, cur_buf(c),
                               c->lay.pop_bytes, hipMemcpyDeviceToDevice, c->stream);
        if (e == hipSuccess) e = lbm::launch_step(c->prm.storage, cur_buf(c), next_buf(c), c->kp, c->stream);
        if (e == hipSuccess) { c->t += 1; c->cur ^= 1; }
    }
    if (e != hipSuccess) return hip_fail(e, "adjoint forward");
    double J;
    lbm_status st = lbm_nusselt(c, wall, &J);
    if (st != LBM_OK) return st;
    lbm_adjoint *a = new (std::nothrow) lbm_adjoint;
    if (!a) return fail(LBM_ERR_DEVICE, "out of host memory");
    a->ctx = c; a->wall = wall; a->nsteps = nsteps; a->K = L.K; a->nck = L.nck; a->ws = ws;
    a->pop = c->lay.pop_bytes;
    a->off_ck = L.off_ck; a->off_seg = L.off_seg; a->off_lam0 = L.off_lam0; a->off_lam1 = L.off_lam1;
    a->off_wf = L.off_wf; a->off_wt = L.off_wt; a->off_we = L.off_we;
    a->off_wtj = L.off_wtj;
    a->J = J;
    *nu_host = J;
    *out = a;
    return LBM_OK;
}

lbm_status lbm_adjoint_backward(lbm_adjoint *a, double dJ, double *grad)
{
    if (!a || !grad) return fail(LBM_ERR_INVALID, "NULL argument");
    lbm_ctx *c = a->ctx;
    const size_t N = (size_t)c->prm.nx * c->prm.ny;
    std::vector<double> wtj;
    nusselt_weights(c, a->wall, dJ, wtj);
    char *ws = a->ws;
    double *lam[2] = {reinterpret_cast<double *>(ws + a->off_lam0), reinterpret_cast<double *>(ws + a->off_lam1)};
    lbm::AdjBufs A;
    A.wf = reinterpret_cast<double *>(ws + a->off_wf);
    A.wt = reinterpret_cast<double *>(ws + a->off_wt);
    A.we = reinterpret_cast<double *>(ws + a->off_we);
    A.grad = grad;
    A.wtj = reinterpret_cast<double *>(ws + a->off_wtj);
    hipError_t e = hipMemcpyAsync(const_cast<double *>(A.wtj), wtj.data(), N * 8, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(grad, 0, N * 8, c->stream);
    int cur = 0;
    A.lam_next = nullptr;
    A.lam = lam[cur];
    if (e == hipSuccess) e = lbm::launch_adjoint_seed(c->kp, A, c->stream);
    auto seg = [&](int64_t i) { return ws + a->off_seg + (size_t)i * a->pop; };
    for (int64_t sg = a->nck - 1; sg >= 0 && e == hipSuccess; --sg) {
        const int64_t t0 = sg * a->K;
        const int64_t t1 = std::min<int64_t>(a->nsteps, t0 + a->K);
        e = hipMemcpyAsync(seg(0), ws + a->off_ck + (size_t)sg * a->pop, a->pop, hipMemcpyDeviceToDevice, c->stream);
        for (int64_t i = 1; i < t1 - t0 && e == hipSuccess; ++i)
            e = lbm::launch_step(c->prm.storage, seg(i - 1), seg(i), c->kp, c->stream);
        for (int64_t i = t1 - t0 - 1; i >= 0 && e == hipSuccess; --i) {
            A.lam_next = lam[cur];
            A.lam = lam[cur ^ 1];
            e = lbm::launch_adjoint_step(c->prm.storage, seg(i), c->kp, A, c->stream);
            cur ^= 1;
        }
    }
    // the seed array on the host must outlive the copy
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(e, "adjoint backward");
    return LBM_OK;
}

void lbm_adjoint_destroy(lbm_adjoint *a) { delete a; }

// ---------------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------------
struct lbm_batch {
    std::vector<lbm_ctx *> ctx;
    int storage;
    hipStream_t stream;
    lbm::BatchProblem *probs;   // device
    int2 *bulk_items, *edge_items, *wall_items, *all_items;
    int nbulk, nedge, nwall, nall;
    int *flags;                 // device, one per problem
    int64_t t;
    int cur;                    // buffer (0/1) of every problem that holds the current state
    int fuse;                   // time steps per batched pass (1, or 2: two-step passes)
    int can_fuse;               // 1 if every problem admits the two-step pass
    int2 *items2[lbm::STEP2_LAUNCHES];   // item tables of the batched two-step pass per launch
    int2 *rows2;
    int nitems2[lbm::STEP2_LAUNCHES], nrows2;
    hipGraph_t graph;           // one-step mode: GRAPH_STEPS steps replayed as one graph
    hipGraphExec_t exec;
    int graph_steps;
    int graph_cur;              // value of cur the graph's launches assume (replays keep it)
    // Two-step passes: the full launch and the walled rows go to a second stream beside the
    // main launch (a graph replays its independent launches one after the other).
    hipStream_t side;
    hipEvent_t ev_join, ev_main, ev_side;
    int bx;                     // block width of the batched one-step update
    int w2;                     // wavefronts per block of the batched two-step main launch
    size_t edge_cap;            // capacity of the edge item table (items)
    std::vector<lbm::BatchProblem> hp;
};

namespace {

// Cost of a two-step wavefront next to a vertical wall relative to a lean one (its
// wall-column work before and after the walk; measured with per-wavefront clock stamps).
constexpr double XWALL_COST = 1.34;

struct BatchLayout {
    std::vector<size_t> off;    // workspace offset of each problem
    size_t off_probs, off_bulk, off_edge, off_wall, off_all, off_flags, off_items2[lbm::STEP2_LAUNCHES], off_rows2, total;
    std::vector<int2> bulk, edge, wall, all, items2[lbm::STEP2_LAUNCHES], rows2;
    bool two;
    std::vector<lbm::KParams> kp;
    std::vector<int> tiles_x;
};

lbm_status batch_layout(const lbm_params *params, int32_t n, BatchLayout &B)
{
    if (!params || n < 1) return fail(LBM_ERR_INVALID, "need at least one problem");
    size_t o = 0;
    B.off.resize(n);
    B.kp.resize(n);
    B.tiles_x.resize(n);
    B.bulk.clear();
    B.edge.clear();
    B.wall.clear();
    B.all.clear();
    for (auto &v : B.items2) v.clear();
    B.rows2.clear();
    B.two = params[0].storage != LBM_F16;
    std::vector<std::vector<int2>> mainp(n);   // main-launch items of each problem
    std::vector<double> cost(n, 0.0);          // their cost in lean wavefronts
    for (int k = 0; k < n; ++k) {
        if (params[k].storage != params[0].storage)
            return fail(LBM_ERR_INVALID, "problem %d: all problems of a batch share one storage type", k);
        lbm_derived d;
        lbm_status st = derive(&params[k], &d);
        if (st != LBM_OK) return fail(st, "problem %d: %s", k, g_err);
        lbm::KParams kp;
        fill_kparams(&params[k], d, kp);
        const Layout lay = layout(&params[k], kp);
        kp.ntx = lay.ntx;
        B.kp[k] = kp;
        B.off[k] = o;
        o += align_up(lay.total, 256);
        const int tx = lbm::batch_tiles_x(params[k].storage, kp, lbm::batch_width(0));
        B.tiles_x[k] = tx;
        const int y0 = kp.py ? 0 : 1, y1 = kp.py ? kp.ny : kp.ny - 1;
        // Batched grids are small (a few tiles per row), so every tile goes to the
        // wall-aware launch: one bulk launch per step instead of an interior and an edge one.
        // The table is sized for the narrowest block width (the most items).
        for (int y = y0; y < y1; ++y)
            for (int t = 0; t < tx; ++t) B.edge.push_back(make_int2(k, y * tx + t));
        const int cx = lbm::batch_check_tiles_x(params[k].storage, kp);
        for (int t = 0; t < cx * kp.ny; ++t) B.all.push_back(make_int2(k, t));
        const int wb = lbm::wall_block_size();
        for (int b = 0; b < (kp.nwall_rows + wb - 1) / wb; ++b) B.wall.push_back(make_int2(k, b));
        if (B.two && lbm::step2_supported(kp)) {
            std::vector<int> xw, lean, fullv;
            int rb = 0;
            long long mn = 0;
            lbm::step2_lists(kp, xw, lean, fullv, rb, mn);
            // per problem its main wavefronts in row-major order (xwall and lean merged by
            // index): neighbouring column chunks of a band then run side by side on one XCD
            // and fetch the cache lines their halo columns share once
            std::vector<int> mainv(xw);
            mainv.insert(mainv.end(), lean.begin(), lean.end());
            std::sort(mainv.begin(), mainv.end());
            for (int w : mainv) mainp[k].push_back(make_int2(k, w));
            cost[k] = (double)lean.size() + XWALL_COST * (double)xw.size();
            for (int w : fullv) B.items2[lbm::STEP2_FULL].push_back(make_int2(k, w));
            for (int r = 0; r < rb; ++r) B.rows2.push_back(make_int2(k, r));
        } else {
            B.two = false;
        }
    }
    if (!B.two) {
        for (auto &v : B.items2) v.clear();
        B.rows2.clear();
    } else {
        // The main launch deals equal-count contiguous ranges of its list to the eight XCDs.
        // Problems are assigned to eight groups, the costliest first, each to the group with
        // the least cost so far, and the groups are listed one after another: every XCD's
        // range then holds a similar mix of narrow and wide problems.
        std::vector<int> order(n);
        for (int k = 0; k < n; ++k) order[k] = k;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
        std::vector<std::vector<int>> groups(8);
        double gcost[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int k : order) {
            const int g = (int)(std::min_element(gcost, gcost + 8) - gcost);
            groups[g].push_back(k);
            gcost[g] += cost[k];
        }
        for (const auto &grp : groups)
            for (int k : grp) B.items2[lbm::STEP2_MAIN].insert(B.items2[lbm::STEP2_MAIN].end(), mainp[k].begin(), mainp[k].end());
    }
    B.off_probs = o; o += align_up((size_t)n * sizeof(lbm::BatchProblem), 256);
    B.off_bulk = o; o += align_up(B.bulk.size() * sizeof(int2) + 8, 256);
    B.off_edge = o; o += align_up(B.edge.size() * sizeof(int2) + 8, 256);
    B.off_wall = o; o += align_up(B.wall.size() * sizeof(int2) + 8, 256);
    B.off_all = o; o += align_up(B.all.size() * sizeof(int2), 256);
    B.off_flags = o; o += align_up((size_t)n * sizeof(int), 256);
    for (int l = 0; l < lbm::STEP2_LAUNCHES; ++l) {
        B.off_items2[l] = o;
        o += align_up(B.items2[l].size() * sizeof(int2), 256);
    }
    B.off_rows2 = o; o += align_up(B.rows2.size() * sizeof(int2), 256);
    B.total = o;
    if (B.all.size() > 0x7fffffff || B.items2[lbm::STEP2_MAIN].size() > 0x7fffffff)
        return fail(LBM_ERR_INVALID, "batch too large");
    return LBM_OK;
}

constexpr int GRAPH_STEPS = 64;   // even: a replay leaves the state in the buffer it started from

hipError_t add_kernel_node(hipGraph_t g, const void *func, int grid, int threads, void **args,
                           const std::vector<hipGraphNode_t> &deps, hipGraphNode_t *node)
{
    hipKernelNodeParams kp = {};
    kp.func = const_cast<void *>(func);
    kp.gridDim = dim3(grid);
    kp.blockDim = dim3(threads);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    return hipGraphAddKernelNode(node, g, deps.empty() ? nullptr : deps.data(), deps.size(), &kp);
}

// GRAPH_STEPS one-step updates of every problem as one graph, starting from buffer b->cur:
// per step the bulk and the wall launches, both after the previous step.
lbm_status batch_build_graph(lbm_batch *b)
{
    hipError_t e = hipGraphCreate(&b->graph, 0);
    if (e != hipSuccess) return hip_fail(e, "hipGraphCreate");
    const lbm::BatchProblem *probs = b->probs;
    std::vector<hipGraphNode_t> prev;
    lbm::BatchKernels K;
    if (!lbm::batch_kernels(b->storage, b->bx, K)) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
        return fail(LBM_ERR_INVALID, "block width %d", b->bx);
    }
    for (int s = 0; s < GRAPH_STEPS && e == hipSuccess; ++s) {
        int parity = (b->cur + s) & 1;
        std::vector<hipGraphNode_t> cur;
        for (int w = 0; w < 3 && e == hipSuccess; ++w) {
            const int nblk = w == 0 ? b->nbulk : (w == 1 ? b->nedge : b->nwall);
            if (nblk == 0) continue;
            const int2 *items = w == 0 ? b->bulk_items : (w == 1 ? b->edge_items : b->wall_items);
            void *args[3] = {(void *)&probs, (void *)&items, (void *)&parity};
            hipGraphNode_t node;
            e = add_kernel_node(b->graph, w == 0 ? K.bulk : (w == 1 ? K.edge : K.wall), nblk,
                                w < 2 ? K.bulk_threads : K.wall_threads, args, prev, &node);
            if (e == hipSuccess) cur.push_back(node);
        }
        prev.swap(cur);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
        return hip_fail(e, "batch graph");
    }
    b->graph_steps = GRAPH_STEPS;
    b->graph_cur = b->cur;
    return LBM_OK;
}

void batch_drop_graph(lbm_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Work tables of the batched update for block width bx: per-problem tile counts and the
// (problem, tile) items, uploaded synchronously.
lbm_status batch_set_width(lbm_batch *b, int bx)
{
    std::vector<int2> edge;
    for (size_t k = 0; k < b->hp.size(); ++k) {
        const lbm::KParams &kp = b->hp[k].P;
        const int tx = lbm::batch_tiles_x(b->storage, kp, bx);
        b->hp[k].tiles_x = tx;
        const int y0 = kp.py ? 0 : 1, y1 = kp.py ? kp.ny : kp.ny - 1;
        for (int y = y0; y < y1; ++y)
            for (int t = 0; t < tx; ++t) edge.push_back(make_int2((int)k, y * tx + t));
    }
    if (edge.size() > b->edge_cap) return fail(LBM_ERR_INVALID, "block width %d: item table too small", bx);
    batch_drop_graph(b);
    hipError_t e = hipMemcpyAsync(b->probs, b->hp.data(), b->hp.size() * sizeof(lbm::BatchProblem),
                                  hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && !edge.empty())
        e = hipMemcpyAsync(b->edge_items, edge.data(), edge.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch tables");
    b->nedge = (int)edge.size();
    b->bx = bx;
    return LBM_OK;
}

// Wavefronts per block of the batched two-step main launch (1, 2 or 4).
lbm_status batch_set_waves2(lbm_batch *b, int waves)
{
    if (waves < 1 || waves > lbm::STEP2_WAVES_PER_BLOCK || (waves & (waves - 1)))
        return fail(LBM_ERR_INVALID, "wavefronts per block %d", waves);
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch width");
    b->w2 = waves;
    return LBM_OK;
}

}  // namespace

size_t lbm_batch_workspace_bytes(const lbm_params *params, int32_t n)
{
    BatchLayout B;
    if (batch_layout(params, n, B) != LBM_OK) return 0;
    return B.total;
}

lbm_status lbm_batch_init(const lbm_params *params, int32_t n, void *workspace, size_t workspace_bytes,
                          void *hip_stream, lbm_batch **out)
{
    if (!out) return fail(LBM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    BatchLayout B;
    lbm_status st = batch_layout(params, n, B);
    if (st != LBM_OK) return st;
    if (!workspace || ((uintptr_t)workspace) % 256) return fail(LBM_ERR_INVALID, "workspace must be non-NULL and 256-byte aligned");
    if (workspace_bytes < B.total) return fail(LBM_ERR_INVALID, "workspace too small: %zu < %zu bytes", workspace_bytes, B.total);
    lbm_batch *b = new (std::nothrow) lbm_batch;
    if (!b) return fail(LBM_ERR_DEVICE, "out of host memory");
    char *ws = static_cast<char *>(workspace);
    b->storage = params[0].storage;
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->t = 0;
    b->cur = 0;
    b->can_fuse = B.two ? 1 : 0;
    b->fuse = B.two ? 2 : 1;
    b->graph = nullptr;
    b->exec = nullptr;
    b->graph_steps = 0;
    b->graph_cur = 0;
    b->side = nullptr;
    b->ev_join = b->ev_main = b->ev_side = nullptr;
    b->bx = lbm::batch_width(0);
    b->w2 = lbm::STEP2_WAVES_PER_BLOCK;
    b->edge_cap = B.edge.size();
    std::vector<lbm::BatchProblem> &hp = b->hp;
    hp.resize(n);
    for (int k = 0; k < n; ++k) {
        lbm_ctx *c = nullptr;
        st = init_ctx(&params[k], ws + B.off[k], workspace_bytes - B.off[k], hip_stream, &c);
        if (st != LBM_OK) {
            for (lbm_ctx *q : b->ctx) delete q;
            delete b;
            return fail(st, "problem %d: %s", k, g_err);
        }
        c->in_batch = 1;
        b->ctx.push_back(c);
        hp[k].P = c->kp;
        hp[k].buf[0] = c->ws + c->lay.off_a;
        hp[k].buf[1] = c->ws + c->lay.off_b;
        hp[k].Pm = c->kpm;
        hp[k].scr = c->ws + c->lay.off_scr;
        hp[k].tiles_x = B.tiles_x[k];
    }
    b->probs = reinterpret_cast<lbm::BatchProblem *>(ws + B.off_probs);
    b->bulk_items = reinterpret_cast<int2 *>(ws + B.off_bulk);
    b->edge_items = reinterpret_cast<int2 *>(ws + B.off_edge);
    b->nedge = (int)B.edge.size();
    b->wall_items = reinterpret_cast<int2 *>(ws + B.off_wall);
    b->all_items = reinterpret_cast<int2 *>(ws + B.off_all);
    b->nall = (int)B.all.size();
    b->flags = reinterpret_cast<int *>(ws + B.off_flags);
    b->nbulk = (int)B.bulk.size();
    b->nwall = (int)B.wall.size();
    for (int l = 0; l < lbm::STEP2_LAUNCHES; ++l) {
        b->items2[l] = reinterpret_cast<int2 *>(ws + B.off_items2[l]);
        b->nitems2[l] = (int)B.items2[l].size();
    }
    b->rows2 = reinterpret_cast<int2 *>(ws + B.off_rows2);
    b->nrows2 = (int)B.rows2.size();
    hipError_t e = hipMemcpyAsync(b->probs, hp.data(), n * sizeof(lbm::BatchProblem), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && b->nbulk)
        e = hipMemcpyAsync(b->bulk_items, B.bulk.data(), B.bulk.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && b->nedge)
        e = hipMemcpyAsync(b->edge_items, B.edge.data(), B.edge.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && b->nwall)
        e = hipMemcpyAsync(b->wall_items, B.wall.data(), B.wall.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && b->nall)
        e = hipMemcpyAsync(b->all_items, B.all.data(), B.all.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream);
    for (int l = 0; l < lbm::STEP2_LAUNCHES; ++l)
        if (e == hipSuccess && b->nitems2[l])
            e = hipMemcpyAsync(b->items2[l], B.items2[l].data(), B.items2[l].size() * sizeof(int2),
                               hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && b->nrows2)
        e = hipMemcpyAsync(b->rows2, B.rows2.data(), B.rows2.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream);
    // the layout's host vectors are released on return: wait for the copies
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        for (lbm_ctx *q : b->ctx) delete q;
        delete b;
        return hip_fail(e, "batch tables");
    }
    *out = b;
    return LBM_OK;
}

namespace {

// One step of every problem (bulk and wall launches) from buffer b->cur.
hipError_t batch_single(lbm_batch *b)
{
    hipError_t e = lbm::launch_batch_step(b->storage, b->bx, b->probs, b->bulk_items, b->nbulk, b->edge_items,
                                          b->nedge, b->wall_items, b->nwall, b->cur, b->stream);
    if (e == hipSuccess) {
        ++b->t;
        b->cur ^= 1;
    }
    return e;
}

hipError_t batch_ensure_side(lbm_batch *b)
{
    if (b->side) return hipSuccess;
    hipError_t e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_main, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_side, hipEventDisableTiming);
    return e;
}

// npass two-step passes of every problem, ordered as run_passes orders one problem's: the
// main launch on the batch's stream, the full launch and the walled rows on the side stream;
// pass p's main launch waits for the side stream's pass p - 1, its full launch for the main
// launch of pass p - 1.  advance: pass p reads buffer cur and writes the other one, then cur
// flips (the time advances); otherwise every pass reads and writes the same buffers (the
// autotuner's timing passes, which leave the state as it is).  waves: wavefronts per block
// of the main launch.
hipError_t batch_passes(lbm_batch *b, int64_t npass, bool advance, int waves)
{
    hipError_t e = batch_ensure_side(b);
    if (e == hipSuccess) e = hipEventRecord(b->ev_join, b->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->side, b->ev_join, 0);
    for (int64_t p = 0; p < npass && e == hipSuccess; ++p) {
        if (p > 0) {
            e = hipStreamWaitEvent(b->stream, b->ev_side, 0);
            if (e == hipSuccess) e = hipStreamWaitEvent(b->side, b->ev_main, 0);
        }
        if (e == hipSuccess)
            e = lbm::launch_batch_step2(b->storage, b->probs, b->items2, b->nitems2, b->rows2, b->nrows2, b->cur,
                                        waves, b->stream, b->side);
        if (e == hipSuccess) e = hipEventRecord(b->ev_side, b->side);
        if (e == hipSuccess) e = hipEventRecord(b->ev_main, b->stream);
        if (e == hipSuccess && advance) {
            b->t += 2;
            b->cur ^= 1;
        }
    }
    if (e == hipSuccess && npass > 0) e = hipStreamWaitEvent(b->stream, b->ev_side, 0);
    return e;
}

}  // namespace

lbm_status lbm_batch_step(lbm_batch *b, int64_t nsteps)
{
    if (!b) return fail(LBM_ERR_INVALID, "batch is NULL");
    if (nsteps < 0) return fail(LBM_ERR_INVALID, "nsteps < 0");
    int64_t left = nsteps;
    hipError_t e = hipSuccess;
    if (b->fuse == 2) {
        e = batch_passes(b, left / 2, true, b->w2);
        if (e != hipSuccess) return hip_fail(e, "batch passes");
        left %= 2;
    } else {
        // a graph replays from the buffer it was built for: one single step realigns `cur`
        if (b->exec && b->cur != b->graph_cur && left > GRAPH_STEPS) {
            e = batch_single(b);
            if (e != hipSuccess) return hip_fail(e, "batch step");
            --left;
        }
        if (left >= GRAPH_STEPS && !b->exec) {
            lbm_status st = batch_build_graph(b);
            if (st != LBM_OK) return st;
        }
        while (left >= GRAPH_STEPS && b->cur == b->graph_cur) {
            e = hipGraphLaunch(b->exec, b->stream);
            if (e != hipSuccess) return hip_fail(e, "batch graph launch");
            left -= GRAPH_STEPS;
            b->t += GRAPH_STEPS;
        }
    }
    while (left > 0) {
        e = batch_single(b);
        if (e != hipSuccess) return hip_fail(e, "batch step");
        --left;
    }
    for (lbm_ctx *c : b->ctx) { c->t = b->t; c->cur = b->cur; }
    return LBM_OK;
}

lbm_status lbm_batch_set_fusion(lbm_batch *b, int32_t steps_per_pass)
{
    if (!b) return fail(LBM_ERR_INVALID, "batch is NULL");
    if (steps_per_pass != 1 && steps_per_pass != 2) return fail(LBM_ERR_INVALID, "steps per pass must be 1 or 2");
    if (steps_per_pass == 2 && !b->can_fuse)
        return fail(LBM_ERR_UNSUPPORTED, "two-step passes need FP32/FP64 storage and every grid at least 4 x 8 nodes");
    if (b->fuse != steps_per_pass) batch_drop_graph(b);
    b->fuse = steps_per_pass;
    return LBM_OK;
}

int32_t lbm_batch_fusion(const lbm_batch *b) { return b ? b->fuse : 0; }

lbm_ctx *lbm_batch_problem(lbm_batch *b, int32_t k)
{
    if (!b || k < 0 || k >= (int32_t)b->ctx.size()) return nullptr;
    return b->ctx[k];
}

lbm_status lbm_batch_check(lbm_batch *b, int32_t *flags_host)
{
    if (!b || !flags_host) return fail(LBM_ERR_INVALID, "NULL argument");
    const int n = (int)b->ctx.size();
    hipError_t e = hipMemsetAsync(b->flags, 0, n * sizeof(int), b->stream);
    if (e == hipSuccess)
        e = lbm::launch_batch_check(b->storage, b->probs, b->all_items, b->nall, b->cur, b->flags, b->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(flags_host, b->flags, n * sizeof(int), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch check");
    for (int k = 0; k < n; ++k)
        if (flags_host[k]) return fail(LBM_ERR_NONFINITE, "problem %d holds non-finite values", k);
    return LBM_OK;
}

lbm_status lbm_batch_autotune(lbm_batch *b, int32_t steps, int32_t *width, double *ms_per_step)
{
    if (!b) return fail(LBM_ERR_INVALID, "batch is NULL");
    if (steps < 1) return fail(LBM_ERR_INVALID, "steps must be >= 1");
    const int parity = b->cur;
    const bool two = b->fuse == 2;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    int best = -1;
    float best_ms = 0.0f;
    lbm_status st = LBM_OK;
    for (int i = 0; i < LBM_BATCH_NUM_WIDTHS && e == hipSuccess && st == LBM_OK; ++i) {
        const int bx = lbm::batch_width(i);
        if (!two) {
            st = batch_set_width(b, bx);
            if (st != LBM_OK) break;
        }
        // every launch reads the current buffers and writes the other ones (and, for
        // two-step passes, the scratch rows), so the state is kept
        auto run = [&](int n) {
            if (two) return batch_passes(b, n, false, bx / 64);
            hipError_t r = hipSuccess;
            for (int s = 0; s < n && r == hipSuccess; ++s)
                r = lbm::launch_batch_step(b->storage, b->bx, b->probs, b->bulk_items, b->nbulk, b->edge_items,
                                           b->nedge, b->wall_items, b->nwall, parity, b->stream);
            return r;
        };
        const int reps = two ? (steps + 1) / 2 : steps;
        e = run(2);
        if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
        if (e == hipSuccess) e = run(reps);
        if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess) {
            ms /= (two ? 2 * reps : reps);
            if (ms_per_step) ms_per_step[i] = ms;
            if (best < 0 || ms < best_ms) { best = i; best_ms = ms; }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st != LBM_OK) return st;
    if (e != hipSuccess) return hip_fail(e, "batch autotune");
    st = two ? batch_set_waves2(b, lbm::batch_width(best) / 64) : batch_set_width(b, lbm::batch_width(best));
    if (st != LBM_OK) return st;
    if (width) *width = two ? 64 * b->w2 : b->bx;
    return LBM_OK;
}

lbm_status lbm_batch_set_width(lbm_batch *b, int32_t width)
{
    if (!b) return fail(LBM_ERR_INVALID, "batch is NULL");
    for (int i = 0; i < LBM_BATCH_NUM_WIDTHS; ++i)
        if (lbm::batch_width(i) == width)
            return b->fuse == 2 ? batch_set_waves2(b, width / 64) : batch_set_width(b, width);
    return fail(LBM_ERR_INVALID, "width %d is not one of 64, 128, 256", width);
}

void lbm_batch_destroy(lbm_batch *b)
{
    if (!b) return;
    batch_drop_graph(b);
    if (b->side) {
        (void)hipStreamSynchronize(b->side);
        (void)hipStreamDestroy(b->side);
    }
    if (b->ev_join) (void)hipEventDestroy(b->ev_join);
    if (b->ev_main) (void)hipEventDestroy(b->ev_main);
    if (b->ev_side) (void)hipEventDestroy(b->ev_side);
    for (lbm_ctx *c : b->ctx) release_ctx(c);
    delete b;
}

}  // extern "C"
