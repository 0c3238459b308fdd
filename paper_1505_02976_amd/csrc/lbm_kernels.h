// Launchers of the HIP kernels (host side).  storage: 0 = FP64, 1 = FP32, 2 = FP16.
#pragma once

#include "lbm_device.h"

namespace lbm {

hipError_t launch_init(int storage, void *dst, const KParams &P, const double *T, const double *p,
                       const double *ux, const double *uy, hipStream_t st);
hipError_t launch_step(int storage, const void *src, void *dst, const KParams &P, hipStream_t st);
// The two launches of one step separately (bulk nodes, wall nodes).
hipError_t launch_step_bulk(int storage, const void *src, void *dst, const KParams &P, hipStream_t st);
hipError_t launch_step_wall(int storage, const void *src, void *dst, const KParams &P, hipStream_t st);
hipError_t launch_fields(int storage, const void *src, const KParams &P, void *const out[9], int f32,
                         hipStream_t st);
hipError_t launch_residual(int storage, const void *src, const KParams &P, double *snap,
                           double *partial, double *out, hipStream_t st);
hipError_t launch_nusselt(int storage, const void *src, const KParams &P, int wall, double L,
                          double dT, double *out, hipStream_t st);
hipError_t launch_state(int storage, void *buf, const KParams &P, double *io, bool get, hipStream_t st);
long long residual_partials(const KParams &P);

}  // namespace lbm
