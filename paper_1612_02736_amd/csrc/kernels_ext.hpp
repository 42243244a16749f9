// Launchers of kernels_ext.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "types.hpp"

namespace hps {

// r1 = g - A u at interior nodes and the boundary fluxes into flux; with
// g == nullptr, r1 = sigma u - A u and no fluxes (flux is not used)
hipError_t launch_residual(int p, const LeafDesc *leafd, int nleaf, const double *coef,
                           const double *uc, const double *g, double sigma, double *r1,
                           double *flux,
                           const double *Dh, const double *Dh2, const double *Lloc, int q,
                           int nrhs, hipStream_t st);
hipError_t launch_jump(const int32_t *jn, const int32_t *fa, const int32_t *fb,
                       const int32_t *fp, int64_t n, const double *flux, int64_t flux_stride,
                       const double *f, int64_t f_stride, double *jump, int nrhs,
                       hipStream_t st);
hipError_t launch_accumulate(double *x, int64_t xs, double *y, int64_t ys, int64_t n, int nrhs,
                             int copy_back, hipStream_t st);
hipError_t launch_maxabs2(const double *a, const double *b, int64_t n, double *out,
                          hipStream_t st);
hipError_t launch_cbar(const double *u, const double *gbar, double *cbar, int p, int64_t nl,
                       int nrhs, hipStream_t st);

}  // namespace hps
