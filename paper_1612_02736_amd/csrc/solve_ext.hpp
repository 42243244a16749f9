// Solve-stage extensions: FP64 residual of the global collocation system,
// mixed-precision iterative refinement and the adjoint (transposed) sweeps.
#pragma once
#include <hip/hip_runtime.h>

#include "handle.hpp"

int solve_ext_init(hps_handle *H);
int solve_ext_mixed(hps_handle *H, const double *f, const double *g, int nrhs, double *u,
                    const hps_solve_opts *opts, hipStream_t st);
int hps_solve_pass(hps_handle *H, const double *f, const double *g, int nrhs, double *u,
                   int prec, const double *jump, hipStream_t st);
hps::Bases make_bases(hps_handle *H);
int run_prog(hps_handle *H, std::vector<hps::Step> &prog, hps::Bases bs, int nrhs,
             int prec, hipStream_t st);
int ensure_solve_buffers(hps_handle *H, int nrhs);
