#include "solve_ext.hpp"

namespace hps {
struct SolveExt {};
void solve_ext_free(SolveExt *p) { delete p; }
}  // namespace hps

int solve_ext_init(hps_handle *H) { (void)H; return HPS_OK; }

int solve_ext_run_up_with_jump(hps_handle *, const hps::Bases &, int, int, hipStream_t) {
  return hps::fail(HPS_EINVAL, "flux-jump sources are not available");
}

int solve_ext_mixed(hps_handle *, const double *, const double *, int, double *,
                    const hps_solve_opts *, hipStream_t) {
  return hps::fail(HPS_EINVAL, "mixed precision is not available");
}

extern "C" int hps_solve_adjoint(hps_handle *, const double *, int, double *, double *,
                                 const hps_solve_opts *) {
  return hps::fail(HPS_EINVAL, "adjoint is not available");
}

extern "C" int hps_coeff_grad_c(hps_handle *, const double *, const double *, int, double *,
                                void *) {
  return hps::fail(HPS_EINVAL, "adjoint is not available");
}
