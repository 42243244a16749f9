// Solve-stage extensions on top of the planned programs:
//  * mixed precision: FP32 sweeps (FP32 copies of the FP64-built operators)
//    corrected by iterative refinement against the FP64 residual of the
//    global collocation system;
//  * the adjoint: transposed sweeps of Algorithm 2 and the gradient with
//    respect to the zeroth-order coefficient.
#include "solve_ext.hpp"

#include <algorithm>
#include <cmath>
#include <string>

#include "kernels.hpp"
#include "kernels_ext.hpp"

namespace hps {

struct SolveExt {
  DevArray<double> xug, jump, r1, flux, duc, zf, red;
  int cap = 0;
};

void solve_ext_free(SolveExt *p) { delete p; }

}  // namespace hps

using namespace hps;

int solve_ext_init(hps_handle *H) {
  H->ext.reset(new SolveExt);
  return HPS_OK;
}

static int ext_buffers(hps_handle *H, int nrhs) {
  SolveExt &E = *H->ext;
  if (E.cap >= nrhs) return HPS_OK;
  const size_t N = size_t(H->pl.n_gauss), nl = size_t(H->nleaf);
  HIPCHK(E.xug.alloc(N * nrhs));
  HIPCHK(E.jump.alloc(N * nrhs));
  HIPCHK(E.r1.alloc(nl * H->mi * nrhs));
  HIPCHK(E.flux.alloc(nl * H->g4 * nrhs));
  HIPCHK(E.duc.alloc(nl * H->p * H->p * nrhs));
  HIPCHK(E.zf.alloc(size_t(H->n_bdry) * nrhs));
  HIPCHK(hipMemset(E.zf.p, 0, sizeof(double) * H->n_bdry * nrhs));
  HIPCHK(E.jump.p ? hipMemset(E.jump.p, 0, sizeof(double) * N * nrhs) : hipSuccess);
  HIPCHK(E.red.alloc(2));
  E.cap = nrhs;
  return HPS_OK;
}

// u_c(I_ce) = L u_ge in FP64 from the global Gauss vector held in BUF_VEC
static int recompute_exterior(hps_handle *H, double *u, int nrhs, hipStream_t st) {
  Bases bs = make_bases(H);
  bs.d[BUF_IN2] = u;
  return run_prog(H, H->ext_prog, bs, nrhs, 0, st);
}

int solve_ext_mixed(hps_handle *H, const double *f, const double *g, int nrhs, double *u,
                    const hps_solve_opts *opts, hipStream_t st) {
  if (!H->has_fp32) return fail(HPS_EINVAL, "mixed precision needs a build with keep_fp32");
  if (!H->conforming)
    return fail(HPS_EINVAL, "mixed precision is available on trees without refined interfaces");
  int rc = ext_buffers(H, nrhs);
  if (rc) return rc;
  SolveExt &E = *H->ext;
  const int max_iter = opts && opts->max_iter > 0 ? opts->max_iter : 6;
  const double tol = opts && opts->ir_tol > 0.0 ? opts->ir_tol : 1e-10;
  const int64_t N = H->pl.n_gauss;
  const int64_t ucn = int64_t(H->nleaf) * H->p * H->p;
  // first FP32 pass on the original data
  rc = hps_solve_pass(H, f, g, nrhs, u, 1, nullptr, st);
  if (rc) return rc;
  // the global Gauss vector is RHS-interleaved in BUF_VEC: N * nrhs contiguous
  double *vug = H->vec.p + H->ug_off * nrhs;
  const int64_t nug = N * nrhs;
  HIPCHK(launch_fill(E.xug.p, 0.0, nug, st));
  HIPCHK(launch_accumulate(E.xug.p, 0, vug, 0, nug, 1, 0, st));
  rc = recompute_exterior(H, u, nrhs, st);
  if (rc) return rc;
  // Stopping rule: each FP32 sweep solves the correction equation to a
  // relative accuracy rho (about 1e-6), so after a correction du the error is
  // about rho |du|.  rho is estimated as the ratio of successive corrections
  // (the first "correction" being the first sweep's u itself), and the
  // refinement stops once the size of the last correction or, with a safety
  // factor of 100, that estimate of the remaining error is at most ir_tol.
  int it = 0;
  double ratio = 1.0, prev = 1.0;
  for (; it < max_iter; ++it) {
    HIPCHK(launch_residual(H->p, H->d_leaf.p, H->nleaf, H->coef.p, u, g, 0.0, E.r1.p, E.flux.p,
                           H->aux.p + H->Dh_off, H->aux.p + H->Dh2_off, H->d_lloc.p, H->q, nrhs,
                           st));
    HIPCHK(launch_jump(H->d_jn.p, H->d_fa.p, H->d_fb.p, H->d_fp.p, H->n_jump, E.flux.p,
                       int64_t(H->nleaf) * H->g4, f, H->n_bdry, E.jump.p, nrhs, st));
    rc = hps_solve_pass(H, E.zf.p, E.r1.p, nrhs, E.duc.p, 1, E.jump.p, st);
    if (rc) return rc;
    HIPCHK(launch_accumulate(E.xug.p, 0, vug, 0, nug, 1, 1, st));
    HIPCHK(launch_accumulate(u, ucn, E.duc.p, ucn, ucn, nrhs, 0, st));
    rc = recompute_exterior(H, u, nrhs, st);
    if (rc) return rc;
    HIPCHK(launch_maxabs2(E.duc.p, u, ucn * nrhs, E.red.p, st));
    double m[2];
    HIPCHK(hipMemcpyAsync(m, E.red.p, sizeof(m), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    // the reduction maps NaN to +inf, so a non-finite entry shows in m[]
    if (!std::isfinite(m[0]) || !std::isfinite(m[1]))
      return fail(HPS_ENONFINITE, "non-finite entry in the refined solution or its correction");
    ratio = m[1] > 0.0 ? m[0] / m[1] : (m[0] > 0.0 ? HUGE_VAL : 0.0);
    const double rho = prev > 0.0 ? ratio / prev : HUGE_VAL;
    prev = ratio;
    if (ratio <= tol || (rho <= 1e-3 && 100.0 * rho * ratio <= tol)) {
      ratio = std::min(ratio, rho * ratio);
      ++it;
      break;
    }
  }
  if (opts && opts->iters_out) *opts->iters_out = it;
  if (opts && opts->resid_out) *opts->resid_out = ratio;
  if (!(ratio <= tol))
    return fail(HPS_ENOCONV, "iterative refinement stopped at max|du|/max|u| = " +
                                 std::to_string(ratio) + " above ir_tol");
  return HPS_OK;
}

extern "C" int hps_solve_adjoint(hps_handle *h, const double *ubar, int nrhs, double *fbar,
                                 double *gbar, const hps_solve_opts *opts) {
  if (!h || !ubar || !fbar || !gbar) return fail(HPS_EINVAL, "NULL argument");
  if (nrhs <= 0) return fail(HPS_EINVAL, "nrhs must be positive");
  if (h->econ) return fail(HPS_EINVAL, "the adjoint needs the stored leaf operators F");
  hipStream_t st = opts ? (hipStream_t)opts->stream : nullptr;
  int rc = ensure_solve_buffers(h, nrhs);
  if (rc) return rc;
  Bases bs = make_bases(h);
  bs.d[BUF_IN0] = (void *)ubar;
  bs.d[BUF_IN1] = fbar;
  bs.d[BUF_IN2] = gbar;
  rc = run_prog(h, h->adj_down_prog, bs, nrhs, 0, st);
  if (rc) return rc;
  rc = run_prog(h, h->adj_up_prog, bs, nrhs, 0, st);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(st));
  return HPS_OK;
}

extern "C" int hps_coeff_grad_c(hps_handle *h, const double *u, const double *gbar, int nrhs,
                                double *cbar, void *stream) {
  if (!h || !u || !gbar || !cbar) return fail(HPS_EINVAL, "NULL argument");
  if (nrhs <= 0) return fail(HPS_EINVAL, "nrhs must be positive");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(launch_cbar(u, gbar, cbar, h->p, h->nleaf, nrhs, st));
  HIPCHK(hipStreamSynchronize(st));
  return HPS_OK;
}

extern "C" int hps_apply_operator(hps_handle *h, const double *u, int nrhs, double sigma,
                                  double *out, void *stream) {
  if (!h || !u || !out) return fail(HPS_EINVAL, "NULL argument");
  if (nrhs <= 0) return fail(HPS_EINVAL, "nrhs must be positive");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(launch_residual(h->p, h->d_leaf.p, h->nleaf, h->coef.p, u, nullptr, sigma, out, nullptr,
                         h->aux.p + h->Dh_off, h->aux.p + h->Dh2_off, h->d_lloc.p, h->q, nrhs, st));
  HIPCHK(hipStreamSynchronize(st));
  return HPS_OK;
}
