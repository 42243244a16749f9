// Leaf interior inversions F = A_ci,ci^-1 of the build stage (Sec. 3.3).
#include "gj_core.hpp"

#include <cstdlib>
#include <string>

namespace hps {

template <int P, int TR, int TC, int RA, int CB>
__global__ __launch_bounds__((gj_threads<TR, TC>())) void gj_leaf_kernel(
    const LeafDesc *__restrict__ descs, int nleaf, Bases bs,
    const double *__restrict__ Dh_g, const double *__restrict__ Dh2_g,
    const int32_t *__restrict__ ice, int me, int32_t *__restrict__ info) {
  constexpr int PI = P - 2, MI = PI * PI;
  __shared__ GJShared<TR, TC, RA, CB> sh;
  __shared__ double cf[6][P * P];
  __shared__ double Dh[P * P], Dh2[P * P];
  const int leaf = blockIdx.x;
  if (leaf >= nleaf) return;
  const LeafDesc &d = descs[leaf];
  const double *coef = (const double *)bs.d[BUF_COEF] + d.coef;
  const int tid = threadIdx.x;
  for (int i = tid; i < 6 * P * P; i += blockDim.x) cf[i / (P * P)][i % (P * P)] = coef[i];
  for (int i = tid; i < P * P; i += blockDim.x) { Dh[i] = Dh_g[i]; Dh2[i] = Dh2_g[i]; }
  __syncthreads();
  const double sx = d.sx, sy = d.sy;
  auto entry = [&](int ga, int gb) -> double {
    // ga: grid index of the collocation row, gb: grid index of the column
    const int iy = ga / P, ix = ga - iy * P, jy = gb / P, jx = gb - jy * P;
    double v = -2.0 * cf[1][ga] * sx * sy * Dh[iy * P + jy] * Dh[ix * P + jx];
    if (iy == jy) v += -cf[0][ga] * sx * sx * Dh2[ix * P + jx] + cf[3][ga] * sx * Dh[ix * P + jx];
    if (ix == jx) v += -cf[2][ga] * sy * sy * Dh2[iy * P + jy] + cf[4][ga] * sy * Dh[iy * P + jy];
    if (ga == gb) v += cf[5][ga];
    return v;
  };
  auto grid_of = [](int a) { const int y = a / PI; return (y + 1) * P + (a - y * PI) + 1; };
  // A_ci,ce (mi x me, column-major) for the leaf products
  if (d.Aie >= 0) {
    double *Aie = (double *)bs.d[BUF_SCR] + d.Aie;
    for (int idx = tid; idx < MI * me; idx += blockDim.x) {
      const int a = idx % MI, e = idx / MI;
      Aie[idx] = entry(grid_of(a), ice[e]);
    }
  }
  int tr, tc;
  gj_owner<TR, TC, RA, CB>(tid, tr, tc);
  double a[RA][CB];
#pragma unroll
  for (int i = 0; i < RA; ++i) {
    const int row = tr + TR * i;
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      const int col = tc + TC * b;
      a[i][b] = (row < MI && col < MI) ? entry(grid_of(row), grid_of(col)) : 0.0;
    }
  }
  gj_core<TR, TC, RA, CB>(a, MI, tr, tc, sh);
  double *F = (double *)bs.d[d.fbuf] + d.F;
  gj_store<TR, TC, RA, CB>(a, MI, tr, tc, sh, F, MI);
  if (tid == 0) info[d.info] = sh.info;
}


template <int P, int NW, int RA, int CB>
__global__ __launch_bounds__(NW * 64) void gj2_leaf_kernel(
    const LeafDesc *__restrict__ descs, int nleaf, Bases bs,
    const double *__restrict__ Dh_g, const double *__restrict__ Dh2_g,
    const int32_t *__restrict__ ice, int me, int32_t *__restrict__ info) {
  constexpr int PI = P - 2, MI = PI * PI;
  static_assert(64 * RA >= MI && NW * CB >= MI, "block too small");
  __shared__ GJ2Shared<NW, RA> sh;
  __shared__ double cf[6][P * P];
  __shared__ double Dh[P * P], Dh2[P * P];
  const int leaf = blockIdx.x;
  if (leaf >= nleaf) return;
  const LeafDesc &d = descs[leaf];
  const double *coef = (const double *)bs.d[BUF_COEF] + d.coef;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (int i = tid; i < 6 * P * P; i += NW * 64) cf[i / (P * P)][i % (P * P)] = coef[i];
  for (int i = tid; i < P * P; i += NW * 64) { Dh[i] = Dh_g[i]; Dh2[i] = Dh2_g[i]; }
  __syncthreads();
  const double sx = d.sx, sy = d.sy;
  auto entry = [&](int ga, int gb) -> double {
    const int iy = ga / P, ix = ga - iy * P, jy = gb / P, jx = gb - jy * P;
    double v = -2.0 * cf[1][ga] * sx * sy * Dh[iy * P + jy] * Dh[ix * P + jx];
    if (iy == jy) v += -cf[0][ga] * sx * sx * Dh2[ix * P + jx] + cf[3][ga] * sx * Dh[ix * P + jx];
    if (ix == jx) v += -cf[2][ga] * sy * sy * Dh2[iy * P + jy] + cf[4][ga] * sy * Dh[iy * P + jy];
    if (ga == gb) v += cf[5][ga];
    return v;
  };
  auto grid_of = [](int a) { const int y = a / PI; return (y + 1) * P + (a - y * PI) + 1; };
  if (d.Aie >= 0) {             // A_ci,ce for the leaf products
    double *Aie = (double *)bs.d[BUF_SCR] + d.Aie;
    for (int idx = tid; idx < MI * me; idx += NW * 64) {
      const int a = idx % MI, e = idx / MI;
      Aie[idx] = entry(grid_of(a), ice[e]);
    }
  }
  // rows MI .. MI + hrows - 1 (padding rows otherwise) carry D_ge,ci: they
  // are never pivots, and the sweeps turn them into -D_ge,ci A_ci,ci^-1 = -H
  // (with the columns in pivot order), the flux map of the particular
  // solution (Sec. 3.4), so H needs no product with the stored F
  const int hrows = d.hrows;
  const double *Dci = (const double *)bs.d[BUF_WS] + d.Dci;
  double a[RA][CB];
#pragma unroll
  for (int i = 0; i < RA; ++i) {
    const int row = lane + 64 * i;
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      const int col = wid + NW * b;
      double v = 0.0;
      if (col < MI) {
        if (row < MI) v = entry(grid_of(row), grid_of(col));
        else if (row - MI < hrows) v = Dci[(row - MI) + int64_t(col) * hrows];
      }
      a[i][b] = v;
    }
  }
  gj2_core<NW, RA, CB>(a, MI, lane, wid, sh);
  if (hrows > 0) {
    double *Hp = (double *)bs.d[BUF_WS] + d.H;
#pragma unroll
    for (int i = 0; i < RA; ++i) {
      const int row = lane + 64 * i;
      if (row < MI || row - MI >= hrows) continue;
#pragma unroll
      for (int b = 0; b < CB; ++b) {
        const int col = wid + NW * b;
        if (col < MI) Hp[(row - MI) + int64_t(sh.pivrow[col]) * hrows] = -a[i][b];
      }
    }
  }
  double *F = (double *)bs.d[d.fbuf] + d.F;
#pragma unroll
  for (int i = 0; i < RA; ++i) {
    const int row = lane + 64 * i;
    if (row >= MI) continue;
    const int kr = sh.stepof[row];
    const double sg = sh.sig[kr];
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      const int col = wid + NW * b;
      if (col < MI)
        F[kr + int64_t(sh.pivrow[col]) * MI] = sg * (a[i][b] + (col == kr ? 1.0 : 0.0));
    }
  }
  if (tid == 0) info[d.info] = sh.info;
}


// p = 16 runs the blocked matrix-core kernel (kernels_gjb_leaf.hip) unless
// HPS_LEAF_GJ=rank1 selects the column-owner rank-1 kernel above (same
// outputs up to rounding), kept for comparison.
static bool leaf_rank1_p16() {
  static const bool r1 = [] {
    const char *e = std::getenv("HPS_LEAF_GJ");
    return e && std::string(e) == "rank1";
  }();
  return r1;
}

hipError_t launch_gj_leaf(int p, const LeafDesc *descs, int nleaf, const Bases &bs,
                          const double *Dh, const double *Dh2, const int32_t *ice,
                          int me, int32_t *info, hipStream_t st) {
  if (nleaf <= 0) return hipSuccess;
  switch (p) {
    case 16:
      if (!leaf_rank1_p16())
        return launch_gjb_leaf(descs, nleaf, bs, Dh, Dh2, ice, me, info, st);
      hipLaunchKernelGGL((gj2_leaf_kernel<16, 8, 4, 25>), dim3(nleaf), dim3(512), 0, st, descs,
                         nleaf, bs, Dh, Dh2, ice, me, info);
      break;
    case 12:
      hipLaunchKernelGGL((gj_leaf_kernel<12, 20, 20, 5, 5>), dim3(nleaf), dim3(gj_threads<20, 20>()), 0, st,
                         descs, nleaf, bs, Dh, Dh2, ice, me, info);
      break;
    case 10:
      hipLaunchKernelGGL((gj_leaf_kernel<10, 8, 8, 8, 8>), dim3(nleaf), dim3(64), 0, st,
                         descs, nleaf, bs, Dh, Dh2, ice, me, info);
      break;
    case 8:
      hipLaunchKernelGGL((gj_leaf_kernel<8, 8, 8, 5, 5>), dim3(nleaf), dim3(64), 0, st,
                         descs, nleaf, bs, Dh, Dh2, ice, me, info);
      break;
    case 6:
      hipLaunchKernelGGL((gj_leaf_kernel<6, 8, 8, 2, 2>), dim3(nleaf), dim3(64), 0, st,
                         descs, nleaf, bs, Dh, Dh2, ice, me, info);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int gj_leaf_supported(int p) { return p == 16 || p == 12 || p == 10 || p == 8 || p == 6; }


}  // namespace hps
