// Leaf interior inversions F = A_ci,ci^-1 of the build stage (Sec. 3.3).
#include "gj_core.hpp"

#include <cstdlib>
#include <string>

namespace hps {

template <int P, int TR, int TC, int RA, int CB>
__global__ __launch_bounds__((gj_threads<TR, TC>())) void gj_leaf_kernel(
    const LeafDesc *__restrict__ descs, int nleaf, Bases bs,
    const double *__restrict__ Dh_g, const double *__restrict__ Dh2_g,
    int32_t *__restrict__ info) {
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
    int32_t *__restrict__ info) {
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
                          const double *Dh, const double *Dh2, int32_t *info, hipStream_t st) {
  if (nleaf <= 0) return hipSuccess;
  switch (p) {
    case 16:
      if (!leaf_rank1_p16())
        return launch_gjb_leaf(descs, nleaf, bs, Dh, Dh2, info, st);
      hipLaunchKernelGGL((gj2_leaf_kernel<16, 8, 4, 25>), dim3(nleaf), dim3(512), 0, st, descs,
                         nleaf, bs, Dh, Dh2, info);
      break;
    case 12:
      hipLaunchKernelGGL((gj_leaf_kernel<12, 20, 20, 5, 5>), dim3(nleaf), dim3(gj_threads<20, 20>()), 0, st,
                         descs, nleaf, bs, Dh, Dh2, info);
      break;
    case 10:
      hipLaunchKernelGGL((gj_leaf_kernel<10, 8, 8, 8, 8>), dim3(nleaf), dim3(64), 0, st,
                         descs, nleaf, bs, Dh, Dh2, info);
      break;
    case 8:
      hipLaunchKernelGGL((gj_leaf_kernel<8, 8, 8, 5, 5>), dim3(nleaf), dim3(64), 0, st,
                         descs, nleaf, bs, Dh, Dh2, info);
      break;
    case 6:
      hipLaunchKernelGGL((gj_leaf_kernel<6, 8, 8, 2, 2>), dim3(nleaf), dim3(64), 0, st,
                         descs, nleaf, bs, Dh, Dh2, info);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int gj_leaf_supported(int p) { return p == 16 || p == 12 || p == 10 || p == 8 || p == 6; }

// B = A_ci,ce L for every leaf (Sec. 3.3: the leaf's particular-solution
// flux map needs S_ci = -F A_ci,ce L).  An interior row a of the collocated
// operator restricted to the exterior nodes is
//   cxy(a) K1(a, :) + cxx(a) K2(a, :) + cx(a) K3(a, :) + cyy(a) K4(a, :) + cy(a) K5(a, :)
// with fixed K_t (products of the reference differentiation matrices), so
// B(a, :) = sum_t c_t(a) M_t(a, :) with M_t = K_t L formed once per role on
// the host: five row-scaled fixed matrices instead of a product with the
// leaf's A_ci,ce.  Workgroup (c, jb) takes chunk c of leaves that share a
// role (chunks[2c] = first entry in lidx, chunks[2c + 1] = count) and the
// columns 12 jb .. 12 jb + 11 of B: thread a keeps row a of that slice of the
// five M_t in registers across the chunk's leaves and writes row a of each
// leaf's B slice (column-major, ld mi).
constexpr int kLeafBCols = 12;

__global__ __launch_bounds__(256) void leaf_b_kernel(const LeafDesc *__restrict__ descs,
                                                     Bases bs, const int32_t *__restrict__ chunks,
                                                     const int32_t *__restrict__ lidx, int p,
                                                     int g4) {
  const int first = chunks[2 * blockIdx.x], cnt = chunks[2 * blockIdx.x + 1];
  const int pi = p - 2, mi = pi * pi, pp = p * p;
  const int a = threadIdx.x;
  if (a >= mi) return;
  const int j0 = kLeafBCols * blockIdx.y, nj = min(kLeafBCols, g4 - j0);
  const int64_t tot = int64_t(mi) * g4;
  const int y = a / pi, ga = (y + 1) * p + (a - y * pi) + 1;   // grid node of interior row a
  double m[5][kLeafBCols];
  {
    const double *M = (const double *)bs.d[BUF_WS] + descs[lidx[first]].Mb;
#pragma unroll
    for (int t = 0; t < 5; ++t)
#pragma unroll
      for (int j = 0; j < kLeafBCols; ++j)
        m[t][j] = j < nj ? M[t * tot + a + int64_t(j0 + j) * mi] : 0.0;
  }
#pragma unroll 4
  for (int k = 0; k < cnt; ++k) {
    const LeafDesc &d = descs[lidx[first + k]];
    const double *cf = (const double *)bs.d[BUF_COEF] + d.coef;
    const double sx = d.sx, sy = d.sy;
    const double c1 = -2.0 * cf[pp + ga] * sx * sy, c2 = -cf[ga] * sx * sx,
                 c3 = cf[3 * pp + ga] * sx, c4 = -cf[2 * pp + ga] * sy * sy,
                 c5 = cf[4 * pp + ga] * sy;
    double *B = (double *)bs.d[BUF_SCR] + d.Bout + a + int64_t(j0) * mi;
#pragma unroll
    for (int j = 0; j < kLeafBCols; ++j) {
      double v = c1 * m[0][j];
      v = fma(c2, m[1][j], v);
      v = fma(c3, m[2][j], v);
      v = fma(c4, m[3][j], v);
      v = fma(c5, m[4][j], v);
      if (j < nj) B[int64_t(j) * mi] = v;
    }
  }
}

hipError_t launch_leaf_b(const LeafDesc *descs, const int32_t *chunks, int nchunks,
                         const int32_t *lidx, const Bases &bs, int p, int g4, hipStream_t st) {
  if (nchunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(leaf_b_kernel, dim3(nchunks, (g4 + kLeafBCols - 1) / kLeafBCols), dim3(256),
                     0, st, descs, bs, chunks, lidx, p, g4);
  return hipGetLastError();
}

}  // namespace hps
