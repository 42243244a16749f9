// Interface inversions X = (T33a - T33b)^-1 of the merges (Sec. 4) that fit
// one workgroup's registers (m <= 196).
#include "gj_core.hpp"

namespace hps {

template <int TR, int TC, int RA, int CB>
__global__ __launch_bounds__((gj_threads<TR, TC>())) void gj_merge_kernel(
    const MergeInvDesc *__restrict__ descs, int nd, Bases bs,
    int32_t *__restrict__ info) {
  __shared__ GJShared<TR, TC, RA, CB> sh;
  const int idx = blockIdx.x;
  if (idx >= nd) return;
  const MergeInvDesc &d = descs[idx];
  const double *Ta = (const double *)bs.d[BUF_WS] + d.Ta;
  const double *Tb = (const double *)bs.d[BUF_WS] + d.Tb;
  const int n = d.m;
  const int tid = threadIdx.x;
  int tr, tc;
  gj_owner<TR, TC, RA, CB>(tid, tr, tc);
  double a[RA][CB];
#pragma unroll
  for (int i = 0; i < RA; ++i) {
    const int row = tr + TR * i;
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      const int col = tc + TC * b;
      a[i][b] = (row < n && col < n)
                    ? Ta[row + int64_t(col) * d.lda] - Tb[row + int64_t(col) * d.ldb]
                    : 0.0;
    }
  }
  gj_core<TR, TC, RA, CB>(a, n, tr, tc, sh);
  gj_store<TR, TC, RA, CB>(a, n, tr, tc, sh, (double *)bs.d[BUF_WS] + d.X, n);
  if (tid == 0) info[d.info] = sh.info;
}

// Interface inversion X = (T33a - T33b)^-1 on the column-owner core (m up to
// 64 RA and NW CB): same storage of X as gj_merge_kernel.
template <int NW, int RA, int CB>
__global__ __launch_bounds__(NW * 64) void gj2_merge_kernel(
    const MergeInvDesc *__restrict__ descs, int nd, Bases bs,
    int32_t *__restrict__ info) {
  __shared__ GJ2Shared<NW, RA> sh;
  const int idx = blockIdx.x;
  if (idx >= nd) return;
  const MergeInvDesc &d = descs[idx];
  const double *Ta = (const double *)bs.d[BUF_WS] + d.Ta;
  const double *Tb = (const double *)bs.d[BUF_WS] + d.Tb;
  const int n = d.m;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  double a[RA][CB];
#pragma unroll
  for (int i = 0; i < RA; ++i) {
    const int row = lane + 64 * i;
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      const int col = wid + NW * b;
      a[i][b] = (row < n && col < n)
                    ? Ta[row + int64_t(col) * d.lda] - Tb[row + int64_t(col) * d.ldb]
                    : 0.0;
    }
  }
  gj2_core<NW, RA, CB>(a, n, lane, wid, sh);
  double *X = (double *)bs.d[BUF_WS] + d.X;
#pragma unroll
  for (int i = 0; i < RA; ++i) {
    const int row = lane + 64 * i;
    if (row >= n) continue;
    const int kr = sh.stepof[row];
    const double sg = sh.sig[kr];
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      const int col = wid + NW * b;
      if (col < n) X[kr + int64_t(sh.pivrow[col]) * n] = sg * (a[i][b] + (col == kr ? 1.0 : 0.0));
    }
  }
  if (tid == 0) info[d.info] = sh.info;
}


// size classes of the register-resident interface inversion
int gj_merge_class(int m) {
  if (m <= 32) return 0;
  if (m <= 64) return 1;
  if (m <= 128) return 2;
  if (m <= 196) return 3;
  return -1;
}

hipError_t launch_gj_merge(int cls, const MergeInvDesc *descs, int nd, const Bases &bs,
                           int32_t *info, hipStream_t st) {
  if (nd <= 0) return hipSuccess;
  switch (cls) {
    case 0:
      hipLaunchKernelGGL((gj_merge_kernel<8, 8, 4, 4>), dim3(nd), dim3(64), 0, st, descs, nd,
                         bs, info);
      break;
    case 1:
      hipLaunchKernelGGL((gj2_merge_kernel<4, 1, 16>), dim3(nd), dim3(256), 0, st, descs, nd,
                         bs, info);
      break;
    case 2:
      hipLaunchKernelGGL((gj2_merge_kernel<8, 2, 16>), dim3(nd), dim3(512), 0, st, descs, nd,
                         bs, info);
      break;
    case 3:
      hipLaunchKernelGGL((gj2_merge_kernel<8, 4, 25>), dim3(nd), dim3(512), 0, st, descs, nd,
                         bs, info);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}


}  // namespace hps
