// Solve-stage applies on the vector ALU (fewer than 16 right-hand sides),
// split-K finalize and vector utilities.
#include "kernel_util.hpp"

namespace hps {


template <typename TA, typename TC_, int NR, bool TRANS>
__global__ __launch_bounds__(256) void apply_kernel(
    const ApplyDesc *__restrict__ descs, const int32_t *__restrict__ tmap,
    int64_t ntiles, Bases bs, int nrhs) {
  constexpr int KC = NR >= 16 ? 64 : 256;
  constexpr int RC = NR < 8 ? NR : 8;     // RHS per cross-wave reduction round
  __shared__ TC_ Bsh[KC][NR];
  __shared__ TC_ red[4][64][RC];
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= ntiles) return;
  const ApplyDesc &d = descs[tmap[tile]];
  const int64_t t = tile - d.tile0;
  const int rbi = int(t % d.rb), slice = int(t / d.rb);
  const int K = d.K1 + (d.mode == 0 ? d.K2 : 0);
  const int kper = (K + d.ksl - 1) / d.ksl;
  const int k0 = slice * kper, k1 = min(K, k0 + kper);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int row = rbi * 64 + lane;
  const int r0 = blockIdx.y * NR;
  const TA *A = (const TA *)bs.d[d.abuf] + d.aoff;
  const int lda = d.lda;
  TC_ acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) acc[r] = TC_(0);
  for (int kc = k0; kc < k1; kc += KC) {
    const int kn = min(KC, k1 - kc);
    for (int e = tid; e < kn * NR; e += 256) {
      const int kk = e % kn, r = e / kn, k = kc + kk, rg = r0 + r;
      double v = 0.0;
      if (rg < nrhs) {
        if (d.mode == 0) {
          v = k < d.K1 ? vload(bs, d.B1, k, rg, nrhs) : vload(bs, d.B2, k - d.K1, rg, nrhs);
        } else if (d.mode == 1) {
          v = vload(bs, d.B1, k, rg, nrhs) - vload(bs, d.B2, k, rg, nrhs);
          if (d.B3.buf >= 0) v += vload(bs, d.B3, k, rg, nrhs);
        } else {
          v = vload(bs, d.B1, k, rg, nrhs) + vload(bs, d.B2, k, rg, nrhs);
        }
      }
      Bsh[kk][r] = TC_(v);
    }
    __syncthreads();
    const int q4 = (kn + 3) >> 2, ka = wid * q4, kz = min(kn, ka + q4);
    if (row < d.M) {
      if (!TRANS) {
        // output row `row` of A (column-major): stride lda along k
        const TA *Ap = A + row + int64_t(kc) * lda;
#pragma unroll 8
        for (int kk = ka; kk < kz; ++kk) {
          const TC_ av = TC_(Ap[int64_t(kk) * lda]);
#pragma unroll
          for (int r = 0; r < NR; ++r) acc[r] = fma(av, Bsh[kk][r], acc[r]);
        }
      } else {
        // output = column `row` of A: contiguous along k
        const TA *Ap = A + int64_t(row) * lda + kc;
#pragma unroll 8
        for (int kk = ka; kk < kz; ++kk) {
          const TC_ av = TC_(Ap[kk]);
#pragma unroll
          for (int r = 0; r < NR; ++r) acc[r] = fma(av, Bsh[kk][r], acc[r]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int rc = 0; rc < NR; rc += RC) {
#pragma unroll
    for (int r = 0; r < RC; ++r) red[wid][lane][r] = acc[rc + r];
    __syncthreads();
    if (wid == 0 && row < d.M) {
#pragma unroll
      for (int r = 0; r < RC; ++r) {
        const int rg = r0 + rc + r;
        if (rg >= nrhs) continue;
        const double s = double(red[0][lane][r]) + double(red[1][lane][r]) +
                         double(red[2][lane][r]) + double(red[3][lane][r]);
        if (d.ksl == 1) {
          double val = d.alpha * s;
          if (d.D.buf >= 0) val += d.beta * vload(bs, d.D, row, rg, nrhs);
          *vaddr(bs, d.C, row, rg, nrhs) = val;
        } else {
          ((double *)bs.d[BUF_SCR])[d.part * nrhs + (int64_t(slice) * nrhs + rg) * d.M + row] = s;
        }
      }
    }
    __syncthreads();
  }
}


// Sum the split-K partials of each descriptor in slice order.
__global__ __launch_bounds__(256) void apply_finalize_kernel(
    const ApplyDesc *__restrict__ descs, const int32_t *__restrict__ list, int nlist,
    Bases bs, int nrhs) {
  const ApplyDesc &d = descs[list[blockIdx.y]];
  const int64_t tot = int64_t(d.M) * nrhs;
  const double *part = (const double *)bs.d[BUF_SCR] + d.part * nrhs;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int rg = int(e / d.M), row = int(e - int64_t(rg) * d.M);
    double s = 0.0;
    for (int sl = 0; sl < d.ksl; ++sl) s += part[(int64_t(sl) * nrhs + rg) * d.M + row];
    double val = d.alpha * s;
    if (d.D.buf >= 0) val += d.beta * vload(bs, d.D, row, rg, nrhs);
    *vaddr(bs, d.C, row, rg, nrhs) = val;
  }
}

// dst(map_d(i), r) = src(map_s(i), r) for i < n, r < nrhs
__global__ __launch_bounds__(256) void copy_map_kernel(Bases bs, VRef dst, VRef src,
                                                       int64_t n, int nrhs) {
  const int64_t tot = n * nrhs;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int r = int(e / n);
    const int64_t i = e - int64_t(r) * n;
    *vaddr(bs, dst, i, r, nrhs) = vload(bs, src, i, r, nrhs);
  }
}

__global__ __launch_bounds__(256) void vecop_kernel(const VecOpDesc *__restrict__ descs,
                                                    int nd, Bases bs, int nrhs) {
  const VecOpDesc &d = descs[blockIdx.y];
  const int64_t tot = int64_t(d.n) * nrhs;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int r = int(e / d.n);
    const int64_t k = e - int64_t(r) * d.n;
    double v = 0.0;
    if (d.a.buf >= 0) v += d.ca * vload(bs, d.a, k, r, nrhs);
    if (d.b.buf >= 0) v += d.cb * vload(bs, d.b, k, r, nrhs);
    *vaddr(bs, d.dst, k, r, nrhs) = v;
  }
}

__global__ __launch_bounds__(256) void cast_f32_kernel(const double *__restrict__ src,
                                                       float *__restrict__ dst, int64_t n) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < n;
       e += int64_t(gridDim.x) * blockDim.x)
    dst[e] = float(src[e]);
}

// flag = 1 if any element differs from the same element of the first block
// of `per` (translation-invariant builds: every leaf's coefficients equal
// leaf 0's); NaN counts as different
__global__ __launch_bounds__(256) void block_diff_kernel(const double *__restrict__ src,
                                                         int64_t per, int64_t n,
                                                         int32_t *__restrict__ flag) {
  bool diff = false;
  for (int64_t e = per + blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < n;
       e += int64_t(gridDim.x) * blockDim.x)
    diff |= !(src[e] == src[e % per]);
  if (diff) atomicOr(flag, 1);
}

__global__ __launch_bounds__(256) void fill_kernel(double *__restrict__ dst, double v, int64_t n) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < n;
       e += int64_t(gridDim.x) * blockDim.x)
    dst[e] = v;
}


template <typename TA, typename TC_, bool TRANS>
void launch_apply_valu_t(const ApplyDesc *descs, const int32_t *tmap,
                           int64_t ntiles, const Bases &bs, int nrhs, hipStream_t st) {
  const int64_t nblk = (ntiles + 7) / 8 * 8;
#define HPS_APPLY_NR(NRV)                                                                  \
  hipLaunchKernelGGL((apply_kernel<TA, TC_, NRV, TRANS>),                                 \
                     dim3(unsigned(nblk), unsigned((nrhs + NRV - 1) / NRV)), dim3(256), 0, st, \
                     descs, tmap, ntiles, bs, nrhs)
  if (nrhs > 16) HPS_APPLY_NR(32);
  else if (nrhs > 8) HPS_APPLY_NR(16);
  else if (nrhs > 4) HPS_APPLY_NR(8);
  else if (nrhs > 2) HPS_APPLY_NR(4);
  else if (nrhs > 1) HPS_APPLY_NR(2);
  else HPS_APPLY_NR(1);
#undef HPS_APPLY_NR
}


template void launch_apply_valu_t<double, double, true>(const ApplyDesc *, const int32_t *, int64_t, const Bases &, int, hipStream_t);
template void launch_apply_valu_t<double, double, false>(const ApplyDesc *, const int32_t *, int64_t, const Bases &, int, hipStream_t);
template void launch_apply_valu_t<float, float, true>(const ApplyDesc *, const int32_t *, int64_t, const Bases &, int, hipStream_t);
template void launch_apply_valu_t<float, float, false>(const ApplyDesc *, const int32_t *, int64_t, const Bases &, int, hipStream_t);

hipError_t launch_apply_finalize(const ApplyDesc *descs, const int32_t *list, int nlist,
                                 int64_t maxm, const Bases &bs, int nrhs, hipStream_t st) {
  if (nlist <= 0) return hipSuccess;
  hipLaunchKernelGGL(apply_finalize_kernel, dim3(grid_1d(maxm * nrhs, 256), nlist), dim3(256),
                     0, st, descs, list, nlist, bs, nrhs);
  return hipGetLastError();
}

hipError_t launch_copy_map(const Bases &bs, const VRef &dst, const VRef &src, int64_t n,
                           int nrhs, hipStream_t st) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_map_kernel, dim3(grid_1d(n * nrhs)), dim3(256), 0, st, bs, dst, src,
                     n, nrhs);
  return hipGetLastError();
}

hipError_t launch_vecop(const VecOpDesc *descs, int nd, int64_t maxn, const Bases &bs, int nrhs,
                        hipStream_t st) {
  if (nd <= 0) return hipSuccess;
  hipLaunchKernelGGL(vecop_kernel, dim3(grid_1d(maxn * nrhs, 64), nd), dim3(256), 0, st, descs,
                     nd, bs, nrhs);
  return hipGetLastError();
}

hipError_t launch_block_diff(const double *src, int64_t per, int64_t n, int32_t *flag,
                             hipStream_t st) {
  if (n <= per) return hipSuccess;
  hipLaunchKernelGGL(block_diff_kernel, dim3(grid_1d(n - per, 1024)), dim3(256), 0, st, src, per,
                     n, flag);
  return hipGetLastError();
}

hipError_t launch_cast_f32(const double *src, float *dst, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(cast_f32_kernel, dim3(grid_1d(n)), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_fill(double *dst, double v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_1d(n)), dim3(256), 0, st, dst, v, n);
  return hipGetLastError();
}


}  // namespace hps
