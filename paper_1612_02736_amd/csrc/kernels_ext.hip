// Kernels of the solve-stage extensions: the FP64 residual of the global
// collocation system (for iterative refinement of FP32 solves), vector
// updates and reductions, and the coefficient gradient of the adjoint.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "kernels_ext.hpp"
#include "kernel_util.hpp"

namespace hps {

// One workgroup per leaf, looping over the right-hand sides (the leaf's
// coefficients and reference matrices are read once).  Residual of the
// collocated PDE at interior nodes, r = g - A u (Sec. 3.2, same A as the
// build), and the leaf's boundary fluxes D_ge,c u (Sec. 3.4) in side order
// S, E, N, W.  SHIFT = true returns sigma u - A u instead and no fluxes (the
// right side of an implicit time step, Sec. 7.6); it is a separate
// instantiation so that the residual keeps its register budget.
template <int P, bool SHIFT>
__global__ __launch_bounds__(256) void residual_kernel(
    const LeafDesc *__restrict__ leafd, int nleaf, const double *__restrict__ coef,
    const double *__restrict__ uc, const double *__restrict__ g, double sigma,
    double *__restrict__ r1, double *__restrict__ flux, const double *__restrict__ Dh_g,
    const double *__restrict__ Dh2_g,
    const double *__restrict__ Lloc_g, int q, int nrhs) {
  constexpr int PP = P * P, PI = P - 2, MI = PI * PI;
  __shared__ double u[PP], dx[PP], dy[PP], Dh[PP], Dh2[PP], cf[6][PP], Lloc[P * P];
  const int leaf = blockIdx.x, tid = threadIdx.x;
  const int64_t nl = nleaf;
  const LeafDesc &d = leafd[leaf];
  const double sx = d.sx, sy = d.sy;
  for (int i = tid; i < PP; i += 256) {
    Dh[i] = Dh_g[i];
    Dh2[i] = Dh2_g[i];
  }
  for (int i = tid; i < q * P; i += 256) Lloc[i] = Lloc_g[i];
  for (int i = tid; i < 6 * PP; i += 256) cf[i / PP][i % PP] = coef[int64_t(leaf) * 6 * PP + i];
  for (int r = 0; r < nrhs; ++r) {
    for (int i = tid; i < PP; i += 256) u[i] = uc[(int64_t(r) * nl + leaf) * PP + i];
    __syncthreads();
    // reference-coordinate first derivatives on the whole grid
    for (int t = tid; t < PP; t += 256) {
      const int iy = t / P, ix = t - iy * P;
      double sxv = 0.0, syv = 0.0;
#pragma unroll
      for (int j = 0; j < P; ++j) {
        sxv += Dh[ix * P + j] * u[iy * P + j];
        syv += Dh[iy * P + j] * u[j * P + ix];
      }
      dx[t] = sxv;
      dy[t] = syv;
    }
    __syncthreads();
    for (int a = tid; a < MI; a += 256) {
      const int y = a / PI, iy = y + 1, ix = a - y * PI + 1, t = iy * P + ix;
      double uxx = 0.0, uyy = 0.0, uxy = 0.0;
#pragma unroll
      for (int j = 0; j < P; ++j) {
        uxx += Dh2[ix * P + j] * u[iy * P + j];
        uyy += Dh2[iy * P + j] * u[j * P + ix];
        uxy += Dh[iy * P + j] * dx[j * P + ix];
      }
      const double Au = -cf[0][t] * sx * sx * uxx - 2.0 * cf[1][t] * sx * sy * uxy -
                        cf[2][t] * sy * sy * uyy + cf[3][t] * sx * dx[t] + cf[4][t] * sy * dy[t] +
                        cf[5][t] * u[t];
      const int64_t o = (int64_t(r) * nl + leaf) * MI + a;
      if constexpr (SHIFT) r1[o] = sigma * u[t] - Au;
      else r1[o] = g[o] - Au;
    }
    for (int k = SHIFT ? 4 * q : tid; k < 4 * q; k += 256) {
      const int side = k / q, kk = k - side * q;
      double v = 0.0;
      for (int j = 0; j < P; ++j) {
        const double l = Lloc[kk * P + j];
        if (side == 0) v += l * sy * dy[0 * P + j];
        else if (side == 1) v += l * sx * dx[j * P + (P - 1)];
        else if (side == 2) v += l * sy * dy[(P - 1) * P + j];
        else v += l * sx * dx[j * P + 0];
      }
      flux[(int64_t(r) * nl + leaf) * 4 * q + k] = v;
    }
    __syncthreads();   // u, dx, dy are rewritten for the next right-hand side
  }
}

// p = 16: the same residual with the derivative products as 16 x 16 matrix
// products on the matrix cores.  With U(iy, ix) = u[iy * 16 + ix] and Dh the
// reference first-derivative matrix (row-major), Dh2 = Dh^2:
//   Ux = U Dh^T, Uxx = U Dh2^T, Uy = Dh U, Uyy = Dh2 U, Uxy = Dh Ux.
// One workgroup of four wavefronts per leaf; wavefront w takes the
// right-hand sides w, w + 4, ...  Layouts of v_mfma_f64_16x16x4: lane l
// supplies A[l & 15][k0 + (l >> 4)] and B[k0 + (l >> 4)][l & 15], and result
// register v of lane l is entry ((l >> 4) + 4 v, l & 15).  The A fragment of
// Dh, Dh[l & 15][k0 + (l >> 4)], is also the B fragment of Dh^T, and the B
// fragment of U at k-step v is U at result entry v, so u is read once.  Ux
// and Uy pass through the wavefront's own LDS tile (for Uxy and the fluxes).
template <bool SHIFT>
__global__ __launch_bounds__(256) void residual16_kernel(
    const LeafDesc *__restrict__ leafd, int nleaf, const double *__restrict__ coef,
    const double *__restrict__ uc, const double *__restrict__ g, double sigma,
    double *__restrict__ r1, double *__restrict__ flux, const double *__restrict__ Dh_g,
    const double *__restrict__ Dh2_g, const double *__restrict__ Lloc_g, int q, int nrhs) {
  constexpr int P = 16, PP = P * P, PI = P - 2, MI = PI * PI;
  __shared__ double Wx[4][P][P + 1], Wy[4][P][P + 1];
  __shared__ double Ll[P * P];
  const int leaf = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int64_t nl = nleaf;
  const LeafDesc &d = leafd[leaf];
  const double sx = d.sx, sy = d.sy;
  double fD[4], fD2[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    fD[kk] = Dh_g[li * P + 4 * kk + lk];
    fD2[kk] = Dh2_g[li * P + 4 * kk + lk];
  }
  // coefficients at this lane's result entries, folded with the scalings
  double a0[4], a1[4], a2[4], a3[4], a4[4], a5[4];
  const double *cl = coef + int64_t(leaf) * 6 * PP;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int t = (lk + 4 * v) * P + li;
    a0[v] = -cl[t] * sx * sx;
    a1[v] = -2.0 * cl[PP + t] * sx * sy;
    a2[v] = -cl[2 * PP + t] * sy * sy;
    a3[v] = cl[3 * PP + t] * sx;
    a4[v] = cl[4 * PP + t] * sy;
    a5[v] = cl[5 * PP + t];
  }
  if (!SHIFT)
    for (int i = tid; i < q * P; i += 256) Ll[i] = Lloc_g[i];
  __syncthreads();
  for (int r = w; r < nrhs; r += 4) {
    const double *u = uc + (int64_t(r) * nl + leaf) * PP;
    double uA[4], uB[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      uA[kk] = u[li * P + 4 * kk + lk];
      uB[kk] = u[(4 * kk + lk) * P + li];
    }
    dbl4 ux = {0.0, 0.0, 0.0, 0.0}, uxx = ux, uy = ux, uyy = ux, uxy = ux;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      ux = __builtin_amdgcn_mfma_f64_16x16x4f64(uA[kk], fD[kk], ux, 0, 0, 0);
      uxx = __builtin_amdgcn_mfma_f64_16x16x4f64(uA[kk], fD2[kk], uxx, 0, 0, 0);
      uy = __builtin_amdgcn_mfma_f64_16x16x4f64(fD[kk], uB[kk], uy, 0, 0, 0);
      uyy = __builtin_amdgcn_mfma_f64_16x16x4f64(fD2[kk], uB[kk], uyy, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Wx[w][lk + 4 * v][li] = ux[v];
      Wy[w][lk + 4 * v][li] = uy[v];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
      uxy = __builtin_amdgcn_mfma_f64_16x16x4f64(fD[kk], Wx[w][4 * kk + lk][li], uxy, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = lk + 4 * v, col = li;
      if (row >= 1 && row <= PI && col >= 1 && col <= PI) {
        const double Au = a0[v] * uxx[v] + a1[v] * uxy[v] + a2[v] * uyy[v] + a3[v] * ux[v] +
                          a4[v] * uy[v] + a5[v] * uB[v];
        const int64_t o = (int64_t(r) * nl + leaf) * MI + (row - 1) * PI + (col - 1);
        if constexpr (SHIFT) r1[o] = sigma * uB[v] - Au;
        else r1[o] = g[o] - Au;
      }
    }
    if constexpr (!SHIFT) {
      for (int k = lane; k < 4 * q; k += 64) {
        const int side = k / q, kk = k - side * q;
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < P; ++j) {
          const double l = Ll[kk * P + j];
          const double dv = side == 0 ? sy * Wy[w][0][j]
                          : side == 1 ? sx * Wx[w][j][P - 1]
                          : side == 2 ? sy * Wy[w][P - 1][j]
                                      : sx * Wx[w][j][0];
          v = fma(l, dv, v);
        }
        flux[(int64_t(r) * nl + leaf) * 4 * q + k] = v;
      }
    }
    // this wavefront's LDS tiles are rewritten by its next right-hand side
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// Residual of the flux rows, written RHS-interleaved (jump[node * nrhs + r]):
// at an interior node, the beta side's leaf flux minus the alpha side's
// (fb, fa); at a Neumann node (fb < 0), the data psi (f[fp]) minus the leaf
// flux.
__global__ __launch_bounds__(256) void jump_kernel(const int32_t *__restrict__ jn,
                                                   const int32_t *__restrict__ fa,
                                                   const int32_t *__restrict__ fb,
                                                   const int32_t *__restrict__ fp, int64_t n,
                                                   const double *__restrict__ flux,
                                                   int64_t flux_stride,
                                                   const double *__restrict__ f,
                                                   int64_t f_stride, double *__restrict__ jump,
                                                   int nrhs) {
  const int64_t tot = n * nrhs;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int r = int(e / n);
    const int64_t i = e - int64_t(r) * n;
    const double other = fb[i] >= 0 ? flux[r * flux_stride + fb[i]] : f[r * f_stride + fp[i]];
    jump[int64_t(jn[i]) * nrhs + r] = other - flux[r * flux_stride + fa[i]];
  }
}

// x(k, r) += y(k, r); y(k, r) = x(k, r)  (strided blocks of n per RHS)
__global__ __launch_bounds__(256) void accumulate_kernel(double *__restrict__ x, int64_t xs,
                                                         double *__restrict__ y, int64_t ys,
                                                         int64_t n, int nrhs, int copy_back) {
  const int64_t tot = n * nrhs;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int r = int(e / n);
    const int64_t k = e - int64_t(r) * n;
    const double v = x[r * xs + k] + y[r * ys + k];
    x[r * xs + k] = v;
    if (copy_back) y[r * ys + k] = v;
  }
}

// out[0] = max |a|, out[1] = max |b| over n entries, a NaN entry counting
// as +inf (fmax would drop it).  Non-negative doubles order like their bit
// patterns, so each workgroup's maximum is merged with an unsigned 64-bit
// atomic max; out must hold zeros on entry.
__global__ __launch_bounds__(256) void maxabs2_kernel(const double *__restrict__ a,
                                                      const double *__restrict__ b, int64_t n,
                                                      unsigned long long *__restrict__ out) {
  __shared__ double sa[256], sb[256];
  double ma = 0.0, mb = 0.0;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < n;
       e += int64_t(gridDim.x) * blockDim.x) {
    const double va = fabs(a[e]), vb = fabs(b[e]);
    ma = fmax(ma, va == va ? va : HUGE_VAL);
    mb = fmax(mb, vb == vb ? vb : HUGE_VAL);
  }
  sa[threadIdx.x] = ma;
  sb[threadIdx.x] = mb;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sa[threadIdx.x] = fmax(sa[threadIdx.x], sa[threadIdx.x + s]);
      sb[threadIdx.x] = fmax(sb[threadIdx.x], sb[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicMax(out, (unsigned long long)__double_as_longlong(sa[0]));
    atomicMax(out + 1, (unsigned long long)__double_as_longlong(sb[0]));
  }
}

__global__ void zero2_kernel(unsigned long long *out) {
  if (threadIdx.x < 2) out[threadIdx.x] = 0ull;
}

// cbar = -gbar * u at interior nodes, 0 at exterior nodes
__global__ __launch_bounds__(256) void cbar_kernel(const double *__restrict__ u,
                                                   const double *__restrict__ gbar,
                                                   double *__restrict__ cbar, int p, int64_t nl,
                                                   int nrhs) {
  const int pp = p * p, pi = p - 2;
  const int64_t tot = int64_t(nrhs) * nl * pp;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t lr = e / pp;
    const int t = int(e - lr * pp), iy = t / p, ix = t - iy * p;
    double v = 0.0;
    if (iy > 0 && iy < p - 1 && ix > 0 && ix < p - 1)
      v = -gbar[lr * pi * pi + (iy - 1) * pi + (ix - 1)] * u[e];
    cbar[e] = v;
  }
}

static inline unsigned grid1(int64_t n) {
  int64_t b = (n + 255) / 256;
  return unsigned(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

template <bool SHIFT>
static hipError_t launch_residual_t(int p, const LeafDesc *leafd, int nleaf, const double *coef,
                                    const double *uc, const double *g, double sigma, double *r1,
                                    double *flux, const double *Dh, const double *Dh2,
                                    const double *Lloc, int q, int nrhs, hipStream_t st) {
  dim3 grid(nleaf);
  if (p == 16) {
    hipLaunchKernelGGL((residual16_kernel<SHIFT>), grid, dim3(256), 0, st, leafd, nleaf, coef, uc,
                       g, sigma, r1, flux, Dh, Dh2, Lloc, q, nrhs);
    return hipGetLastError();
  }
  switch (p) {
#define HPS_RES_CASE(PV)                                                                      \
    case PV:                                                                                  \
      hipLaunchKernelGGL((residual_kernel<PV, SHIFT>), grid, dim3(256), 0, st, leafd, nleaf,  \
                         coef, uc, g, sigma, r1, flux, Dh, Dh2, Lloc, q, nrhs);               \
      break;
    HPS_RES_CASE(16)
    HPS_RES_CASE(12)
    HPS_RES_CASE(10)
    HPS_RES_CASE(8)
    HPS_RES_CASE(6)
#undef HPS_RES_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_residual(int p, const LeafDesc *leafd, int nleaf, const double *coef,
                           const double *uc, const double *g, double sigma, double *r1,
                           double *flux, const double *Dh, const double *Dh2, const double *Lloc,
                           int q, int nrhs, hipStream_t st) {
  if (g) {
    if (!flux) return hipErrorInvalidValue;
    return launch_residual_t<false>(p, leafd, nleaf, coef, uc, g, sigma, r1, flux, Dh, Dh2, Lloc,
                                    q, nrhs, st);
  }
  return launch_residual_t<true>(p, leafd, nleaf, coef, uc, g, sigma, r1, flux, Dh, Dh2, Lloc,
                                 q, nrhs, st);
}

hipError_t launch_jump(const int32_t *jn, const int32_t *fa, const int32_t *fb,
                       const int32_t *fp, int64_t n, const double *flux, int64_t flux_stride,
                       const double *f, int64_t f_stride, double *jump, int nrhs,
                       hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(jump_kernel, dim3(grid1(n * nrhs)), dim3(256), 0, st, jn, fa, fb, fp, n,
                     flux, flux_stride, f, f_stride, jump, nrhs);
  return hipGetLastError();
}

hipError_t launch_accumulate(double *x, int64_t xs, double *y, int64_t ys, int64_t n, int nrhs,
                             int copy_back, hipStream_t st) {
  hipLaunchKernelGGL(accumulate_kernel, dim3(grid1(n * nrhs)), dim3(256), 0, st, x, xs, y, ys, n,
                     nrhs, copy_back);
  return hipGetLastError();
}

hipError_t launch_maxabs2(const double *a, const double *b, int64_t n, double *out,
                          hipStream_t st) {
  unsigned long long *o = reinterpret_cast<unsigned long long *>(out);
  hipLaunchKernelGGL(zero2_kernel, dim3(1), dim3(64), 0, st, o);
  // a few workgroups per CU: each merges its maximum with one atomic
  const int64_t nb = std::min<int64_t>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(maxabs2_kernel, dim3(unsigned(nb < 1 ? 1 : nb)), dim3(256), 0, st, a, b, n,
                     o);
  return hipGetLastError();
}

hipError_t launch_cbar(const double *u, const double *gbar, double *cbar, int p, int64_t nl,
                       int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(cbar_kernel, dim3(grid1(int64_t(nrhs) * nl * p * p)), dim3(256), 0, st, u,
                     gbar, cbar, p, nl, nrhs);
  return hipGetLastError();
}

}  // namespace hps
