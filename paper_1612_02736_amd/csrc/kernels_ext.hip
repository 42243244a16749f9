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

// FP64 residual of the collocated PDE at interior nodes, r = g - A u
// (Sec. 3.2, the same A as the build), and the leaf's boundary fluxes
// D_ge,c u (Sec. 3.4) in side order S, E, N, W.  SHIFT = true returns
// sigma u - A u instead and no fluxes (the right side of an implicit time
// step, Sec. 7.6).
// p <= 16: the same residual with the derivative products as 16 x 16 matrix
// products on the matrix cores (a p x p grid sits in the top-left corner of
// a zero-padded 16 x 16 tile, which leaves the products on the grid exact).
// With U(iy, ix) = u[iy * p + ix] and Dh the reference first-derivative
// matrix (row-major), Dh2 = Dh^2:
//   Ux = U Dh^T, Uxx = U Dh2^T, Uy = Dh U, Uyy = Dh2 U, Uxy = Dh Ux.
// Workgroup (leaf, j) has four wavefronts; wavefront w takes right-hand side
// 4 j + w, so every wavefront has one independent chain of loads, products
// and stores (the four right-hand sides of a leaf share its coefficients
// through the L2 cache).  Layouts of v_mfma_f64_16x16x4: lane l supplies
// A[l & 15][k0 + (l >> 4)] and B[k0 + (l >> 4)][l & 15], and result register
// v of lane l is entry ((l >> 4) + 4 v, l & 15).  The A fragment of Dh,
// Dh[l & 15][k0 + (l >> 4)], is also the B fragment of Dh^T.  u and g are
// read and r1 written with coalesced accesses through the wavefront's own
// LDS tiles; Ux and Uy pass through LDS too (for Uxy and the fluxes).
template <int P, bool SHIFT>
__global__ __launch_bounds__(256) void residual_mfma_kernel(
    const LeafDesc *__restrict__ leafd, int nleaf, const double *__restrict__ coef,
    const double *__restrict__ uc, const double *__restrict__ g, double sigma,
    double *__restrict__ r1, double *__restrict__ flux, const double *__restrict__ Dh_g,
    const double *__restrict__ Dh2_g, const double *__restrict__ Lloc_g, int q, int nrhs) {
  static_assert(P >= 4 && P <= 16, "one 16 x 16 tile per grid");
  constexpr int PP = P * P, PI = P - 2, MI = PI * PI;
  __shared__ double Us[4][16][17], Wx[4][16][17], Wy[4][16][17];
  __shared__ double Gs[4][MI];
  __shared__ double Ll[16 * P];
  const int leaf = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int64_t nl = nleaf;
  const LeafDesc &d = leafd[leaf];
  const double sx = d.sx, sy = d.sy;
  double fD[4], fD2[4];
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int kc = 4 * kk + lk;
    const bool in = li < P && kc < P;
    fD[kk] = in ? Dh_g[li * P + kc] : 0.0;
    fD2[kk] = in ? Dh2_g[li * P + kc] : 0.0;
  }
  // coefficients at this lane's result entries, folded with the scalings
  double a0[4], a1[4], a2[4], a3[4], a4[4], a5[4];
  const double *cl = coef + int64_t(leaf) * 6 * PP;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = lk + 4 * v;
    const bool in = row < P && li < P;
    const int t = in ? row * P + li : 0;
    a0[v] = in ? -cl[t] * sx * sx : 0.0;
    a1[v] = in ? -2.0 * cl[PP + t] * sx * sy : 0.0;
    a2[v] = in ? -cl[2 * PP + t] * sy * sy : 0.0;
    a3[v] = in ? cl[3 * PP + t] * sx : 0.0;
    a4[v] = in ? cl[4 * PP + t] * sy : 0.0;
    a5[v] = in ? cl[5 * PP + t] : 0.0;
  }
  for (int i = lane; i < 16 * 17; i += 64) (&Us[w][0][0])[i] = 0.0;   // the padding stays 0
  if (!SHIFT)
    for (int i = tid; i < q * P; i += 256) Ll[i] = Lloc_g[i];
  __syncthreads();
  const int r = int(blockIdx.y) * 4 + w;
  if (r < nrhs) {
    const int64_t lr = int64_t(r) * nl + leaf;
    const double *u = uc + lr * PP;
    for (int t = lane; t < PP; t += 64) Us[w][t / P][t % P] = u[t];
    if (!SHIFT)
      for (int t = lane; t < MI; t += 64) Gs[w][t] = g[lr * MI + t];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double uA[4], uB[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      uA[kk] = Us[w][li][4 * kk + lk];
      uB[kk] = Us[w][4 * kk + lk][li];
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
    // the interior residual, staged in Gs (each entry read, then rewritten,
    // by the one lane that owns it)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = lk + 4 * v, col = li;
      if (row >= 1 && row <= PI && col >= 1 && col <= PI) {
        const double Au = a0[v] * uxx[v] + a1[v] * uxy[v] + a2[v] * uyy[v] + a3[v] * ux[v] +
                          a4[v] * uy[v] + a5[v] * uB[v];
        const int a = (row - 1) * PI + (col - 1);
        if constexpr (SHIFT) Gs[w][a] = sigma * uB[v] - Au;
        else Gs[w][a] = Gs[w][a] - Au;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int t = lane; t < MI; t += 64) r1[lr * MI + t] = Gs[w][t];
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
        flux[lr * 4 * q + k] = v;
      }
    }
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
  dim3 grid(nleaf, (nrhs + 3) / 4);
  switch (p) {
#define HPS_RES_CASE(PV)                                                                       \
    case PV:                                                                                   \
      hipLaunchKernelGGL((residual_mfma_kernel<PV, SHIFT>), grid, dim3(256), 0, st, leafd,     \
                         nleaf, coef, uc, g, sigma, r1, flux, Dh, Dh2, Lloc, q, nrhs);         \
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
