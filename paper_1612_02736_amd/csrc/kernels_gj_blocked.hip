// Blocked Gauss-Jordan inversion of large interface blocks (m > 196) of the
// merges (Sec. 4).
#include "gj_core.hpp"

namespace hps {

// ---------------------------------------------------------------------------
// Blocked Gauss-Jordan for large interface blocks
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void zdiff_kernel(const MergeInvDesc *__restrict__ descs,
                                                    int nd, Bases bs) {
  const MergeInvDesc &d = descs[blockIdx.y];
  const int n = d.m;
  const double *Ta = (const double *)bs.d[BUF_WS] + d.Ta;
  const double *Tb = (const double *)bs.d[BUF_WS] + d.Tb;
  double *X = (double *)bs.d[BUF_WS] + d.X;
  const int64_t tot = int64_t(n) * n;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t col = e / n, row = e - col * n;
    X[e] = Ta[row + col * d.lda] - Tb[row + col * d.ldb];
  }
}

// Blocked Gauss-Jordan with implicit partial pivoting (no row interchanges),
// one launch per panel of NB columns.  The panel sweep is the textbook one
// restricted to the panel's columns: the pivot row of column k is the unused
// row of largest magnitude.  If R is the set of a panel's pivot rows and L the
// product of its elementary sweep matrices, L differs from I only in the
// columns R and the swept panel column c holds L(:, r_c); every other column
// B therefore becomes L B = (B with rows R set to 0) + P W, with P the swept
// panel columns and W(c, :) = B(r_c, :).  After the last panel the swept
// matrix M has M[r_k][k'] = inv[k][r_k'], which gj_perm_kernel turns into the
// inverse.  pivrow[k] = r_k and stepof[r] = the step that used row r (-1
// before) live in int scratch.
//
// Launch kb (kb < 0: the first) has one workgroup per strip of NB columns:
// every strip other than panel kb applies panel kb's update (the strip is
// held in registers, row t + NT i by thread t; the threads holding the rows R
// copy them to LDS as W), and the strip of the next panel then sweeps its
// columns in the same registers.  The sweep keeps pivot rows unscaled until
// the pivot row itself is written (one multiply per row and column step).  So the next panel's
// sweep follows its update without a launch in between, and only the
// columns of a strip are written by the strip's own workgroup.
//
// The sweep takes one barrier per column: every wavefront's best candidate
// row travels to LDS with its key, so after the barrier all threads read the
// pivot row from the winning wavefront's slot.
template <int NB, int RPT, int NT>
__global__ __launch_bounds__(NT) void gj_step_kernel(
    const MergeInvDesc *__restrict__ descs, int nd, int kb, Bases bs,
    int32_t *__restrict__ g_all, int32_t *__restrict__ info) {
  constexpr int NW = NT / 64;
  __shared__ unsigned wkey[2][NW];
  __shared__ double crow[2][NW][NB];
  __shared__ __align__(16) double Wsh[NB][NB];
  __shared__ int rsh[NB];
  const MergeInvDesc &d = descs[blockIdx.y];
  const int n = d.m;
  const int c0 = int(blockIdx.x) * NB;
  const int nxt = kb < 0 ? 0 : kb + NB;
  if (c0 >= n || kb >= n) return;             // kb >= n: this matrix is done
  if (kb >= 0 && c0 == kb) return;            // the swept panel itself
  const bool sweep = (c0 == nxt);
  if (kb < 0 && !sweep) return;
  const int ncv = min(NB, n - c0);
  double *A = (double *)bs.d[BUF_WS] + d.X;
  int32_t *pivrow = g_all + d.ipiv;
  int32_t *stepof = pivrow + n;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  double pan[RPT][NB];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int row = tid + NT * i;
#pragma unroll
    for (int c = 0; c < NB; ++c)
      pan[i][c] = (row < n && c < ncv) ? A[row + int64_t(c0 + c) * n] : 0.0;
  }
  if (kb >= 0) {
    // update by panel kb: pan <- (pan with rows R set to 0) + P W
    const int nbv = min(NB, n - kb);
    const double *P = A + int64_t(kb) * n;
    // my rows of the swept panel kb, loaded up front where registers allow
    constexpr bool PRE = RPT <= 2;
    double pr[PRE ? RPT : 1][NB];
    if constexpr (PRE) {
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int row = tid + NT * i;
#pragma unroll
        for (int c = 0; c < NB; ++c)
          pr[i][c] = (row < n && c < nbv) ? P[row + int64_t(c) * n] : 0.0;
      }
    }
    if (tid < NB) rsh[tid] = tid < nbv ? pivrow[kb + tid] : -1;
    for (int e = tid; e < NB * NB; e += NT)
      if (e / NB >= nbv) Wsh[e / NB][e % NB] = 0.0;
    __syncthreads();
    // W = the strip's rows R (old values), from the threads that hold them
    unsigned rmask = 0u;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int row = tid + NT * i;
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (rsh[c] == row) {
          rmask |= 1u << i;
#pragma unroll
          for (int j = 0; j < NB; ++j) Wsh[c][j] = pan[i][j];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < RPT; ++i)
      if ((rmask >> i) & 1u) {
#pragma unroll
        for (int j = 0; j < NB; ++j) pan[i][j] = 0.0;
      }
    if constexpr (PRE) {
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const double2 *wr = reinterpret_cast<const double2 *>(&Wsh[c][0]);
#pragma unroll
        for (int j2 = 0; j2 < NB / 2; ++j2) {
          const double2 w = wr[j2];
#pragma unroll
          for (int i = 0; i < RPT; ++i) {
            pan[i][2 * j2] = fma(pr[i][c], w.x, pan[i][2 * j2]);
            pan[i][2 * j2 + 1] = fma(pr[i][c], w.y, pan[i][2 * j2 + 1]);
          }
        }
        // one row of W in flight at a time (register pressure)
        asm volatile("" ::: "memory");
      }
    } else {
#pragma unroll 2
      for (int c = 0; c < nbv; ++c) {
        double pc[RPT];
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          const int row = tid + NT * i;
          pc[i] = row < n ? P[row + int64_t(c) * n] : 0.0;
        }
        const double2 *wr = reinterpret_cast<const double2 *>(&Wsh[c][0]);
#pragma unroll
        for (int j2 = 0; j2 < NB / 2; ++j2) {
          const double2 w = wr[j2];
#pragma unroll
          for (int i = 0; i < RPT; ++i) {
            pan[i][2 * j2] = fma(pc[i], w.x, pan[i][2 * j2]);
            pan[i][2 * j2 + 1] = fma(pc[i], w.y, pan[i][2 * j2 + 1]);
          }
        }
      }
    }
  }
  int first_bad = 0;
  if (sweep) {
    const int nbv = ncv;
    unsigned umask = 0u;          // rows already used as pivots (or padding)
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int row = tid + NT * i;
      if (row >= n || stepof[row] >= 0) umask |= 1u << i;
    }
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      if (c < nbv) {
        const int par = c & 1;
        unsigned key = 0;
        int bi = 0;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          const unsigned k2 = ((umask >> i) & 1u) ? 0u : pivot_key(pan[i][c], tid + NT * i);
          if (k2 > key) { key = k2; bi = i; }
        }
        const unsigned wmax = wave_max_u32(key);
        if (key == wmax && key != 0) {             // this wavefront's candidate row
#pragma unroll
          for (int i = 0; i < RPT; ++i)
            if (i == bi) {
#pragma unroll
              for (int cc = 0; cc < NB; ++cc) crow[par][wid][cc] = pan[i][cc];
            }
        }
        if (lane == 0) wkey[par][wid] = wmax;
        __syncthreads();
        unsigned best = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) best = max(best, wkey[par][w]);
        // row r is held by thread r mod NT, so its candidate slot is that
        // thread's wavefront
        const int r = __builtin_amdgcn_readfirstlane(key_row(best));
        const double *prow = crow[par][(r % NT) >> 6];
        if (tid == 0) {
          pivrow[c0 + c] = r;
          stepof[r] = c0 + c;
        }
        const double piv = prow[c];
        const bool ok = (piv != 0.0) && isfinite(piv);
        if (!ok && first_bad == 0) first_bad = isfinite(piv) ? (c0 + c + 1) : -(c0 + c + 1);
        const double ip = ok ? recip_f64(piv) : 0.0;
        double sr[NB];             // the pivot row, unscaled
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) sr[cc] = prow[cc];
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          const double f = pan[i][c] * ip;
#pragma unroll
          for (int cc = 0; cc < NB; ++cc)
            if (cc != c) pan[i][cc] = fma(-f, sr[cc], pan[i][cc]);
          pan[i][c] = -f;
          if (tid + NT * i == r) {                 // the pivot row itself
            umask |= 1u << i;
#pragma unroll
            for (int cc = 0; cc < NB; ++cc) pan[i][cc] = cc == c ? ip : sr[cc] * ip;
          }
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int row = tid + NT * i;
    if (row < n) {
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < ncv) A[row + int64_t(c0 + c) * n] = pan[i][c];
    }
  }
  if (sweep && tid == 0 && first_bad != 0 && info[d.info] == 0) info[d.info] = first_bad;
}

// stepof = -1 before the first panel; pivrow[k] = k (in range even if a
// failed build leaves a step without a pivot)
__global__ __launch_bounds__(256) void gj_ginit_kernel(const MergeInvDesc *__restrict__ descs,
                                                       int nd, int32_t *__restrict__ g_all) {
  const MergeInvDesc &d = descs[blockIdx.y];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.m; i += gridDim.x * blockDim.x) {
    g_all[d.ipiv + i] = i;
    g_all[d.ipiv + d.m + i] = -1;
  }
}

// Inverse from the swept matrix: X[i][j] = M[pivrow[i]][stepof[j]], through a
// scratch copy Y of M (first pass copies, second gathers).
__global__ __launch_bounds__(256) void gj_perm_kernel(const MergeInvDesc *__restrict__ descs,
                                                      int nd, Bases bs, int to_scratch,
                                                      const int32_t *__restrict__ g_all) {
  const MergeInvDesc &d = descs[blockIdx.y];
  const int n = d.m;
  double *X = (double *)bs.d[BUF_WS] + d.X;
  double *Y = (double *)bs.d[BUF_SCR] + d.W;   // scratch copy (n x n)
  const int32_t *pivrow = g_all + d.ipiv, *stepof = pivrow + n;
  const int64_t tot = int64_t(n) * n;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < tot;
       e += int64_t(gridDim.x) * blockDim.x) {
    if (to_scratch) {
      Y[e] = X[e];
    } else {
      const int64_t col = e / n, row = e - col * n;
      const int sc = stepof[col];              // < 0 only after a failed sweep
      X[e] = Y[pivrow[row] + int64_t(sc < 0 ? 0 : sc) * n];
    }
  }
}



hipError_t launch_zdiff(const MergeInvDesc *descs, int nd, int maxm, const Bases &bs,
                        hipStream_t st) {
  if (nd <= 0) return hipSuccess;
  hipLaunchKernelGGL(zdiff_kernel, dim3(grid_1d(int64_t(maxm) * maxm, 512), nd), dim3(256),
                     0, st, descs, nd, bs);
  return hipGetLastError();
}

int panel_nb(int maxm) { (void)maxm; return 16; }

// strips of NB columns per matrix, one workgroup each (kb < 0: first launch)
hipError_t launch_gj_panel(const MergeInvDesc *descs, int nd, int kb, int maxm,
                           const Bases &bs, int32_t *g, int32_t *info, hipStream_t st) {
  if (nd <= 0) return hipSuccess;
  constexpr int NB = 16;
  const dim3 grid(unsigned((maxm + NB - 1) / NB), unsigned(nd));
  if (maxm <= 256)
    hipLaunchKernelGGL((gj_step_kernel<NB, 1, 256>), grid, dim3(256), 0, st, descs, nd, kb, bs,
                       g, info);
  else if (maxm <= 512)
    hipLaunchKernelGGL((gj_step_kernel<NB, 1, 512>), grid, dim3(512), 0, st, descs, nd, kb, bs,
                       g, info);
  else if (maxm <= 1024)
    hipLaunchKernelGGL((gj_step_kernel<NB, 2, 512>), grid, dim3(512), 0, st, descs, nd, kb, bs,
                       g, info);
  else if (maxm <= 2048)
    hipLaunchKernelGGL((gj_step_kernel<NB, 4, 512>), grid, dim3(512), 0, st, descs, nd, kb, bs,
                       g, info);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_gj_ginit(const MergeInvDesc *descs, int nd, int maxm, int32_t *g,
                           hipStream_t st) {
  if (nd <= 0) return hipSuccess;
  hipLaunchKernelGGL(gj_ginit_kernel, dim3(grid_1d(maxm, 64), nd), dim3(256), 0, st, descs, nd, g);
  return hipGetLastError();
}

hipError_t launch_gj_colperm(const MergeInvDesc *descs, int nd, int maxm, const Bases &bs,
                             int32_t *g, int32_t *unused, hipStream_t st) {
  (void)unused;
  if (nd <= 0) return hipSuccess;
  hipLaunchKernelGGL(gj_perm_kernel, dim3(grid_1d(int64_t(maxm) * maxm, 512), nd),
                     dim3(256), 0, st, descs, nd, bs, 1, g);
  hipLaunchKernelGGL(gj_perm_kernel, dim3(grid_1d(int64_t(maxm) * maxm, 512), nd),
                     dim3(256), 0, st, descs, nd, bs, 0, g);
  return hipGetLastError();
}



}  // namespace hps
