// Register-resident Gauss-Jordan cores shared by the leaf and interface
// inversion kernels (device templates only).
#pragma once
#include "kernel_util.hpp"

namespace hps {

// ---------------------------------------------------------------------------
// Register-resident Gauss-Jordan inversion
// ---------------------------------------------------------------------------
// Threads per workgroup of the register-resident kernels: TR*TC rounded up to
// whole wavefronts, so every wavefront has all lanes active.  The extra
// threads repeat the first threads' rows and columns: they compute the same
// values and store the same values to the same places.
template <int TR, int TC>
constexpr int gj_threads() { return (TR * TC + 63) / 64 * 64; }

template <int TR, int TC, int RA, int CB>
__device__ __forceinline__ void gj_owner(int tid, int &tr, int &tc) {
  const int t = tid < TR * TC ? tid : tid - TR * TC;
  tr = t % TR;
  tc = t / TR;
}

template <int TR, int TC, int RA, int CB>
struct GJShared {
  double colbuf[2][TR * RA];
  double rowbuf[TC * CB];
  double sig[TR * RA];              // 1 / pivot of step k
  unsigned cand[2][2];
  int pivrow[TR * RA];
  int stepof[TR * RA];
  int info;
};

// Pivot candidate of column ctc + TC*slot among the unused rows, held by the TR
// threads with tc == ctc (a contiguous run of TR threads that spans one or two
// wavefronts).  Each of those wavefronts reduces its lanes and lane 0 stores
// the result in slot 0 (first wavefront of the run) or 1.  Padding rows are
// marked used in umask from the start.  The keys of one thread's rows differ
// from pivot_key(x, tr + TR*i) by the common offset tr in the row field, which
// is subtracted after the thread's own maximum is taken.
template <int TR, int TC, int RA, int CB>
__device__ __forceinline__ void gj_candidate(const double (&a)[RA][CB], const unsigned umask,
                                             const int ctc, const int slot, const int tr,
                                             const int tc, GJShared<TR, TC, RA, CB> &sh,
                                             const int par) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int lo = ctc * TR, hi = lo + TR - 1;          // owner thread range
  const int wlo = lo >> 6, whi = hi >> 6;
  if (wid < wlo || wid > whi) return;                 // uniform per wavefront
  unsigned key = 0;
  if (tc == ctc) {
#pragma unroll
    for (int i = 0; i < RA; ++i) {
      double x = 0.0;
#pragma unroll
      for (int b = 0; b < CB; ++b) if (b == slot) x = a[i][b];
      const unsigned k2 = ((umask >> i) & 1u) ? 0u : pivot_key(x, TR * i);   // bits >= 16 hold tc
      key = k2 > key ? k2 : key;
    }
    if (key) key -= unsigned(tr);
  }
  key = wave_max_u32(key);
  if (lane == 0) {
    sh.cand[par][wid == wlo ? 0 : 1] = key;
    if (wlo == whi) sh.cand[par][1] = 0;
  }
}

// In-place Gauss-Jordan sweeps with implicit partial pivoting.  Thread
// (tr, tc) owns rows tr + TR*i and columns tc + TC*b.
//
// Step k = TC*kb + kk eliminates column k, which sits in register slot kb of
// the threads with tc == kk.  The outer loop over kb is unrolled so that the
// slot is a compile-time constant.  Rows and columns >= n of the padded block
// start at 0 and stay 0 (each update multiplies by a zero row or column
// entry), so no bounds tests are needed.
//
// Pivot rows are kept unscaled: if sig_r = 1 / pivot of the step that chose
// row r, the swept matrix M of the textbook algorithm has
//   M[r][j] = sig_r * (a[r][j] + [j == k_r])
// where k_r is that step.  This is consistent because a sweep is homogeneous
// in each row (a row and its entry in the pivot column scale together), a
// pivot row needs no update in its own step (its pivot-column entry is
// published as 0), and the entry (r, k_r) never feeds another entry, so its
// unit value of the textbook algorithm can be added at the end.  On exit
// M[r_k][k'] = inv[k][r_k'] where r_k is the pivot row of step k.
template <int TR, int TC, int RA, int CB>
__device__ __forceinline__ void gj_core(double (&a)[RA][CB], const int n,
                                        const int tr, const int tc,
                                        GJShared<TR, TC, RA, CB> &sh) {
  const int tid = threadIdx.x;
  // bits 0..RA-1: used rows among my RA rows; bits 16..: tc (one register for
  // both keeps the step loop within 128 VGPRs)
  unsigned umask = unsigned(tc) << 16;
#pragma unroll
  for (int i = 0; i < RA; ++i)
    if (tr + TR * i >= n) umask |= 1u << i;
  if (tid == 0) sh.info = 0;
  if (tc == 0) {
#pragma unroll
    for (int i = 0; i < RA; ++i) sh.colbuf[0][tr + TR * i] = a[i][0];
  }
  gj_candidate<TR, TC, RA, CB>(a, umask, 0, 0, tr, tc, sh, 0);
  __syncthreads();
#pragma unroll
  for (int kb = 0; kb < CB; ++kb) {
    const int kend = min(TC, n - kb * TC);
    for (int kk = 0; kk < kend; ++kk) {
      const int k = kb * TC + kk;
      const int par = k & 1;
      double *cb = sh.colbuf[par];
      const unsigned k0 = sh.cand[par][0], k1c = sh.cand[par][1];
      const int r = __builtin_amdgcn_readfirstlane(key_row(k0 > k1c ? k0 : k1c));
      const int ir = __builtin_amdgcn_readfirstlane(r / TR);
      const bool rown = (tr == r - ir * TR);
      // publish the pivot row; its own entry of the pivot column becomes 0
#pragma unroll
      for (int i = 0; i < RA; ++i)
        if (i == ir && rown) {
#pragma unroll
          for (int b = 0; b < CB; ++b) sh.rowbuf[int(umask >> 16) + TC * b] = a[i][b];
        }
      if (rown) umask |= 1u << ir;
      if (tid == 0) {
        sh.pivrow[k] = r;
        sh.stepof[r] = k;
        cb[r] = 0.0;
      }
      __syncthreads();
      const double piv = sh.rowbuf[k];
      const bool ok = (piv != 0.0) && isfinite(piv);
      const double ip = ok ? 1.0 / piv : 0.0;
      if (tid == 0) {
        sh.sig[k] = ip;
        if (!ok && sh.info == 0) sh.info = isfinite(piv) ? (k + 1) : -(k + 1);
      }
      double s[CB];
#pragma unroll
      for (int b = 0; b < CB; ++b) s[b] = sh.rowbuf[int(umask >> 16) + TC * b] * ip;
#pragma unroll
      for (int i = 0; i < RA; ++i) {
        const double f = cb[tr + TR * i];
#pragma unroll
        for (int b = 0; b < CB; ++b) a[i][b] = fma(-f, s[b], a[i][b]);
      }
      if (int(umask >> 16) == kk) {
#pragma unroll
        for (int i = 0; i < RA; ++i) a[i][kb] = -cb[tr + TR * i] * ip;
      }
      if (kk + 1 < kend) {
        if (int(umask >> 16) == kk + 1) {
#pragma unroll
          for (int i = 0; i < RA; ++i) sh.colbuf[par ^ 1][tr + TR * i] = a[i][kb];
        }
        gj_candidate<TR, TC, RA, CB>(a, umask, kk + 1, kb, tr, int(umask >> 16), sh, par ^ 1);
      } else if (kb + 1 < CB && k + 1 < n) {
        if (int(umask >> 16) == 0) {
#pragma unroll
          for (int i = 0; i < RA; ++i) {
            double x = 0.0;
#pragma unroll
            for (int b = 0; b < CB; ++b) if (b == kb + 1) x = a[i][b];
            sh.colbuf[par ^ 1][tr + TR * i] = x;
          }
        }
        gj_candidate<TR, TC, RA, CB>(a, umask, 0, kb + 1, tr, int(umask >> 16), sh, par ^ 1);
      }
      __syncthreads();
    }
  }
}

// X[k][r_k'] = M[r_k][k'] with M from the unscaled sweep (see gj_core).
template <int TR, int TC, int RA, int CB>
__device__ __forceinline__ void gj_store(const double (&a)[RA][CB], const int n,
                                         const int tr, const int tc,
                                         const GJShared<TR, TC, RA, CB> &sh,
                                         double *X, const int ldx) {
#pragma unroll
  for (int i = 0; i < RA; ++i) {
    const int row = tr + TR * i;
    if (row >= n) continue;
    const int kr = sh.stepof[row];
    const double sg = sh.sig[kr];
    const int64_t orow = kr;
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      const int col = tc + TC * b;
      if (col < n)
        X[orow + int64_t(sh.pivrow[col]) * ldx] = sg * (a[i][b] + (col == kr ? 1.0 : 0.0));
    }
  }
}

// Leaf: A_ci,ci and A_ci,ce of
//   A = -C11 Dx^2 - 2 C12 Dx Dy - C22 Dy^2 + C1 Dx + C2 Dy + C   (Sec. 3.2)
// from the nodal coefficients and the reference matrix Dh (p x p, row-major)
// and its square Dh2.

// ---------------------------------------------------------------------------
// Column-owner Gauss-Jordan (flag-synchronised, no barrier per step)
// ---------------------------------------------------------------------------
// NW wavefronts; lane l owns rows l + 64 i (i < RA) and wavefront w owns
// columns w + NW b (b < CB), so a whole column lives in one wavefront.  Step
// k = NW b + w eliminates column k, held in slot b of wavefront w; the loop
// over b is unrolled so that slot is a compile-time constant.  The owner of
// column k has searched its pivot with a wavefront reduction and published
// the column (pivot row entry set to 0), the pivot row index and the pivot
// value in LDS; every wavefront reads its part of the pivot row from its own
// registers (readlane of lane r mod 64) and applies the rank-1 update, the
// owner of column k + 1 updating and publishing that column before its
// others.  There is no barrier per step: published steps live in a ring of D
// LDS slots, a wavefront starts step k once the counter `ready` has reached
// k, and the owner of column k + 1 reuses the slot of step k + 1 - D once
// every wavefront's `done` counter shows it has read that step.  Each step
// waits only on steps before it, so the waits always end; each is bounded
// all the same.  Pivot rows stay unscaled as in gj_core.
template <int NW, int RA>
struct GJ2Shared {
  static constexpr int D = 4;   // published steps held at once (a ring)
  double fbuf[D][64 * RA];   // published pivot column (pivot row entry 0)
  double piv[D];
  int rsel[D];
  double sig[64 * RA];       // 1 / pivot of step k
  int pivrow[64 * RA];
  int stepof[64 * RA];
  int info;
  int ready;                 // last published step
  int done[NW];              // last step each wavefront has finished with
  int abort;                 // a wait ran out (never in a correct run)
};


// 1 / x by the hardware reciprocal refined with two Newton steps
// (r <- r + r (1 - x r)), within an ulp or two of the division; x must be
// finite and nonzero.
__device__ __forceinline__ double recip_f64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane(int(unsigned(b)), l);
  const unsigned hi = __builtin_amdgcn_readlane(int(unsigned(b >> 32)), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Owner wavefront of column k (in its slot `slot`, a compile-time constant
// after unrolling): pivot search over the unused rows, then publish column,
// pivot row and pivot value for step k.
template <int NW, int RA, int CB>
__device__ __forceinline__ void gj2_publish(const double (&a)[RA][CB], unsigned umask, int slot,
                                            int k, int lane, GJ2Shared<NW, RA> &sh) {
  double x[RA];
#pragma unroll
  for (int i = 0; i < RA; ++i) {
    x[i] = 0.0;
#pragma unroll
    for (int c = 0; c < CB; ++c) if (c == slot) x[i] = a[i][c];
  }
  unsigned key = 0;
#pragma unroll
  for (int i = 0; i < RA; ++i) {
    const unsigned k2 = ((umask >> i) & 1u) ? 0u : pivot_key(x[i], 64 * i);
    key = k2 > key ? k2 : key;
  }
  if (key) key -= unsigned(lane);
  const unsigned wmax = wave_max_u32(key);
  const int r = __builtin_amdgcn_readfirstlane(key_row(wmax));
  const int ir = r >> 6, rl = r & 63;
  const int par = k % GJ2Shared<NW, RA>::D;
  double pv = 0.0;
#pragma unroll
  for (int i = 0; i < RA; ++i) {
    sh.fbuf[par][lane + 64 * i] = (lane + 64 * i == r) ? 0.0 : x[i];
    if (i == ir) pv = readlane_f64(x[i], rl);
  }
  if (lane == 0) {
    sh.piv[par] = pv;
    sh.rsel[par] = r;
    sh.pivrow[k] = r;
    sh.stepof[r] = k;
    const bool ok = (pv != 0.0) && isfinite(pv);
    sh.sig[k] = ok ? recip_f64(pv) : 0.0;
    if (!ok && sh.info == 0) sh.info = isfinite(pv) ? (k + 1) : -(k + 1);
    // the wavefront's LDS writes above are performed in order, so a reader
    // that sees ready >= k also sees step k's column, row and pivot
    __hip_atomic_store(&sh.ready, k, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

// Bounded waits of the flag-synchronised sweep: each spins (with s_sleep)
// until its condition holds, and gives up after 2^20 polls, setting abort so
// that every later wait returns at once and the kernel ends (the result is
// then reported as failed through info).
template <int NW, int RA>
__device__ __forceinline__ void gj2_giveup(GJ2Shared<NW, RA> &sh) {
  __hip_atomic_store(&sh.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <int NW, int RA>
__device__ __forceinline__ void gj2_wait_ready(GJ2Shared<NW, RA> &sh, int k) {
  for (unsigned spins = 0;; ++spins) {
    const int v = __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(&sh.ready, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
    if (v >= k) return;
    if (__builtin_amdgcn_readfirstlane(
            __hip_atomic_load(&sh.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)))
      return;
    if (spins >= (1u << 20)) { gj2_giveup(sh); return; }
    __builtin_amdgcn_s_sleep(1);
  }
}

// every wavefront has read step k (so its ring slot may be reused)
template <int NW, int RA>
__device__ __forceinline__ void gj2_wait_done(GJ2Shared<NW, RA> &sh, int k) {
  for (unsigned spins = 0;; ++spins) {
    int m = __hip_atomic_load(&sh.done[0], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
    for (int w = 1; w < NW; ++w)
      m = min(m, __hip_atomic_load(&sh.done[w], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
    if (__builtin_amdgcn_readfirstlane(m) >= k) return;
    if (__builtin_amdgcn_readfirstlane(
            __hip_atomic_load(&sh.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)))
      return;
    if (spins >= (1u << 20)) { gj2_giveup(sh); return; }
    __builtin_amdgcn_s_sleep(1);
  }
}

// Pivot-row entries of every slot except SKIP and SKIP + 1 (already used).
template <int RA, int CB, int SKIP>
__device__ __forceinline__ void gj2_pivot_row(const double (&a)[RA][CB], int ir, int rl,
                                              double (&s)[CB]) {
#pragma unroll
  for (int b = 0; b < CB; ++b) s[b] = 0.0;
#pragma unroll
  for (int i = 0; i < RA; ++i)
    if (i == ir) {
#pragma unroll
      for (int b = 0; b < CB; ++b)
        if (b != SKIP && b != SKIP + 1) s[b] = readlane_f64(a[i][b], rl);
    }
}

// Steps k = NW B + kk (kk < NW) for register slot B, then the next slot
// (template recursion keeps every slot index a compile-time constant).
template <int NW, int RA, int CB, int B>
__device__ __forceinline__ void gj2_slots(double (&a)[RA][CB], const int n, const int lane,
                                          const int wid, unsigned &umask, GJ2Shared<NW, RA> &sh) {
  if constexpr (B < CB) {
    constexpr int D = GJ2Shared<NW, RA>::D;
    const int kend = min(NW, n - B * NW);
    for (int kk = 0; kk < kend; ++kk) {
      const int k = B * NW + kk, par = k % D;
      gj2_wait_ready(sh, k);
      const int r = __builtin_amdgcn_readfirstlane(sh.rsel[par]);
      const double piv = sh.piv[par];
      const bool ok = (piv != 0.0) && isfinite(piv);
      const double ip = ok ? recip_f64(piv) : 0.0;
      const int ir = r >> 6, rl = r & 63;
      if (lane == rl) umask |= 1u << ir;
      double f[RA];
#pragma unroll
      for (int i = 0; i < RA; ++i) f[i] = sh.fbuf[par][lane + 64 * i] * ip;
      // step k read (the wavefront's LDS accesses are performed in order)
      if (lane == 0)
        __hip_atomic_store(&sh.done[wid], k, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
      // slots B and B + 1 first (column k + 1 is in one of them), with only
      // their pivot-row entries read, so the owner of column k + 1 reaches
      // its publication early; then the other pivot-row entries and slots
      double sB = 0.0, sB1 = 0.0;
#pragma unroll
      for (int i = 0; i < RA; ++i)
        if (i == ir) {
          sB = readlane_f64(a[i][B], rl);
          if constexpr (B + 1 < CB) sB1 = readlane_f64(a[i][B + 1], rl);
        }
#pragma unroll
      for (int i = 0; i < RA; ++i) a[i][B] = fma(-f[i], sB, a[i][B]);
      if constexpr (B + 1 < CB) {
#pragma unroll
        for (int i = 0; i < RA; ++i) a[i][B + 1] = fma(-f[i], sB1, a[i][B + 1]);
      }
      if (wid == kk) {
#pragma unroll
        for (int i = 0; i < RA; ++i) a[i][B] = -f[i];
      }
      // the owner of column k + 1 publishes step k + 1 once every wavefront
      // has read step k + 1 - D, whose ring slot it reuses
      if (kk + 1 < kend) {
        if (wid == kk + 1) {
          gj2_wait_done(sh, k + 1 - D);
          gj2_publish<NW, RA, CB>(a, umask, B, k + 1, lane, sh);
        }
      } else if (B + 1 < CB && k + 1 < n) {
        if (wid == 0) {
          gj2_wait_done(sh, k + 1 - D);
          gj2_publish<NW, RA, CB>(a, umask, B + 1 < CB ? B + 1 : B, k + 1, lane, sh);
        }
      }
      double s[CB];
      gj2_pivot_row<RA, CB, B>(a, ir, rl, s);
#pragma unroll
      for (int i = 0; i < RA; ++i)
#pragma unroll
        for (int c = 0; c < CB; ++c)
          if (c != B && c != B + 1) a[i][c] = fma(-f[i], s[c], a[i][c]);
    }
    gj2_slots<NW, RA, CB, B + 1>(a, n, lane, wid, umask, sh);
  }
}

template <int NW, int RA, int CB>
__device__ __forceinline__ void gj2_core(double (&a)[RA][CB], const int n, const int lane,
                                         const int wid, GJ2Shared<NW, RA> &sh) {
  unsigned umask = 0u;                    // used (or padding) rows among my RA rows
#pragma unroll
  for (int i = 0; i < RA; ++i)
    if (lane + 64 * i >= n) umask |= 1u << i;
  if (threadIdx.x == 0) {
    sh.info = 0;
    sh.ready = -1;
    sh.abort = 0;
  }
  if (threadIdx.x < NW) sh.done[threadIdx.x] = -1;
  __syncthreads();
  if (wid == 0) gj2_publish<NW, RA, CB>(a, umask, 0, 0, lane, sh);
  gj2_slots<NW, RA, CB, 0>(a, n, lane, wid, umask, sh);
  __syncthreads();
  if (threadIdx.x == 0 && sh.abort) sh.info = kGjSyncTimeout;
  __syncthreads();
}

// Leaf kernel on the column-owner core (same outputs as gj_leaf_kernel).

}  // namespace hps
