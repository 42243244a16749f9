// HIP kernels of the HPS build and solve stages (gfx950 / CDNA4).
//
// * gj_leaf / gj_merge: in-place Gauss-Jordan inversion with partial
//   pivoting of one matrix per workgroup, the matrix held in registers in a
//   2-D block-cyclic layout.  Builds F = A_ci,ci^-1 (Sec. 3.3, eq. alpine1)
//   and X = (T33a - T33b)^-1 (Sec. 4).  Every wavefront searches the pivot
//   column redundantly from LDS, so one barrier publishes the column and one
//   publishes the pivot row per elimination step.
// * gj_panel / gj_colperm: blocked Gauss-Jordan for interface blocks too
//   large for registers; the rank-NB update between panels is a GEMM.
// * gemm_f64: grouped FP64 GEMM on MFMA 16x16x4 tiles for the leaf products
//   (S, H, T of Algorithm 1) and the merge products (S = X R, T update).
// * apply: grouped matrix-times-vectors of the solve stage (Algorithm 2),
//   gathered right-hand sides, scattered results, split-K with a fixed
//   reduction order (results are bitwise reproducible).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kernels.hpp"
#include "types.hpp"

namespace hps {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));


// Tiles handed out so that the blocks one XCD receives (block b runs on XCD
// b % 8) form a contiguous run of logical tiles: neighbouring tiles share
// operands through that XCD's L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nblk) {
  const int64_t per = nblk >> 3;
  return (b & 7) * per + (b >> 3);
}

// Pivot search keys (32 bits): the high word of |x| (non-negative, so its bit
// pattern orders like the value) with its low 12 bits replaced by 4095 - row.
// The largest key is an |x| within a factor 1 - 2^-8 of the largest (the
// 11 exponent bits and 8 leading mantissa bits are compared) and, among
// those, the lowest row: threshold partial pivoting with threshold 1 - 2^-8.
// Rows that are not candidates carry key 0.  NaN and infinite entries exceed
// every finite key, so a non-finite pivot is found and reported.
__device__ __forceinline__ unsigned pivot_key(double x, int row) {
  const unsigned hi = unsigned((unsigned long long)__double_as_longlong(x) >> 32) & 0x7FFFFFFFu;
  return (hi & ~0xFFFu) | unsigned(4095 - row);
}
__device__ __forceinline__ int key_row(unsigned k) { return 4095 - int(k & 0xFFFu); }

template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned dpp_max_u32(unsigned v) {
  const unsigned o = unsigned(__builtin_amdgcn_update_dpp(0, int(v), CTRL, ROWS, 0xF, false));
  return o > v ? o : v;
}

// Maximum of a 32-bit key over the 64 lanes, returned wave-uniform: DPP
// butterflies inside each 16-lane row, then row_bcast:15 and row_bcast:31 fold
// the rows into lane 63.
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  v = dpp_max_u32<0xB1, 0xF>(v);     // quad_perm [1,0,3,2]
  v = dpp_max_u32<0x4E, 0xF>(v);     // quad_perm [2,3,0,1]
  v = dpp_max_u32<0x141, 0xF>(v);    // row_half_mirror
  v = dpp_max_u32<0x140, 0xF>(v);    // row_mirror
  v = dpp_max_u32<0x142, 0xA>(v);    // row_bcast:15 into rows 1 and 3
  v = dpp_max_u32<0x143, 0xC>(v);    // row_bcast:31 into rows 2 and 3
  return unsigned(__builtin_amdgcn_readlane(int(v), 63));
}

// ---------------------------------------------------------------------------
// Grouped FP64 GEMM (MFMA)
// ---------------------------------------------------------------------------
// TM x TN output tile per workgroup (4 wavefronts in 2 x 2, each TM/2 x TN/2
// = TM/32 x TN/32 MFMA tiles), K in chunks of BK through two LDS buffers: the
// next chunk is fetched into registers and stored into the other buffer
// while the MFMAs run on the current one, one barrier per chunk.  A
// wavefront whose part of the tile lies wholly outside M x N and the k-steps
// past K in the last chunk skip their MFMAs (scalar branches).  OCC is the
// minimum number of wavefronts per SIMD the register allocation must allow.
template <int TM, int TN, int BK, int OCC>
__global__ __launch_bounds__(256, OCC) void gemm_f64_kernel(
    const GemmDesc *__restrict__ descs, const int32_t *__restrict__ tmap,
    int64_t ntiles, Bases bs) {
  constexpr int NI = TM / 32, NJ = TN / 32;      // MFMA tiles per wavefront
  constexpr int AKS = 256 / TM, NA = BK * TM / 256;
  constexpr int BCS = 256 / BK, NBV = BK * TN / 256;
  __shared__ double As[2][BK][TM + 1];
  __shared__ double Bs[2][BK][TN + 1];
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= ntiles) return;
  const GemmDesc &d = descs[tmap[tile]];
  const int64_t t = tile - d.tile0;
  const int row0 = int(t / d.tn) * TM, col0 = int(t % d.tn) * TN;
  const int M = d.M, N = d.N, K = d.K;
  const double *A = (const double *)bs.d[d.A.buf] + d.A.off;
  const double *B = (const double *)bs.d[d.B.buf] + d.B.off;
  const int lda = d.A.ld, ldb = d.B.ld;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wid & 1, wn = wid >> 1;
  const int wr0 = row0 + wm * (TM / 2), wc0 = col0 + wn * (TN / 2);
  const bool wave_on = wr0 < M && wc0 < N;        // my part meets the matrix
  // per-thread load coordinates
  const int ar = tid % TM, ak = tid / TM;         // A: row ar, k = ak + AKS s
  const int bk = tid % BK, bc = tid / BK;         // B: k = bk, cols bc + BCS s
  const bool arow_ok = row0 + ar < M;
  const double *Ap = A + (row0 + ar);
  dbl4 acc[NI][NJ];
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  double ra[NA], rb[NBV];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int s = 0; s < NA; ++s) {
      const int gk = k0 + ak + AKS * s;
      ra[s] = (arow_ok && gk < K) ? Ap[int64_t(gk) * lda] : 0.0;
    }
    const int gk = k0 + bk;
#pragma unroll
    for (int s = 0; s < NBV; ++s) {
      const int gc = col0 + bc + BCS * s;
      rb[s] = (gk < K && gc < N) ? B[gk + int64_t(gc) * ldb] : 0.0;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int s = 0; s < NA; ++s) As[buf][ak + AKS * s][ar] = ra[s];
#pragma unroll
    for (int s = 0; s < NBV; ++s) Bs[buf][bk][bc + BCS * s] = rb[s];
  };
  if (K > 0) {
    fetch(0);
    stash(0);
  }
  __syncthreads();
  const int li = lane & 15;
  int buf = 0;
  for (int k0 = 0; k0 < K; k0 += BK) {
    const bool more = k0 + BK < K;
    if (more) fetch(k0 + BK);
    const int klen = min(BK, K - k0);
    if (wave_on) {
      // k-step operands: the next step's are read from LDS while this
      // step's MFMAs run (two register sets; the asm statement keeps the
      // compiler from hoisting further reads)
      double av[2][NI], bv[2][NJ];
#define HPS_GEMM_RD(KK, SET)                                                             \
  {                                                                                      \
    const int ka = (KK) + (lane >> 4);                                                   \
    _Pragma("unroll") for (int i = 0; i < NI; ++i)                                       \
        av[SET][i] = As[buf][ka][wm * (TM / 2) + i * 16 + li];                           \
    _Pragma("unroll") for (int j = 0; j < NJ; ++j)                                       \
        bv[SET][j] = Bs[buf][ka][wn * (TN / 2) + j * 16 + li];                           \
  }
#define HPS_GEMM_MM(SET)                                                                 \
  _Pragma("unroll") for (int i = 0; i < NI; ++i)                                         \
      _Pragma("unroll") for (int j = 0; j < NJ; ++j) acc[i][j] =                         \
          __builtin_amdgcn_mfma_f64_16x16x4f64(av[SET][i], bv[SET][j], acc[i][j], 0, 0, 0);
      if (klen == BK) {           // whole chunk: no branches between k-steps
        HPS_GEMM_RD(0, 0)
#pragma unroll
        for (int st = 0; st < BK / 4; ++st) {
          if (st + 1 < BK / 4) HPS_GEMM_RD(4 * (st + 1), (st + 1) & 1)
          HPS_GEMM_MM(st & 1)
          asm volatile("" ::: "memory");
        }
      } else {
#pragma unroll
        for (int st = 0; st < BK / 4; ++st)
          if (4 * st < klen) {
            HPS_GEMM_RD(4 * st, 0)
            HPS_GEMM_MM(0)
          }
      }
#undef HPS_GEMM_RD
#undef HPS_GEMM_MM
    }
    // the other buffer was last read in the previous chunk, before the
    // barrier that ended it
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  double *C = (double *)bs.d[d.C.buf] + d.C.off;
  const double *D = d.D.buf >= 0 ? (const double *)bs.d[d.D.buf] + d.D.off : nullptr;
  const int32_t *crow = d.crow >= 0 ? bs.imap + d.crow : nullptr;
  const int32_t *ccol = d.ccol >= 0 ? bs.imap + d.ccol : nullptr;
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // f64 16x16x4 result layout: lane l, register v holds row (l >> 4) + 4 v,
        // column l & 15
        const int row = wr0 + i * 16 + (lane >> 4) + 4 * v;
        const int col = wc0 + j * 16 + (lane & 15);
        if (row < M && col < N) {
          double val = d.alpha * acc[i][j][v];
          if (D) val += d.beta * D[row + int64_t(col) * d.D.ld];
          const int64_t cr = crow ? crow[row] : row;
          const int64_t cc = ccol ? ccol[col] : col;
          C[cr + cc * d.C.ld] = val;
        }
      }
}

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
  double a[RA][CB];
#pragma unroll
  for (int i = 0; i < RA; ++i) {
    const int row = lane + 64 * i;
#pragma unroll
    for (int b = 0; b < CB; ++b) {
      const int col = wid + NW * b;
      a[i][b] = (row < MI && col < MI) ? entry(grid_of(row), grid_of(col)) : 0.0;
    }
  }
  gj2_core<NW, RA, CB>(a, MI, lane, wid, sh);
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

// stepof = -1 before the first panel
__global__ __launch_bounds__(256) void gj_ginit_kernel(const MergeInvDesc *__restrict__ descs,
                                                       int nd, int32_t *__restrict__ g_all) {
  const MergeInvDesc &d = descs[blockIdx.y];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.m; i += gridDim.x * blockDim.x)
    g_all[d.ipiv + d.m + i] = -1;
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
      X[e] = Y[pivrow[row] + int64_t(stepof[col]) * n];
    }
  }
}

// ---------------------------------------------------------------------------
// Solve-stage applies
// ---------------------------------------------------------------------------
// Element (k, r) of a vector operand: RHS-major (stride >= 0) at
// off + idx + r * stride, or RHS-interleaved (stride < 0) at (off + idx) * nrhs + r.
__device__ __forceinline__ double *vaddr(const Bases &bs, const VRef &v, int64_t k, int r,
                                         int nrhs) {
  const int64_t idx = v.off + (v.map >= 0 ? bs.imap[v.map + k] : k);
  double *b = (double *)bs.d[v.buf];
  return v.stride >= 0 ? b + idx + r * v.stride : b + idx * nrhs + r;
}

__device__ __forceinline__ double vload(const Bases &bs, const VRef &v, int64_t k, int r,
                                        int nrhs) {
  return *vaddr(bs, v, k, r, nrhs);
}

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

// A vector operand resolved once per workgroup: element (k, r) is
// b[map[k] * kmul + r * rstep], where b already includes the operand's offset
// (interleaved: kmul = nrhs, rstep = 1; RHS-major: kmul = 1, rstep = stride)
// and an unmapped operand reads the identity map.
struct VSrc {
  const double *b;
  const int32_t *map;
  int32_t kmul, rstep;
};
__device__ __forceinline__ VSrc vsrc(const Bases &bs, const VRef &v, int nrhs) {
  VSrc s;
  const bool il = v.stride < 0;
  s.b = v.buf >= 0 ? (const double *)bs.d[v.buf] + (il ? v.off * nrhs : v.off) : nullptr;
  s.map = v.map >= 0 ? bs.imap + v.map : bs.iota;
  s.kmul = il ? nrhs : 1;
  s.rstep = il ? 1 : int32_t(v.stride);
  return s;
}


// Right operand entries (kc + kk, r0 + r) of one k chunk into registers:
// entry j of thread tid is (kk, r) = (tid % KC, tid / KC + (256 / KC) j) when
// kfast, else (tid / NR + (256 / NR) j, tid % NR).  The gather indices of
// the tile's k range are in LDS (ixs, read once per tile), so a chunk costs
// one memory round trip.  Entries past the chunk or past nrhs read a valid
// element and are zeroed.
template <int NR, int KC>
__device__ __forceinline__ void stage_regs(double (&breg)[KC * NR / 256], int mode, int K1,
                                           const VSrc &s1, const VSrc &s2, const VSrc &s3,
                                           const int (*ixs)[512], int k0, int kc, int kn,
                                           int r0, int nrhs, int tid, bool kfast) {
  constexpr int NB = KC * NR / 256;
  const int kk0 = kfast ? tid % KC : tid / NR, r00 = kfast ? tid / KC : tid % NR;
  int kx[NB], rx[NB];
  bool ok[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int kk = kfast ? kk0 : kk0 + (256 / NR) * j;
    const int r = kfast ? r00 + (256 / KC) * j : r00;
    ok[j] = kk < kn && r0 + r < nrhs;
    kx[j] = ok[j] ? kc + kk : kc;
    rx[j] = ok[j] ? r0 + r : r0;
  }
  if (mode == 0) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const bool in2 = kx[j] >= K1;
      const double *b = in2 ? s2.b : s1.b;
      const int64_t o = int64_t(ixs[0][kx[j] - k0]) * (in2 ? s2.kmul : s1.kmul) +
                        int64_t(rx[j]) * (in2 ? s2.rstep : s1.rstep);
      breg[j] = b[o];
    }
  } else {
    const bool has3 = mode == 1 && s3.b;
    double va[NB], vb[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      va[j] = s1.b[int64_t(ixs[0][kx[j] - k0]) * s1.kmul + int64_t(rx[j]) * s1.rstep];
      vb[j] = s2.b[int64_t(ixs[1][kx[j] - k0]) * s2.kmul + int64_t(rx[j]) * s2.rstep];
    }
    if (has3) {
      double vc[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j)
        vc[j] = s3.b[int64_t(ixs[2][kx[j] - k0]) * s3.kmul + int64_t(rx[j]) * s3.rstep];
#pragma unroll
      for (int j = 0; j < NB; ++j) breg[j] = va[j] - vb[j] + vc[j];
    } else if (mode == 2) {
#pragma unroll
      for (int j = 0; j < NB; ++j) breg[j] = va[j] + vb[j];
    } else {
#pragma unroll
      for (int j = 0; j < NB; ++j) breg[j] = va[j] - vb[j];
    }
  }
#pragma unroll
  for (int j = 0; j < NB; ++j)
    if (!ok[j]) breg[j] = 0.0;
}

// Matrix-core apply for 16 or more right-hand sides, FP64 or FP32 operators:
// the same tiles (64 operator rows x one k-slice) as apply_kernel, with the
// 64 rows split over the four wavefronts (16 each) and 16 x 16 x 4 MFMA
// steps over k, so no cross-wavefront reduction is needed.  NT16 =
// right-hand-side tiles of 16 per workgroup.  Operand layouts (both
// precisions): lane l holds A(l % 16, l / 16) and B(l / 16, l % 16); result
// register v of lane l is C((l >> 4) + 4 v, l & 15) for f64 and
// C(4 (l >> 4) + v, l & 15) for f32.  FP32 operators accumulate in FP32 and
// the result is widened to FP64 when stored.
//
// Software pipeline over k chunks of KC: the operator entries and the right
// operand of chunk c + 1 are loaded into registers while chunk c runs on the
// matrix cores; the right operand goes through a double-buffered LDS tile, so
// one barrier per chunk suffices.  The right operand is read along its
// contiguous direction (k for RHS-major arrays, right-hand sides otherwise).
template <typename T> struct MfmaT;
template <> struct MfmaT<double> {
  typedef dbl4 acc_t;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <> struct MfmaT<float> {
  typedef flt4 acc_t;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

template <typename TA, int NT16, bool TRANS>
__global__ __launch_bounds__(256) void apply_mfma_kernel(
    const ApplyDesc *__restrict__ descs, const int32_t *__restrict__ tmap,
    int64_t ntiles, Bases bs, int nrhs) {
  typedef MfmaT<TA> M;
  constexpr int NR = 16 * NT16;
  // k per chunk: 32 for FP64 operators (four wavefronts per SIMD fit in the
  // register file, so more workgroups keep operator loads in flight), 64 for
  // FP32
  constexpr int KC = sizeof(TA) == 8 ? 32 : 64;
  constexpr int NB = KC * NR / 256;          // right-operand entries per thread
  __shared__ TA Bsh[2][KC][NR + 1];
  __shared__ int ixs[3][512];               // gather indices of the tile's k range
  const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= ntiles) return;
  const ApplyDesc &d = descs[tmap[tile]];
  const int64_t t = tile - d.tile0;
  const int rbi = int(t % d.rb), slice = int(t / d.rb);
  const int K = d.K1 + (d.mode == 0 ? d.K2 : 0);
  const int kper = (K + d.ksl - 1) / d.ksl;
  const int k0 = slice * kper, k1 = min(K, k0 + kper);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int r0 = blockIdx.y * NR;
  const TA *A = (const TA *)bs.d[d.abuf] + d.aoff;
  const int lda = d.lda;
  const int arow = rbi * 64 + wid * 16 + (lane & 15);   // operand row of this lane
  const bool arow_ok = arow < d.M;
  // a wavefront whose 16 rows all lie past M only helps stage the right operand
  const bool wave_on = rbi * 64 + __builtin_amdgcn_readfirstlane(wid) * 16 < d.M;
  const int kl = lane >> 4;
  typename M::acc_t acc[NT16];
#pragma unroll
  for (int u = 0; u < NT16; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = TA(0);
  TA abuf[KC / 4];
  double breg[NB];
  const int mode = d.mode, K1 = d.K1;
  const VSrc s1 = vsrc(bs, d.B1, nrhs), s2 = vsrc(bs, d.B2, nrhs), s3 = vsrc(bs, d.B3, nrhs);
  for (int k = k0 + tid; k < k1; k += 256) {
    if (mode == 0) {
      ixs[0][k - k0] = k < K1 ? s1.map[k] : s2.map[k - K1];
    } else {
      ixs[0][k - k0] = s1.map[k];
      ixs[1][k - k0] = s2.map[k];
      if (s3.b) ixs[2][k - k0] = s3.map[k];
    }
  }
  __syncthreads();
  // operator entries of chunk kc: abuf[j] = A(arow, kc + 4 j + kl)
#define HPS_LOAD_CHUNK(KCV, KF)                                                             \
  {                                                                                         \
    const int kn_ = min(KC, k1 - (KCV));                                                    \
    _Pragma("unroll") for (int j = 0; j < KC / 4; ++j) {                                    \
      const int kk = 4 * j + kl;                                                            \
      abuf[j] = (arow_ok && kk < kn_)                                                       \
                    ? (TRANS ? A[int64_t(arow) * lda + (KCV) + kk]                          \
                             : A[arow + int64_t((KCV) + kk) * lda])                         \
                    : TA(0);                                                                \
    }                                                                                       \
    const int kmid = (KCV) + min(kn_ - 1, KC / 2);                                          \
    KF = ((mode == 0 && kmid >= K1) ? s2.kmul : s1.kmul) == 1;                              \
    stage_regs<NR, KC>(breg, mode, K1, s1, s2, s3, ixs, k0, (KCV), kn_, r0, nrhs, tid, KF); \
  }
  bool kfast = false;
  if (k0 < k1) HPS_LOAD_CHUNK(k0, kfast);
  int buf = 0;
  for (int kc = k0; kc < k1; kc += KC) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int kk = kfast ? tid % KC : tid / NR + (256 / NR) * j;
      const int r = kfast ? tid / KC + (256 / KC) * j : tid % NR;
      Bsh[buf][kk][r] = TA(breg[j]);
    }
    TA acur[KC / 4];
#pragma unroll
    for (int j = 0; j < KC / 4; ++j) acur[j] = abuf[j];
    __syncthreads();
    if (kc + KC < k1) HPS_LOAD_CHUNK(kc + KC, kfast);
    if (wave_on) {
#pragma unroll
      for (int j = 0; j < KC / 4; ++j) {
        const int kk = 4 * j + kl;
#pragma unroll
        for (int u = 0; u < NT16; ++u)
          acc[u] = M::mma(acur[j], Bsh[buf][kk][16 * u + (lane & 15)], acc[u]);
      }
    }
    buf ^= 1;
  }
#undef HPS_LOAD_CHUNK
  if (d.ksl == 1 && d.C.stride < 0) {
    // interleaved result: the MFMA layout (lanes along right-hand sides) is
    // already contiguous
#pragma unroll
    for (int u = 0; u < NT16; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = rbi * 64 + wid * 16 + M::row(lane, v);
        const int rg = r0 + 16 * u + (lane & 15);
        if (row >= d.M || rg >= nrhs) continue;
        double val = d.alpha * double(acc[u][v]);
        if (d.D.buf >= 0) val += d.beta * vload(bs, d.D, row, rg, nrhs);
        *vaddr(bs, d.C, row, rg, nrhs) = val;
      }
    return;
  }
  // RHS-major result or split-K partials: transpose through LDS so that
  // lanes run along rows, in the 2 KC >= 64 rows of both right-operand
  // buffers (free after the barrier)
  static_assert(2 * KC >= 64, "transpose needs 64 rows");
  TA (*tr)[NR + 1] = reinterpret_cast<TA (*)[NR + 1]>(&Bsh[0][0][0]);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NT16; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      tr[wid * 16 + M::row(lane, v)][16 * u + (lane & 15)] = acc[u][v];
  __syncthreads();
  const int row = rbi * 64 + lane;
  if (row >= d.M) return;
#pragma unroll
  for (int j = 0; j < NR / 4; ++j) {
    const int r = wid + 4 * j, rg = r0 + r;
    if (rg >= nrhs) continue;
    const double sv = double(tr[lane][r]);
    if (d.ksl == 1) {
      double val = d.alpha * sv;
      if (d.D.buf >= 0) val += d.beta * vload(bs, d.D, row, rg, nrhs);
      *vaddr(bs, d.C, row, rg, nrhs) = val;
    } else {
      ((double *)bs.d[BUF_SCR])[d.part * nrhs + (int64_t(slice) * nrhs + rg) * d.M + row] = sv;
    }
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

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned grid_1d(int64_t n, int64_t cap = 65536) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return unsigned(b);
}

hipError_t launch_gemm(const GemmDesc *descs, const int32_t *tmap, int64_t ntiles,
                       const Bases &bs, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  const int64_t nblk = (ntiles + 7) / 8 * 8;
  hipLaunchKernelGGL((gemm_f64_kernel<64, 64, 16, 1>), dim3(unsigned(nblk)), dim3(256), 0, st,
                     descs, tmap, ntiles, bs);
  return hipGetLastError();
}

hipError_t launch_gj_leaf(int p, const LeafDesc *descs, int nleaf, const Bases &bs,
                          const double *Dh, const double *Dh2, const int32_t *ice,
                          int me, int32_t *info, hipStream_t st) {
  if (nleaf <= 0) return hipSuccess;
  switch (p) {
    case 16:
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

template <typename TA, typename TC_, bool TRANS>
static void launch_apply_t(const ApplyDesc *descs, const int32_t *tmap,
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

hipError_t launch_apply(int prec, const ApplyDesc *descs, const int32_t *tmap,
                        int64_t ntiles, const Bases &bs, int nrhs, hipStream_t st, bool trans) {
  if (ntiles <= 0) return hipSuccess;
  if (nrhs >= 16) {
    const int64_t nblk = (ntiles + 7) / 8 * 8;
    const bool two = nrhs > 16;
    const unsigned gy = unsigned((nrhs + (two ? 31 : 15)) / (two ? 32 : 16));
#define HPS_APPLY_MFMA(TA, NT, TR)                                                           \
  hipLaunchKernelGGL((apply_mfma_kernel<TA, NT, TR>), dim3(unsigned(nblk), gy), dim3(256), 0, \
                     st, descs, tmap, ntiles, bs, nrhs)
    if (prec == 0) {
      if (two) {
        if (trans) HPS_APPLY_MFMA(double, 2, true); else HPS_APPLY_MFMA(double, 2, false);
      } else {
        if (trans) HPS_APPLY_MFMA(double, 1, true); else HPS_APPLY_MFMA(double, 1, false);
      }
    } else {
      if (two) {
        if (trans) HPS_APPLY_MFMA(float, 2, true); else HPS_APPLY_MFMA(float, 2, false);
      } else {
        if (trans) HPS_APPLY_MFMA(float, 1, true); else HPS_APPLY_MFMA(float, 1, false);
      }
    }
#undef HPS_APPLY_MFMA
    return hipGetLastError();
  }
  if (trans) {
    if (prec == 0)
      launch_apply_t<double, double, true>(descs, tmap, ntiles, bs, nrhs, st);
    else
      launch_apply_t<float, float, true>(descs, tmap, ntiles, bs, nrhs, st);
  } else {
    if (prec == 0)
      launch_apply_t<double, double, false>(descs, tmap, ntiles, bs, nrhs, st);
    else
      launch_apply_t<float, float, false>(descs, tmap, ntiles, bs, nrhs, st);
  }
  return hipGetLastError();
}

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
