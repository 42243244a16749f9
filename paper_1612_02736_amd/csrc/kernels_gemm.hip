// Grouped FP64 GEMM on the matrix cores (the leaf and merge products of
// Algorithm 1).
#include "kernel_util.hpp"

namespace hps {

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
  const int msplit = d.msplit;
  // rows from msplit on come from the second A source, if any
  const bool a2 = msplit > 0 && row0 + ar >= msplit;
  const double *Ap = a2 ? (const double *)bs.d[d.A2.buf] + d.A2.off + (row0 + ar - msplit)
                        : A + (row0 + ar);
  const int lda_r = a2 ? d.A2.ld : lda;
  double *C = (double *)bs.d[d.C.buf] + d.C.off;
  const double *D = d.D.buf >= 0 ? (const double *)bs.d[d.D.buf] + d.D.off : nullptr;
  const double *D2 = msplit > 0 && d.D2.buf >= 0 ? (const double *)bs.d[d.D2.buf] + d.D2.off
                                                 : nullptr;
  const int32_t *crow = d.crow >= 0 ? bs.imap + d.crow : nullptr;
  const int32_t *ccol = d.ccol >= 0 ? bs.imap + d.ccol : nullptr;
  // f64 16x16x4 result layout: lane l, register v holds row (l >> 4) + 4 v,
  // column l & 15
  auto out_row = [&](int i, int v) { return wr0 + i * 16 + (lane >> 4) + 4 * v; };
  auto out_col = [&](int j) { return wc0 + j * 16 + (lane & 15); };
  // beta D(row, col), block-diagonal with msplit > 0
  auto dval = [&](int row, int col) -> double {
    if (msplit == 0) return D ? d.beta * D[row + int64_t(col) * d.D.ld] : 0.0;
    if (row < msplit && col < msplit) return D ? d.beta * D[row + int64_t(col) * d.D.ld] : 0.0;
    if (row >= msplit && col >= msplit && D2)
      return d.beta * D2[(row - msplit) + int64_t(col - msplit) * d.D2.ld];
    return 0.0;
  };
  // Small tiles (one or two MFMA tiles per wavefront, mostly short-K merge
  // products): the epilogue's D values and output maps are loaded now, so
  // their latency overlaps the operand fetch instead of following the MFMAs.
  constexpr bool PRE = NI * NJ <= 2;
  double dpre[PRE ? NI : 1][PRE ? NJ : 1][4];
  int64_t crp[PRE ? NI : 1][4], ccp[PRE ? NJ : 1];
  if constexpr (PRE) {
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = out_row(i, v);
        crp[i][v] = row < M ? (crow ? crow[row] : row) : 0;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const int col = out_col(j);
          dpre[i][j][v] = (row < M && col < N) ? dval(row, col) : 0.0;
        }
      }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int col = out_col(j);
      ccp[j] = col < N ? (ccol ? ccol[col] : col) : 0;
    }
  }
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
      ra[s] = (arow_ok && gk < K) ? Ap[int64_t(gk) * lda_r] : 0.0;
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
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = out_row(i, v), col = out_col(j);
        if (row < M && col < N) {
          double val = d.alpha * acc[i][j][v];
          int64_t cr, cc;
          if constexpr (PRE) {
            val += dpre[i][j][v];
            cr = crp[i][v];
            cc = ccp[j];
          } else {
            val += dval(row, col);
            cr = crow ? crow[row] : row;
            cc = ccol ? ccol[col] : col;
          }
          C[cr + cc * d.C.ld] = val;
        }
      }
}


// Tile variants (TM x TN per workgroup, K chunk): 0: 64 x 64, 1: 128 x 64,
// 2: 64 x 128, 3: 128 x 128, 4: 32 x 32, 5: 64 x 32, 6: 32 x 64 (K chunks
// of 16), 7: 64 x 64 with K chunks of 8 (half the LDS of variant 0, so more
// workgroups per CU).  Every variant accumulates each output over k in the
// same order (k-steps of 4, ascending), so all give bitwise the same result.
static const int kVarTM[8] = {64, 128, 64, 128, 32, 64, 32, 64};
static const int kVarTN[8] = {64, 64, 128, 128, 32, 32, 64, 64};
int gemm_variant_tm(int v) { return kVarTM[v]; }
int gemm_variant_tn(int v) { return kVarTN[v]; }

hipError_t launch_gemm(int variant, const GemmDesc *descs, const int32_t *tmap, int64_t ntiles,
                       const Bases &bs, hipStream_t st) {
  if (ntiles <= 0) return hipSuccess;
  const dim3 grid(unsigned((ntiles + 7) / 8 * 8));
  switch (variant) {
    case 0:
      hipLaunchKernelGGL((gemm_f64_kernel<64, 64, 16, 1>), grid, dim3(256), 0, st, descs, tmap,
                         ntiles, bs);
      break;
    case 1:
      hipLaunchKernelGGL((gemm_f64_kernel<128, 64, 16, 1>), grid, dim3(256), 0, st, descs, tmap,
                         ntiles, bs);
      break;
    case 2:
      hipLaunchKernelGGL((gemm_f64_kernel<64, 128, 16, 1>), grid, dim3(256), 0, st, descs, tmap,
                         ntiles, bs);
      break;
    case 3:
      hipLaunchKernelGGL((gemm_f64_kernel<128, 128, 16, 1>), grid, dim3(256), 0, st, descs, tmap,
                         ntiles, bs);
      break;
    case 4:
      hipLaunchKernelGGL((gemm_f64_kernel<32, 32, 16, 1>), grid, dim3(256), 0, st, descs, tmap,
                         ntiles, bs);
      break;
    case 5:
      hipLaunchKernelGGL((gemm_f64_kernel<64, 32, 16, 1>), grid, dim3(256), 0, st, descs, tmap,
                         ntiles, bs);
      break;
    case 6:
      hipLaunchKernelGGL((gemm_f64_kernel<32, 64, 16, 1>), grid, dim3(256), 0, st, descs, tmap,
                         ntiles, bs);
      break;
    case 7:
      hipLaunchKernelGGL((gemm_f64_kernel<64, 64, 8, 1>), grid, dim3(256), 0, st, descs, tmap,
                         ntiles, bs);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}


}  // namespace hps
