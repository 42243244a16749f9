// Solve-stage applies on the matrix cores (16 or more right-hand sides).
#include "kernel_util.hpp"

namespace hps {

template <typename TA, typename TC_, bool TRANS>
void launch_apply_valu_t(const ApplyDesc *descs, const int32_t *tmap, int64_t ntiles,
                         const Bases &bs, int nrhs, hipStream_t st);

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
      launch_apply_valu_t<double, double, true>(descs, tmap, ntiles, bs, nrhs, st);
    else
      launch_apply_valu_t<float, float, true>(descs, tmap, ntiles, bs, nrhs, st);
  } else {
    if (prec == 0)
      launch_apply_valu_t<double, double, false>(descs, tmap, ntiles, bs, nrhs, st);
    else
      launch_apply_valu_t<float, float, false>(descs, tmap, ntiles, bs, nrhs, st);
  }
  return hipGetLastError();
}


}  // namespace hps
