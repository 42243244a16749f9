// Leaf interior inversion F = A_ci,ci^-1 for p = 16 (Sec. 3.3) as a blocked
// Gauss-Jordan whose panel updates run on the FP64 matrix cores.
//
// The matrix block held by one workgroup has 256 rows: the 196 collocation
// rows of A_ci,ci and, below them, the hrows <= 60 rows of D_ge,ci (the flux
// map of the interior grid), which are never pivots; the sweeps turn them into
// -D_ge,ci A_ci,ci^-1 = -H (Sec. 3.4).  Columns 0..191 form 12 strips of 16,
// one per wavefront, held in registers as 16 matrix-core accumulator tiles
// (register v of tile t holds, in lane l, row 16 t + 4 v + (l >> 4) and
// column 16 w + (l & 15) of strip w); columns 192..195 (the tail) live in LDS.
//
// Implicit partial pivoting as in the rank-1 kernels: the pivot of column k is
// the unused row with the largest pivot key, and rows are never exchanged.
// If a panel's sweeps use pivot rows R = {r_c} and leave its swept columns P
// (256 x 16), every other column block B becomes
//     (B with rows R set to 0) + P W,   W(c, :) = B(r_c, :) before the panel,
// because the product of the panel's elementary sweep matrices differs from I
// only in the columns R.  So a panel costs one sequential sweep of 16 columns
// by the wavefront that owns it, and one rank-16 product per other strip, as
// 16 x 16 x 4 MFMA steps with P and W^T read from LDS.
//
// Schedule (one barrier per panel): after the barrier that publishes panel q
// in LDS slot q & 1, the owner of strip q + 1 applies panel q to its strip
// first and sweeps it (writing panel q + 1 into the other slot) while the
// other wavefronts apply panel q to theirs; the owner of strip q, whose strip
// is panel q, applies it to the tail.  The tail's 4 columns are the last
// panel.  Pivot rows are left unscaled (row r_k carries the factor pivot_k,
// which the panel updates preserve since they are linear in the rows), so in
// the end the swept block M holds M(r_k, j) = pivot_k F(k, r_j) and
// M(196 + h, j) = -H(h, r_j).
#include "gj_core.hpp"

namespace hps {

namespace gjb {
constexpr int P = 16, PI = P - 2, MI = PI * PI;   // 196 interior nodes
constexpr int NR = 256;                           // rows: A_ci,ci then D_ge,ci
constexpr int NS = 12;                            // strips of 16 columns in registers
constexpr int NT = NS * 64;
constexpr int TC0 = 16 * NS, TCN = MI - TC0;      // tail columns 192..195
constexpr int S = 18;                             // row stride of a panel slot (doubles)
constexpr int WS = 18;                            // row stride of a W^T buffer
constexpr int NSLOT = 3;                          // published panels held at once (a ring)
static_assert(TCN == 4, "tail layout assumes 4 columns");

struct Shared {
  // swept panels (row-major, stride S); slot 1 first holds the coefficient
  // and reference tables
  __align__(16) double slot[NSLOT][NR * S];
  __align__(16) double wt[NS][16 * WS];      // per wavefront: W^T of the current panel
  double tail[NR * TCN];       // columns 192..195 (row-major)
  double wtail[8 * TCN];       // W of the tail (a half-panel)
  __align__(16) double wbuf[64];   // W of a half-panel sweep (8 x 8)
  int stepof[NR];              // step that used row r as its pivot (-1: none yet)
  int pivrow[MI];              // pivot row of step k
  double sig[MI];              // 1 / pivot of step k
  int info;
  int ready;                   // last published half-panel (2 q + h; the tail: 2 NS)
  int done[NS];                // last panel each wavefront has applied
  int tail_done;               // last panel applied to the tail
  int abort;                   // a wait ran out (never in a correct run)
};

// Pivot search, broadcast of the pivot row and update for step k0 + C of a
// sweep over NC columns held by one wavefront in row layout (lane l holds
// rows l + 64 i, i < 4).  Column C is a compile-time constant.  The pivot row
// reaches every lane through readlane of the owning lane (scalar operands of
// the update).  Bookkeeping stays in registers until the sweep ends: lane C
// keeps the pivot row and 1 / pivot of step C, and `bad` the first failed
// step (+-(k + 1), as info reports it).
template <int NC, int C>
__device__ __forceinline__ void sweep_step(double (&x)[4][NC], unsigned &umask, int k0, int lane,
                                           int &myr, double &mysig, int &bad) {
  unsigned key = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const unsigned k2 = ((umask >> i) & 1u) ? 0u : pivot_key(x[i][C], lane + 64 * i);
    key = k2 > key ? k2 : key;
  }
  const unsigned wmax = wave_max_u32(key);
  // some unused row below 196 always carries a nonzero key; the guard keeps
  // r a valid row index regardless
  const int r = __builtin_amdgcn_readfirstlane(wmax ? key_row(wmax) : 0);
  const int ir = r >> 6, rl = r & 63;
  double pr[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) pr[c] = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (i == ir) {
#pragma unroll
      for (int c = 0; c < NC; ++c) pr[c] = readlane_f64(x[i][c], rl);
    }
  const double piv = pr[C];
  const bool ok = (piv != 0.0) && isfinite(piv);
  const double ip = ok ? recip_f64(piv) : 0.0;
  // pivot rows stay unscaled: row r keeps its entries (multiplier 0) and gets
  // 1 in the pivot column; the factor 1 / pivot is applied when F is stored
  double f[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) f[i] = (lane + 64 * i) == r ? 0.0 : x[i][C] * ip;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if (c == C) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i][c] = fma(-f[i], pr[c], x[i][c]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const bool isr = (lane + 64 * i) == r;
    x[i][C] = isr ? 1.0 : -f[i];
    if (isr) umask |= 1u << i;
  }
  myr = lane == C ? r : myr;
  mysig = lane == C ? ip : mysig;
  if (!ok && bad == 0) bad = isfinite(piv) ? (k0 + C + 1) : -(k0 + C + 1);
}

// Per-lane LDS addresses (lane + 64 i rows of the tables and slots) cost one
// vector operation each, but the compiler hoists them out of the panel loop
// and, short of registers there, keeps them in scratch memory, so that every
// sweep waits for their reloads.  The lane index read afresh from the
// hardware at the start of a step (the count of lanes below this one, in an
// instruction the compiler may not move or merge) keeps them local to it,
// with nothing live across the loop.
__device__ __forceinline__ int lane_now() {
  int l;
  asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
  return l;
}

// Record steps k0 .. k0 + NC - 1 of a finished sweep in LDS.
template <int NC>
__device__ __forceinline__ void sweep_log(int k0, int lane, int myr, double mysig, int bad,
                                          Shared &sh) {
  lane = lane_now();
  if (lane < NC) {
    sh.stepof[myr] = k0 + lane;
    sh.pivrow[k0 + lane] = myr;
    sh.sig[k0 + lane] = mysig;
  }
  if (bad != 0 && lane == 0 && sh.info == 0) sh.info = bad;
  __builtin_amdgcn_wave_barrier();
}

// Bounded waits on the progress counters: each spins (with s_sleep) until its
// condition holds and gives up after 2^20 polls, setting abort so that every
// later wait returns at once and the kernel ends (the result is then
// reported as failed through info).  Every wait is on an earlier panel than
// the waiter's own next step, so the waits always end.
__device__ __forceinline__ bool aborted(Shared &sh) {
  return __builtin_amdgcn_readfirstlane(
             __hip_atomic_load(&sh.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) != 0;
}

__device__ __forceinline__ void wait_at_least(Shared &sh, int &flag, int v) {
  for (unsigned spins = 0;; ++spins) {
    const int f = __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(&flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
    if (f >= v || aborted(sh)) return;
    if (spins >= (1u << 20)) {
      __hip_atomic_store(&sh.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      return;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// every wavefront has applied panel v (so the slot of panel v may be reused)
__device__ __forceinline__ void wait_all_done(Shared &sh, int v) {
  for (unsigned spins = 0;; ++spins) {
    int m = __hip_atomic_load(&sh.done[0], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
    for (int w = 1; w < NS; ++w)
      m = min(m, __hip_atomic_load(&sh.done[w], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
    if (__builtin_amdgcn_readfirstlane(m) >= v || aborted(sh)) return;
    if (spins >= (1u << 20)) {
      __hip_atomic_store(&sh.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      return;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// a wavefront's LDS writes are performed in order, so a reader that sees the
// counter also sees what was written before it
__device__ __forceinline__ void post(int &flag, int v, int lane) {
  __builtin_amdgcn_wave_barrier();
  if (lane == 0) __hip_atomic_store(&flag, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ unsigned used_rows(int lane, const Shared &sh) {
  lane = lane_now();
  unsigned umask = 0u;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = lane + 64 * i;
    if (row >= MI || sh.stepof[row] >= 0) umask |= 1u << i;
  }
  return umask;
}

// Columns TO .. TO + 7 of a panel held in LDS slot sl, after the 8 sweeps
// of steps k0 .. k0 + 7 whose swept columns are FROM .. FROM + 7:
// (rows R zeroed) + P W, with W the old rows R (copied to wbuf first).
__device__ __forceinline__ void apply_half(double *sl, int from, int to, int k0, int lane,
                                           Shared &sh) {
  lane = lane_now();
  {
    const int k = lane >> 3, c = lane & 7;
    sh.wbuf[lane] = sl[sh.pivrow[k0 + k] * S + to + c];
  }
  __builtin_amdgcn_wave_barrier();
  double y[4][8];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = lane + 64 * i;
    const int s = sh.stepof[row] - k0;
    const bool piv = s >= 0 && s < 8;
    const double2 *src = reinterpret_cast<const double2 *>(sl + row * S + to);
#pragma unroll
    for (int c2 = 0; c2 < 4; ++c2) {
      const double2 u = src[c2];
      y[i][2 * c2] = piv ? 0.0 : u.x;
      y[i][2 * c2 + 1] = piv ? 0.0 : u.y;
    }
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const double2 *wk2 = reinterpret_cast<const double2 *>(sh.wbuf + 8 * k);
    const double2 w01 = wk2[0], w23 = wk2[1], w45 = wk2[2], w67 = wk2[3];
    const double wk[8] = {w01.x, w01.y, w23.x, w23.y, w45.x, w45.y, w67.x, w67.y};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double pk = sl[(lane + 64 * i) * S + from + k];
#pragma unroll
      for (int c = 0; c < 8; ++c) y[i][c] = fma(pk, wk[c], y[i][c]);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double2 *dst = reinterpret_cast<double2 *>(sl + (lane + 64 * i) * S + to);
#pragma unroll
    for (int c2 = 0; c2 < 4; ++c2) dst[c2] = make_double2(y[i][2 * c2], y[i][2 * c2 + 1]);
  }
  __builtin_amdgcn_wave_barrier();
}

// Sweep of 8 panel columns COL0 .. COL0 + 7 of slot sl in registers (steps
// k0 .. k0 + 7).
__device__ __forceinline__ void sweep_half(double *sl, int col0, int k0, int lane, Shared &sh) {
  lane = lane_now();
  double x[4][8];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double2 *src = reinterpret_cast<const double2 *>(sl + (lane + 64 * i) * S + col0);
#pragma unroll
    for (int c2 = 0; c2 < 4; ++c2) {
      const double2 u = src[c2];
      x[i][2 * c2] = u.x;
      x[i][2 * c2 + 1] = u.y;
    }
  }
  unsigned umask = used_rows(lane, sh);
  int myr = 0, bad = 0;
  double mysig = 0.0;
  sweep_step<8, 0>(x, umask, k0, lane, myr, mysig, bad);
  sweep_step<8, 1>(x, umask, k0, lane, myr, mysig, bad);
  sweep_step<8, 2>(x, umask, k0, lane, myr, mysig, bad);
  sweep_step<8, 3>(x, umask, k0, lane, myr, mysig, bad);
  sweep_step<8, 4>(x, umask, k0, lane, myr, mysig, bad);
  sweep_step<8, 5>(x, umask, k0, lane, myr, mysig, bad);
  sweep_step<8, 6>(x, umask, k0, lane, myr, mysig, bad);
  sweep_step<8, 7>(x, umask, k0, lane, myr, mysig, bad);
  sweep_log<8>(k0, lane, myr, mysig, bad, sh);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double2 *dst = reinterpret_cast<double2 *>(sl + (lane + 64 * i) * S + col0);
#pragma unroll
    for (int c2 = 0; c2 < 4; ++c2) dst[c2] = make_double2(x[i][2 * c2], x[i][2 * c2 + 1]);
  }
  __builtin_amdgcn_wave_barrier();
}

// Owner of strip q: sweep its 16 columns (steps 16 q .. 16 q + 15) as two
// half-panels of 8 (only 8 columns of 4 rows per lane in registers at a
// time).  The sweeps of the first half (L0) are applied to the second half
// before it is swept (the panel formula at half-panel size); those of the
// second half (L1) are not applied to the first: slot q & 1 and the
// registers are left holding [P0, P1], P0 the first half as L0 left it and
// P1 the second half after L1.  Every other column block then applies L0 and
// L1 in turn, and the owner applies L1 to P0 in the next round.
__device__ __forceinline__ void sweep_strip(dbl4 (&acc)[16], int q, int lane, Shared &sh) {
  lane = lane_now();
  double *sl = sh.slot[q % NSLOT];
  const int g = lane >> 4, n = lane & 15;
#pragma unroll
  for (int t = 0; t < 16; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) sl[(16 * t + 4 * v + g) * S + n] = acc[t][v];
  __builtin_amdgcn_wave_barrier();
  sweep_half(sl, 0, 16 * q, lane, sh);
  post(sh.ready, 2 * q, lane);           // P0 is final: the others may apply L0
  apply_half(sl, 0, 8, 16 * q, lane, sh);
  sweep_half(sl, 8, 16 * q + 8, lane, sh);
  post(sh.ready, 2 * q + 1, lane);
  const int lane2 = lane_now(), g2 = lane2 >> 4, n2 = lane2 & 15;
#pragma unroll
  for (int t = 0; t < 16; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[t][v] = sl[(16 * t + 4 * v + g2) * S + n2];
}

// Rows R of steps k0 .. k0 + K - 1 in this wavefront's strip: copy them to
// W^T and set them to 0 (LEFT: in columns 0..7 only, W^T zero in columns
// 8..15).  The registers that can hold a pivot row are those whose row index
// >> 2 matches some r_c >> 2 (a wave-uniform mask).
template <int K, bool LEFT = false>
__device__ __forceinline__ void gather_w(dbl4 (&acc)[16], int k0, int lane, double *wt,
                                         const Shared &sh) {
  lane = lane_now();
  const int g = lane >> 4, n = lane & 15;
  unsigned long long U = 0ull;
#pragma unroll
  for (int c = 0; c < K; ++c) {
    const int r = __builtin_amdgcn_readfirstlane(sh.pivrow[k0 + c]);
    U |= 1ull << (r >> 2);
  }
#pragma unroll
  for (int t = 0; t < 16; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if ((U >> (4 * t + v)) & 1ull) {
        // lanes whose row is not a pivot row of the panel write to a spare
        // column of W^T (never read)
        const int s = sh.stepof[16 * t + 4 * v + g] - k0;
        const bool pv = s >= 0 && s < K;
        const bool keep = !LEFT || n < 8;
        wt[n * WS + (pv ? s : 16)] = keep ? acc[t][v] : 0.0;
        acc[t][v] = (pv && keep) ? 0.0 : acc[t][v];
      }
  __builtin_amdgcn_wave_barrier();
}

// strip += P W for the 8 panel columns COL0 .. COL0 + 7 of slot sl, with
// W^T from gather_w.  The k index of MFMA step s for lane group kk = l >> 4
// is panel column COL0 + 2 kk + s, so both operands are 2 contiguous doubles
// per lane.  Two tiles at a time, their MFMA chains interleaved.
__device__ __forceinline__ void update_half(dbl4 (&acc)[16], const double *sl, int col0, int lane,
                                            const double *wt) {
  lane = lane_now();
  const int g = lane >> 4, n = lane & 15;
  const double2 b = *reinterpret_cast<const double2 *>(wt + n * WS + 2 * g);
#pragma unroll
  for (int t = 0; t < 16; t += 2) {
    const double2 a0 = *reinterpret_cast<const double2 *>(sl + (16 * t + n) * S + col0 + 2 * g);
    const double2 a1 =
        *reinterpret_cast<const double2 *>(sl + (16 * t + 16 + n) * S + col0 + 2 * g);
    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.x, b.x, acc[t], 0, 0, 0);
    acc[t + 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.x, b.x, acc[t + 1], 0, 0, 0);
    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0.y, b.y, acc[t], 0, 0, 0);
    acc[t + 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1.y, b.y, acc[t + 1], 0, 0, 0);
  }
}

// strip <- L1 (L0 strip) for panel q: each half-panel's rows R zeroed, then
// + P W, the second half gathering its W after the first half's update.
// The caller has waited for the first half (ready >= 2 q); the second half
// is applied once it is published.
__device__ __forceinline__ void update_strip16(dbl4 (&acc)[16], int q, int lane, double *wt,
                                               Shared &sh) {
  const double *sl = sh.slot[q % NSLOT];
  gather_w<8>(acc, 16 * q, lane, wt, sh);
  update_half(acc, sl, 0, lane, wt);
  wait_at_least(sh, sh.ready, 2 * q + 1);
  gather_w<8>(acc, 16 * q + 8, lane, wt, sh);
  update_half(acc, sl, 8, lane, wt);
}

// Owner of panel q, holding [P0, P1]: apply L1 to P0 (columns 0..7).
__device__ __forceinline__ void owner_fixup(dbl4 (&acc)[16], int q, int lane, double *wt,
                                            const Shared &sh) {
  gather_w<8, true>(acc, 16 * q + 8, lane, wt, sh);
  update_half(acc, sh.slot[q % NSLOT], 8, lane, wt);
}

// The last panel (tail columns, steps 192 .. 195, in slot 0): one MFMA step.
__device__ __forceinline__ void update_strip4(dbl4 (&acc)[16], int lane, double *wt,
                                              const Shared &sh) {
  lane = lane_now();
  const int g = lane >> 4, n = lane & 15;
  gather_w<TCN>(acc, TC0, lane, wt, sh);
  const double b = wt[n * WS + g];
  const double *sl = sh.slot[NS % NSLOT];
#pragma unroll
  for (int t = 0; t < 16; ++t)
    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(sl[(16 * t + n) * S + g], b, acc[t], 0, 0, 0);
}

// Tail <- L1 (L0 tail) for panel q, on the vector ALU by the wavefront that
// owns panel q (it has no strip update in that round).
__device__ __forceinline__ void update_tail(int q, int lane, Shared &sh) {
  lane = lane_now();
  const double *sl = sh.slot[q % NSLOT];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int k0 = 16 * q + 8 * h;
    if (lane < 8) {
      const int r = sh.pivrow[k0 + lane];
#pragma unroll
      for (int c = 0; c < TCN; ++c) sh.wtail[lane * TCN + c] = sh.tail[r * TCN + c];
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = lane + 64 * i;
      const int s = sh.stepof[row] - k0;
      const bool piv = s >= 0 && s < 8;
      double y[TCN];
#pragma unroll
      for (int c = 0; c < TCN; ++c) y[c] = piv ? 0.0 : sh.tail[row * TCN + c];
      const double2 *pr = reinterpret_cast<const double2 *>(sl + row * S + 8 * h);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) {
        const double2 pk = pr[k2];
#pragma unroll
        for (int c = 0; c < TCN; ++c) {
          y[c] = fma(pk.x, sh.wtail[(2 * k2) * TCN + c], y[c]);
          y[c] = fma(pk.y, sh.wtail[(2 * k2 + 1) * TCN + c], y[c]);
        }
      }
#pragma unroll
      for (int c = 0; c < TCN; ++c) sh.tail[row * TCN + c] = y[c];
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// Sweep of the tail (steps 192 .. 195), the last panel (index NS).
__device__ __forceinline__ void sweep_tail(int lane, Shared &sh) {
  lane = lane_now();
  double x[4][TCN];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < TCN; ++c) x[i][c] = sh.tail[(lane + 64 * i) * TCN + c];
  unsigned umask = used_rows(lane, sh);
  int myr = 0, bad = 0;
  double mysig = 0.0;
  sweep_step<TCN, 0>(x, umask, TC0, lane, myr, mysig, bad);
  sweep_step<TCN, 1>(x, umask, TC0, lane, myr, mysig, bad);
  sweep_step<TCN, 2>(x, umask, TC0, lane, myr, mysig, bad);
  sweep_step<TCN, 3>(x, umask, TC0, lane, myr, mysig, bad);
  sweep_log<TCN>(TC0, lane, myr, mysig, bad, sh);
  double *sl = sh.slot[NS % NSLOT];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int c = 0; c < TCN; ++c) sl[(lane + 64 * i) * S + c] = x[i][c];
}

}  // namespace gjb

__global__ __launch_bounds__(gjb::NT) void gjb_leaf_kernel(
    const LeafDesc *__restrict__ descs, int nleaf, Bases bs, const double *__restrict__ Dh_g,
    const double *__restrict__ Dh2_g, int32_t *__restrict__ info) {
  using namespace gjb;
  __shared__ Shared sh;
  const int leaf = blockIdx.x;
  if (leaf >= nleaf) return;
  const LeafDesc &d = descs[leaf];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, n = lane & 15;
  // coefficient and reference tables in slot 1 until the first sweep of it;
  // the rows of Dh and Dh2 are padded to DS doubles so that the lanes of one
  // assembly step, which read one column index jx in up to 16 different rows
  // ix, hit different LDS banks
  constexpr int DS = P + 1;
  static_assert(6 * P * P + 2 * P * DS <= NR * S, "tables must fit in one slot");
  double *cf = sh.slot[1], *Dh = cf + 6 * P * P, *Dh2 = Dh + P * DS;
  const double *coef = (const double *)bs.d[BUF_COEF] + d.coef;
  for (int i = tid; i < 6 * P * P; i += NT) cf[i] = coef[i];
  for (int i = tid; i < P * P; i += NT) {
    Dh[i + i / P] = Dh_g[i];
    Dh2[i + i / P] = Dh2_g[i];
  }
  for (int i = tid; i < NR; i += NT) sh.stepof[i] = -1;
  if (tid == 0) {
    sh.info = 0;
    sh.ready = -1;
    sh.tail_done = -1;
    sh.abort = 0;
  }
  if (tid < NS) sh.done[tid] = -1;
  __syncthreads();
  const double sx = d.sx, sy = d.sy;
  auto entry = [&](int ga, int gb) -> double {
    const int iy = ga / P, ix = ga - iy * P, jy = gb / P, jx = gb - jy * P;
    double v = -2.0 * cf[P * P + ga] * sx * sy * Dh[iy * DS + jy] * Dh[ix * DS + jx];
    if (iy == jy) v += -cf[ga] * sx * sx * Dh2[ix * DS + jx] + cf[3 * P * P + ga] * sx * Dh[ix * DS + jx];
    if (ix == jx)
      v += -cf[2 * P * P + ga] * sy * sy * Dh2[iy * DS + jy] + cf[4 * P * P + ga] * sy * Dh[iy * DS + jy];
    if (ga == gb) v += cf[5 * P * P + ga];
    return v;
  };
  auto grid_of = [](int a) { const int y = a / PI; return (y + 1) * P + (a - y * PI) + 1; };
  const int hrows = d.hrows;
  const double *Dci = (const double *)bs.d[BUF_WS] + d.Dci;
  auto init = [&](int row, int col) -> double {
    if (row < MI) return entry(grid_of(row), grid_of(col));
    if (row - MI < hrows) return Dci[(row - MI) + int64_t(col) * hrows];
    return 0.0;
  };
  const int col = 16 * w + n;
  // The strip's entries, 32 rows at a time, through an LDS stage of this
  // wavefront (slots 0 and 2 are free until the first sweep); its rows are
  // padded to SD doubles, since with 16 the 16 rows written by one pass of
  // lanes would all start in the same LDS bank.
  // Lane pair (2 rr, 2 rr + 1) computes row 32 tc + rr, columns 8 (lane & 1)
  // .. + 7 of the strip, with the row's coefficients loaded once: entry
  // (a, b) of A_ci,ci is cxy(a) Dh(iy, jy) Dh(ix, jx) + [iy = jy] (cxx(a)
  // Dh2(ix, jx) + cx(a) Dh(ix, jx)) + [ix = jx] (cyy(a) Dh2(iy, jy) + cy(a)
  // Dh(iy, jy)) + [a = b] c(a) (grid indices of interior nodes a and b).
  constexpr int SD = 17, SW = 32 * SD;
  static_assert(8 * SW <= NR * S && (NS - 8) * SW <= NR * S, "stages must fit in slots 0 and 2");
  double *stage = w < 8 ? &sh.slot[0][0] + SW * w : &sh.slot[2][0] + SW * (w - 8);
  dbl4 acc[16];
  {
    const int rr = lane >> 1, cb = 16 * w + 8 * (lane & 1);
    const int jy0 = cb / PI, jx0 = cb - jy0 * PI;     // interior coordinates of column cb
    double *srow = stage + rr * SD + 8 * (lane & 1);
#pragma unroll
    for (int tc = 0; tc < 8; ++tc) {
      const int row = 32 * tc + rr;
      if (row < MI) {
        const int iy = row / PI + 1, ix = row - (row / PI) * PI + 1, ga = iy * P + ix;
        const double cxy = -2.0 * cf[P * P + ga] * sx * sy, cxx = -cf[ga] * sx * sx,
                     cx = cf[3 * P * P + ga] * sx, cyy = -cf[2 * P * P + ga] * sy * sy,
                     cy = cf[4 * P * P + ga] * sy, c0 = cf[5 * P * P + ga];
        int jy = jy0 + 1, jx = jx0 + 1;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const double dy = Dh[iy * DS + jy], dx = Dh[ix * DS + jx];
          const double d2y = Dh2[iy * DS + jy], d2x = Dh2[ix * DS + jx];
          double v = cxy * dy * dx;
          v += iy == jy ? fma(cxx, d2x, cx * dx) : 0.0;
          v += ix == jx ? fma(cyy, d2y, cy * dy) : 0.0;
          v += row == cb + j ? c0 : 0.0;
          srow[j] = v;
          // next column: jx runs over 1 .. PI, then jy advances
          const bool wrap = jx == PI;
          jx = wrap ? 1 : jx + 1;
          jy = wrap ? jy + 1 : jy;
        }
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j)
          srow[j] = row - MI < hrows ? Dci[(row - MI) + int64_t(cb + j) * hrows] : 0.0;
      }
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc[2 * tc][v] = stage[(4 * v + g) * SD + n];
        acc[2 * tc + 1][v] = stage[(16 + 4 * v + g) * SD + n];
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
  for (int e = tid; e < NR * TCN; e += NT) sh.tail[e] = init(e / TCN, TC0 + e % TCN);
  __syncthreads();
  // No barrier from here on: panels are published through `ready` in a
  // ring of NSLOT slots, each wavefront applies them in order and counts
  // them in done[w], and the sweep of panel q reuses the slot of panel
  // q - NSLOT once every wavefront has applied that panel.
  double *wt = sh.wt[w];
  if (w == 0) {
    sweep_strip(acc, 0, lane, sh);
  }
  for (int q = 0; q < NS; ++q) {
    if (w == q) {
      // this wavefront's strip is panel q ([P0, P1]); the tail takes the
      // panels in order
      wait_at_least(sh, sh.tail_done, q - 1);
      update_tail(q, lane, sh);
      if (q == NS - 1) {
        wait_all_done(sh, NS - NSLOT);
        sweep_tail(lane, sh);
        post(sh.ready, 2 * NS, lane);
      }
      post(sh.tail_done, q, lane);
      // the strip is also in slot q % NSLOT until every wavefront has
      // applied panel q: reload it rather than keep it live above
      const double *sl = sh.slot[q % NSLOT];
#pragma unroll
      for (int t = 0; t < 16; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[t][v] = sl[(16 * t + 4 * v + g) * S + n];
      owner_fixup(acc, q, lane, wt, sh);
      post(sh.done[w], q, lane);
    } else {
      const bool owner = w == q + 1;
      wait_at_least(sh, sh.ready, 2 * q);
      if (owner) {
        __builtin_amdgcn_s_setprio(2);
      } else if (q + 1 < NS && ((w - q - 1) & 3) == 0) {
        // the other wavefronts on the owner's SIMD (wavefront w runs on
        // SIMD w mod 4) leave it alone until its sweep is published: FP64
        // matrix-core and FP64 vector work on one SIMD slow each other
        // down.  They catch up while the next sweep runs on another SIMD.
        wait_at_least(sh, sh.ready, 2 * q + 3);
      }
      update_strip16(acc, q, lane, wt, sh);
      post(sh.done[w], q, lane);
      if (owner) {
        // the tables in slot 1 are read only before the barrier above
        if (q + 1 >= NSLOT) wait_all_done(sh, q + 1 - NSLOT);
        sweep_strip(acc, q + 1, lane, sh);
        __builtin_amdgcn_s_setprio(0);
      }
    }
  }
  wait_at_least(sh, sh.ready, 2 * NS);   // the tail panel
  update_strip4(acc, lane, wt, sh);
  // F(k, r_j) = M(r_k, j); H(h, r_j) = -M(196 + h, j)
  double *F = (double *)bs.d[d.fbuf] + d.F;
  double *Hp = (double *)bs.d[BUF_WS] + d.H;
  const int64_t pc = sh.pivrow[col];
#pragma unroll
  for (int t = 0; t < 16; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * t + 4 * v + g;
      if (row < MI) {
        const int kr = sh.stepof[row];
        F[kr + pc * MI] = sh.sig[kr] * acc[t][v];
      }
      else if (row - MI < hrows) Hp[(row - MI) + pc * hrows] = -acc[t][v];
    }
  for (int e = tid; e < NR * TCN; e += NT) {
    const int row = e / TCN, c = e % TCN;
    const double val = sh.slot[NS % NSLOT][row * S + c];
    const int64_t pt = sh.pivrow[TC0 + c];
    if (row < MI) {
      const int kr = sh.stepof[row];
      F[kr + pt * MI] = sh.sig[kr] * val;
    }
    else if (row - MI < hrows) Hp[(row - MI) + pt * hrows] = -val;
  }
  if (tid == 0) info[d.info] = sh.abort ? kGjSyncTimeout : sh.info;
}

hipError_t launch_gjb_leaf(const LeafDesc *descs, int nleaf, const Bases &bs, const double *Dh,
                           const double *Dh2, int32_t *info, hipStream_t st) {
  if (nleaf <= 0) return hipSuccess;
  hipLaunchKernelGGL(gjb_leaf_kernel, dim3(nleaf), dim3(gjb::NT), 0, st, descs, nleaf, bs, Dh,
                     Dh2, info);
  return hipGetLastError();
}

}  // namespace hps
