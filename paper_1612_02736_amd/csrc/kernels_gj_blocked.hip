// Blocked Gauss-Jordan inversion of large interface blocks (m > 196) of the
// merges (Sec. 4).
#include <cstdlib>

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

// Blocked Gauss-Jordan with implicit partial pivoting (no row interchanges)
// over panels of NB columns.  The panel sweep is the textbook one restricted
// to the panel's columns: the pivot row of column k is the unused row of
// largest magnitude.  If R is the set of a panel's pivot rows and L the
// product of its elementary sweep matrices, L differs from I only in the
// columns R and the swept panel column c holds L(:, r_c); every other column
// B therefore becomes L B = (B with rows R set to 0) + P W, with P the swept
// panel columns and W(c, :) = B(r_c, :).  After the last panel the swept
// matrix M has M[r_k][k'] = inv[k][r_k'], which gj_perm_kernel turns into the
// inverse.  pivrow[k] = r_k and stepof[r] = the step that used row r (-1
// before) live in int scratch.
//
// One workgroup holds one strip of NB columns in registers (row t + NT i by
// thread t).  Two drivers share the strip update and the sweep below: one
// launch per panel (gj_step_kernel), or one launch per level in which every
// strip stays in registers from the first panel to the last and the panels
// pass through memory (gj_level_kernel).

// Loads and stores of panels passed between workgroups inside one launch of
// the level form carry the sc1 cache-policy bit (the bit agent-scope atomics
// use), which keeps them coherent across the XCDs' L2 caches without a
// cache-wide write-back or invalidation.  Panel columns go through buffer
// instructions over the panel (num_records bytes): an offset past the end
// loads 0 and drops a store, so inactive rows and columns need no branch.  Single words
// (pivot rows, counters) are agent-scope relaxed atomics.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int kBufSc1 = 16;               // cache policy: sc1
constexpr unsigned kBufOut = 0x7ffffff0u; // an offset past every panel
__device__ __forceinline__ __amdgpu_buffer_rsrc_t panel_rsrc(const double *p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(p), 0, bytes, 0x00020000);
}
__device__ __forceinline__ double coherent_load(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, kBufSc1));
}
__device__ __forceinline__ void coherent_store(__amdgpu_buffer_rsrc_t r, unsigned off, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, kBufSc1);
}
__device__ __forceinline__ void coherent_store(__amdgpu_buffer_rsrc_t r, unsigned off, int32_t v) {
  __builtin_amdgcn_raw_buffer_store_b32(v, r, off, 0, kBufSc1);
}
__device__ __forceinline__ int32_t coherent_load(const int32_t *p) {
  return __hip_atomic_load(const_cast<int32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void coherent_store(int32_t *p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int NB, int NW>
struct StripShared {
  unsigned wkey[2][NW];
  double crow[2][NW][NB];
  __align__(16) double Wsh[NB][NB];
  int rsh[NB];
  int pivl[NB];                // pivot rows of the strip's sweep
  int timeout;                 // gj_level_kernel: 1 a wait ran out, 2 retired
  int strip;                   // gj_level_kernel: the strip taken
};

// pan <- (pan with rows R set to 0) + P W for a panel of nbv <= K swept
// columns P (column c at P + c n) whose pivot rows are piv[0 .. nbv - 1].  The
// threads holding the rows R copy them to LDS as W first.  Returns the mask
// of this thread's register rows that are in R.  COHERENT: P and piv were
// published by another workgroup of this launch.
template <int NB, int K, int RPT, int NT, bool COHERENT = false>
__device__ __forceinline__ unsigned strip_update(double (&pan)[RPT][NB], const double *P, int n,
                                                 int nbv, const int32_t *piv,
                                                 StripShared<NB, NT / 64> &sh) {
  const int tid = threadIdx.x;
  const __amdgpu_buffer_rsrc_t rs = panel_rsrc(P, COHERENT ? nbv * n * 8 : 0);
  // entry (row, c) of the panel, 0 outside it
  auto ldP = [&](int row, int c) -> double {
    if constexpr (COHERENT)
      return coherent_load(rs, row < n ? unsigned(row + c * n) * 8u : kBufOut);
    else
      return (row < n && c < nbv) ? P[row + int64_t(c) * n] : 0.0;
  };
  // my rows of the swept panel, loaded up front where registers allow
  constexpr bool PRE = RPT <= 2;
  double pr[PRE ? RPT : 1][K];
  if constexpr (PRE) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int row = tid + NT * i;
#pragma unroll
      for (int c = 0; c < K; ++c) pr[i][c] = ldP(row, c);
    }
  }
  if (tid < K) sh.rsh[tid] = tid < nbv ? (COHERENT ? coherent_load(piv + tid) : piv[tid]) : -1;
  for (int e = tid; e < K * NB; e += NT)
    if (e / NB >= nbv) sh.Wsh[e / NB][e % NB] = 0.0;
  __syncthreads();
  // W = the strip's rows R (old values), from the threads that hold them
  unsigned rmask = 0u;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int row = tid + NT * i;
#pragma unroll
    for (int c = 0; c < K; ++c)
      if (sh.rsh[c] == row) {
        rmask |= 1u << i;
#pragma unroll
        for (int j = 0; j < NB; ++j) sh.Wsh[c][j] = pan[i][j];
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
    for (int c = 0; c < K; ++c) {
      const double2 *wr = reinterpret_cast<const double2 *>(&sh.Wsh[c][0]);
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
      for (int i = 0; i < RPT; ++i) pc[i] = ldP(tid + NT * i, c);
      const double2 *wr = reinterpret_cast<const double2 *>(&sh.Wsh[c][0]);
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
  return rmask;
}

// Half h of panel q of the level form (columns 8 h .. 8 h + 7 of the panel in
// Y, as published): L0 for h = 0, L1 for h = 1.
template <int NB, int RPT, int NT, bool COHERENT>
__device__ __forceinline__ unsigned strip_half_update(double (&pan)[RPT][NB], const double *Y,
                                                      int n, int q, int h, const int32_t *pivrow,
                                                      StripShared<NB, NT / 64> &sh) {
  constexpr int H = NB / 2;
  const int k0 = q * NB + h * H;
  return strip_update<NB, H, RPT, NT, COHERENT>(pan, Y + int64_t(k0) * n, n, min(H, n - k0),
                                                pivrow + k0, sh);
}

// Where the level form publishes a strip's panel: its swept columns into the
// scratch copy Y, its pivot rows into pivrow / stepof, and the matrix's
// counter `ready` in half-panels (2 s: columns 0..7 of panel s, 2 s + 1: all).
struct PanelOut {
  double *Y;
  int32_t *ipiv;               // pivrow[n], then stepof[n]
  int32_t *ready;
  int n, s;
};

// Columns cfrom .. cto - 1 of the strip (starting at column c0) and their
// pivot rows, with sc1 stores; the caller waits for them before signalling.
template <int NB, int RPT, int NT>
__device__ __forceinline__ void publish_half(const double (&pan)[RPT][NB], const PanelOut &o,
                                             int c0, int cfrom, int cto,
                                             const StripShared<NB, NT / 64> &sh) {
  const __amdgpu_buffer_rsrc_t rs = panel_rsrc(o.Y + int64_t(c0) * o.n, NB * o.n * 8);
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int row = threadIdx.x + NT * i;
#pragma unroll
    for (int c = 0; c < NB; ++c)
      coherent_store(rs, (row < o.n && c >= cfrom && c < cto) ? unsigned(row + c * o.n) * 8u
                                                               : kBufOut,
                     pan[i][c]);
  }
  // pivot rows (threads of wavefront 0, which also wrote sh.pivl)
  const int t = threadIdx.x, c = cfrom + t;
  if (t < NB) {
    const bool on = c < cto;
    const int r = on ? sh.pivl[c] : 0;
    const __amdgpu_buffer_rsrc_t ri =
        __builtin_amdgcn_make_buffer_rsrc(o.ipiv, 0, 8 * o.n, 0x00020000);
    coherent_store(ri, on ? unsigned(c0 + c) * 4u : kBufOut, r);
    coherent_store(ri, on ? unsigned(o.n + r) * 4u : kBufOut, c0 + c);
  }
}

// Sweep of the nbv columns of the strip starting at column c0, umask holding
// the register rows already used as pivots (or padding).  One barrier per
// column: every wavefront's best candidate row travels to LDS with its key,
// so after the barrier all threads read the pivot row from the winning
// wavefront's slot.  Pivot rows are kept unscaled until the pivot row itself
// is written (one multiply per row and column step).  The pivot rows are
// left in sh.pivl.  With PUB (the level form) the sweep publishes its first
// 8 columns as they stand after step 7 (stores issued before step 8, the
// counter raised after step 10 once they are complete), and the rest after
// the last step.  Returns the first failed step (+-(k + 1), as info reports
// it) or 0.
template <int NB, int RPT, int NT, bool PUB = false>
__device__ __forceinline__ int strip_sweep(double (&pan)[RPT][NB], unsigned &umask, int c0,
                                           int nbv, StripShared<NB, NT / 64> &sh,
                                           const PanelOut *out = nullptr) {
  constexpr int NW = NT / 64;
  constexpr int H = NB / 2;        // columns of the first published half
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  int first_bad = 0;
  // this thread's candidate row for column c (key, register row bi) and the
  // wavefront's maximum key; step c computes them for column c + 1 right
  // after updating that column, so the reduction overlaps the other updates
  unsigned key = 0, wmax = 0;
  int bi = 0;
  auto search = [&](int c) {
    key = 0;
    bi = 0;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const unsigned k2 = ((umask >> i) & 1u) ? 0u : pivot_key(pan[i][c], tid + NT * i);
      if (k2 > key) { key = k2; bi = i; }
    }
    wmax = wave_max_u32(key);
  };
  if (nbv > 0) search(0);
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (c < nbv) {
      if constexpr (PUB)
        if (c == H) publish_half<NB, RPT, NT>(pan, *out, c0, 0, H, sh);
      const int par = c & 1;
      if (key == wmax && key != 0) {             // this wavefront's candidate row
#pragma unroll
        for (int i = 0; i < RPT; ++i)
          if (i == bi) {
#pragma unroll
            for (int cc = 0; cc < NB; ++cc) sh.crow[par][wid][cc] = pan[i][cc];
          }
      }
      if (lane == 0) sh.wkey[par][wid] = wmax;
      if constexpr (PUB)
        if (c == H + 2) __builtin_amdgcn_s_waitcnt(0);   // the first half's stores
      __syncthreads();
      if constexpr (PUB)
        if (c == H + 2 && tid == 0) coherent_store(out->ready, 2 * out->s);
      unsigned best = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) best = max(best, sh.wkey[par][w]);
      // row r is held by thread r mod NT, so its candidate slot is that
      // thread's wavefront
      const int r = __builtin_amdgcn_readfirstlane(key_row(best));
      const double *prow = sh.crow[par][(r % NT) >> 6];
      if (tid == 0) sh.pivl[c] = r;
      const double piv = prow[c];
      const bool ok = (piv != 0.0) && isfinite(piv);
      if (!ok && first_bad == 0) first_bad = isfinite(piv) ? (c0 + c + 1) : -(c0 + c + 1);
      const double ip = ok ? recip_f64(piv) : 0.0;
      double sr[NB];             // the pivot row, unscaled
#pragma unroll
      for (int cc = 0; cc < NB; ++cc) sr[cc] = prow[cc];
      double f[RPT];
      unsigned isr = 0u;         // register rows that are the pivot row
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        f[i] = pan[i][c] * ip;
        if (tid + NT * i == r) isr |= 1u << i;
      }
      umask |= isr;
      if (c + 1 < NB) {
        // the next pivot column first, then its candidate search (the pivot
        // row, fixed below, is already excluded through umask)
#pragma unroll
        for (int i = 0; i < RPT; ++i) pan[i][c + 1] = fma(-f[i], sr[c + 1], pan[i][c + 1]);
        if (c + 1 < nbv) search(c + 1);
      }
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
#pragma unroll
        for (int cc = 0; cc < NB; ++cc)
          if (cc != c && cc != c + 1) pan[i][cc] = fma(-f[i], sr[cc], pan[i][cc]);
        pan[i][c] = -f[i];
      }
      // the pivot row itself, in the one wavefront that holds it
      if (((r % NT) >> 6) == wid) {
#pragma unroll
        for (int i = 0; i < RPT; ++i)
          if ((isr >> i) & 1u) {
#pragma unroll
            for (int cc = 0; cc < NB; ++cc) pan[i][cc] = cc == c ? ip : sr[cc] * ip;
          }
      }
    }
  }
  __syncthreads();
  if constexpr (PUB) {
    // the second half (or the whole panel when it has at most H columns)
    publish_half<NB, RPT, NT>(pan, *out, c0, nbv > H ? H : 0, nbv, sh);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) coherent_store(out->ready, 2 * out->s + 1);
  }
  return first_bad;
}

template <int NB, int RPT, int NT>
__device__ __forceinline__ void strip_load(double (&pan)[RPT][NB], const double *src, int n,
                                           int ncv) {
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int row = threadIdx.x + NT * i;
#pragma unroll
    for (int c = 0; c < NB; ++c)
      pan[i][c] = (row < n && c < ncv) ? src[row + int64_t(c) * n] : 0.0;
  }
}

template <int NB, int RPT, int NT>
__device__ __forceinline__ void strip_store(const double (&pan)[RPT][NB], double *dst, int n,
                                            int ncv) {
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int row = threadIdx.x + NT * i;
    if (row < n) {
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < ncv) dst[row + int64_t(c) * n] = pan[i][c];
    }
  }
}

// Launch kb (kb < 0: the first) has one workgroup per strip: every strip
// other than panel kb applies panel kb's update, and the strip of the next
// panel then sweeps its columns in the same registers, so the next panel's
// sweep follows its update without a launch in between and only the columns
// of a strip are written by the strip's own workgroup.
template <int NB, int RPT, int NT>
__global__ __launch_bounds__(NT) void gj_step_kernel(
    const MergeInvDesc *__restrict__ descs, int nd, int kb, Bases bs,
    int32_t *__restrict__ g_all, int32_t *__restrict__ info) {
  __shared__ StripShared<NB, NT / 64> sh;
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
  double pan[RPT][NB];
  strip_load<NB, RPT, NT>(pan, A + int64_t(c0) * n, n, ncv);
  if (kb >= 0)
    (void)strip_update<NB, NB, RPT, NT>(pan, A + int64_t(kb) * n, n, min(NB, n - kb),
                                        pivrow + kb, sh);
  int first_bad = 0;
  if (sweep) {
    unsigned umask = 0u;          // rows already used as pivots (or padding)
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int row = threadIdx.x + NT * i;
      if (row >= n || stepof[row] >= 0) umask |= 1u << i;
    }
    first_bad = strip_sweep<NB, RPT, NT>(pan, umask, c0, ncv, sh);
    if (threadIdx.x < ncv) {
      const int r = sh.pivl[threadIdx.x];
      pivrow[c0 + threadIdx.x] = r;
      stepof[r] = c0 + threadIdx.x;
    }
  }
  strip_store<NB, RPT, NT>(pan, A + int64_t(c0) * n, n, ncv);
  if (sweep && threadIdx.x == 0 && first_bad != 0 && info[d.info] == 0) info[d.info] = first_bad;
}

// One launch per level (gj_level_kernel, then gj_level_rest_kernel): every
// strip stays in registers while the panels pass through memory.  A
// workgroup takes the next strip of its matrix in order of arrival (a ticket
// counter), applies panels 0 .. s - 1 as they are published, sweeps panel s
// and publishes it in two halves (strip_sweep), and goes on applying the
// later panels.  A panel is applied as two rank-8 updates, its first 8
// columns as they stood after the first 8 steps (L0) and then the rest (L1),
// so a strip applies L0 of panel q while q's owner still sweeps its second
// half, and only L1 separates the end of one sweep from the start of the
// next.  Waits before the sweep are on panels whose owners arrived earlier,
// so they always end; after its sweep a workgroup waits for panel q only
// while q's owner has arrived, and otherwise retires after kRetireTicks
// (records in progress[s] the last panel applied and stores its strip), so no
// workgroup ever waits on one that cannot be scheduled, whatever else runs on
// the device.  gj_level_rest_kernel then applies the panels a retired strip
// missed (none when the grid was resident throughout).  Every wait is also
// bounded (2^20 polls), after which the matrix reports kGjSyncTimeout through
// info.
//
// Ordering across workgroups (which may sit on different XCDs with their own
// L2): the panel, its pivot rows and the counter are written and read with
// sc1 accesses, coherent at agent scope without a cache-wide write-back or
// invalidation.  The publishing workgroup waits for all its stores to
// complete (s_waitcnt on every thread), meets at a barrier, then one thread
// stores the counter; a waiting workgroup polls the counter with one thread,
// meets at a barrier, and only then loads the panel, so every load is issued
// after the counter was seen.
constexpr unsigned kLevelSpinLimit = 1u << 20;
constexpr uint64_t kRetireTicks = 10000;      // 100 us of the 100 MHz real-time counter

template <int NB, int RPT, int NT>
__global__ __launch_bounds__(NT) void gj_level_kernel(
    const MergeInvDesc *__restrict__ descs, int nd, Bases bs, int32_t *__restrict__ g_all,
    int32_t *__restrict__ info, int retire_after_sweep) {
  __shared__ StripShared<NB, NT / 64> sh;
  const MergeInvDesc &d = descs[blockIdx.y];
  const int n = d.m, np = (n + NB - 1) / NB;
  if (int(blockIdx.x) >= np) return;
  const int tid = threadIdx.x;
  int32_t *pivrow = g_all + d.ipiv;
  int32_t *stepof = pivrow + n;
  int32_t *ready = pivrow + 2 * n, *ticket = ready + 1, *progress = ready + kGjLevelCtl;
  if (tid == 0) {
    sh.timeout = 0;
    sh.strip = __hip_atomic_fetch_add(ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  const int s = __builtin_amdgcn_readfirstlane(sh.strip);
  const int c0 = s * NB, ncv = min(NB, n - c0);
  double *A = (double *)bs.d[BUF_WS] + d.X;
  double *Y = (double *)bs.d[BUF_SCR] + d.W;     // published panels (n x n)
  double pan[RPT][NB];
  strip_load<NB, RPT, NT>(pan, A + int64_t(c0) * n, n, ncv);
  unsigned umask = 0u;            // rows already used as pivots (or padding)
#pragma unroll
  for (int i = 0; i < RPT; ++i)
    if (tid + NT * i >= n) umask |= 1u << i;
  // wait for half-panel h of panel h / 2 (retiring instead if that panel
  // follows the sweep and its owner has not arrived); false: stop
  auto wait_half = [&](int h, bool may_retire) -> bool {
    const int q = h >> 1;
    if (tid == 0) {
      uint64_t t0 = 0;
      for (unsigned spins = 0;; ++spins) {
        if (coherent_load(ready) >= h) break;
        if (may_retire && coherent_load(ticket) <= q) {
          const uint64_t t = __builtin_amdgcn_s_memrealtime();
          if (t0 == 0) t0 = t;
          else if (t - t0 > kRetireTicks) {
            sh.timeout = 2;
            break;
          }
        }
        if (spins >= kLevelSpinLimit) {
          sh.timeout = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __syncthreads();
    return sh.timeout == 0;
  };
  constexpr int H = NB / 2;
  int first_bad = 0, done_to = -1;
  bool go = true;
  for (int h = 0; h < 2 * s; ++h) {             // the halves of the full panels before s
    if (!(go = wait_half(h, false))) break;
    umask |= strip_half_update<NB, RPT, NT, true>(pan, Y, n, h >> 1, h & 1, pivrow, sh);
    done_to = (h - 1) >> 1;
  }
  if (go) {
    const PanelOut out{Y, pivrow, ready, n, s};
    first_bad = strip_sweep<NB, RPT, NT, true>(pan, umask, c0, ncv, sh, &out);
    done_to = s;
    for (int q = s + 1; q < np && !retire_after_sweep; ++q) {
      if (!wait_half(2 * q, true)) break;
      (void)strip_half_update<NB, RPT, NT, true>(pan, Y, n, q, 0, pivrow, sh);
      if (n - q * NB > H) {
        if (!wait_half(2 * q + 1, false)) break;
        (void)strip_half_update<NB, RPT, NT, true>(pan, Y, n, q, 1, pivrow, sh);
      }
      done_to = q;
    }
  }
  strip_store<NB, RPT, NT>(pan, A + int64_t(c0) * n, n, ncv);
  if (tid == 0) {
    progress[s] = done_to;
    if (sh.timeout == 1) info[d.info] = kGjSyncTimeout;
    else if (first_bad != 0 && info[d.info] == 0) info[d.info] = first_bad;
  }
}

// The panels after progress[s] that a retired strip s did not apply (all
// published by now).
template <int NB, int RPT, int NT>
__global__ __launch_bounds__(NT) void gj_level_rest_kernel(
    const MergeInvDesc *__restrict__ descs, int nd, Bases bs, int32_t *__restrict__ g_all) {
  __shared__ StripShared<NB, NT / 64> sh;
  const MergeInvDesc &d = descs[blockIdx.y];
  const int n = d.m, np = (n + NB - 1) / NB;
  const int s = blockIdx.x;
  if (s >= np) return;
  const int32_t *pivrow = g_all + d.ipiv;
  const int32_t *progress = pivrow + 2 * n + kGjLevelCtl;
  const int q0 = progress[s] + 1;
  if (q0 >= np) return;
  const int c0 = s * NB, ncv = min(NB, n - c0);
  double *A = (double *)bs.d[BUF_WS] + d.X;
  const double *Y = (const double *)bs.d[BUF_SCR] + d.W;
  double pan[RPT][NB];
  strip_load<NB, RPT, NT>(pan, A + int64_t(c0) * n, n, ncv);
  for (int q = q0; q < np; ++q) {
    if (q == s) continue;
    // the two halves in the order of the level kernel
    (void)strip_half_update<NB, RPT, NT, false>(pan, Y, n, q, 0, pivrow, sh);
    __syncthreads();            // W of this half read by every thread
    if (n - q * NB > NB / 2) {
      (void)strip_half_update<NB, RPT, NT, false>(pan, Y, n, q, 1, pivrow, sh);
      __syncthreads();
    }
  }
  strip_store<NB, RPT, NT>(pan, A + int64_t(c0) * n, n, ncv);
}

// stepof = -1 before the first panel; pivrow[k] = k (in range even if a
// failed build leaves a step without a pivot); no panel published yet
__global__ __launch_bounds__(256) void gj_ginit_kernel(const MergeInvDesc *__restrict__ descs,
                                                       int nd, int32_t *__restrict__ g_all) {
  const MergeInvDesc &d = descs[blockIdx.y];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.m; i += gridDim.x * blockDim.x) {
    g_all[d.ipiv + i] = i;
    g_all[d.ipiv + d.m + i] = -1;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {   // gj_level_kernel: ready, ticket
    g_all[d.ipiv + 2 * d.m] = -1;
    g_all[d.ipiv + 2 * d.m + 1] = 0;
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

// The level form (matrices of up to 1024 rows, one row per thread: larger
// ones need more rows per thread than the registers hold next to a resident
// strip).
static const void *level_kernel_for(int maxm, int &nt) {
  constexpr int NB = 16;
  if (maxm <= 256) { nt = 256; return (const void *)gj_level_kernel<NB, 1, 256>; }
  if (maxm <= 512) { nt = 512; return (const void *)gj_level_kernel<NB, 1, 512>; }
  if (maxm <= 1024) { nt = 1024; return (const void *)gj_level_kernel<NB, 1, 1024>; }
  nt = 0;
  return nullptr;
}

// The level form is chosen where its grid (strips x matrices) is resident at
// once on the current device (otherwise strips would retire and leave their
// work to gj_level_rest_kernel).  HPS_GJ_LEVEL=0 selects the per-panel form.
bool gj_level_fits(int maxm, int nd) {
  const char *e = std::getenv("HPS_GJ_LEVEL");
  if (e && e[0] == '0') return false;
  int nt = 0;
  const void *k = level_kernel_for(maxm, nt);
  if (!k || nd <= 0) return false;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return false;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, nt, 0) != hipSuccess) return false;
  const int64_t grid = int64_t((maxm + 15) / 16) * nd;
  return grid <= int64_t(per_cu) * cus;
}

template <int RPT, int NT>
static hipError_t level_launch(const MergeInvDesc *descs, int nd, int maxm, const Bases &bs,
                               int32_t *g, int32_t *info, int retire, hipStream_t st) {
  constexpr int NB = 16;
  const dim3 grid(unsigned((maxm + NB - 1) / NB), unsigned(nd));
  hipLaunchKernelGGL((gj_level_kernel<NB, RPT, NT>), grid, dim3(NT), 0, st, descs, nd, bs, g,
                     info, retire);
  hipLaunchKernelGGL((gj_level_rest_kernel<NB, RPT, NT>), grid, dim3(NT), 0, st, descs, nd, bs,
                     g);
  return hipGetLastError();
}

hipError_t launch_gj_level(const MergeInvDesc *descs, int nd, int maxm, const Bases &bs,
                           int32_t *g, int32_t *info, int retire, hipStream_t st) {
  if (nd <= 0) return hipSuccess;
  if (maxm <= 256) return level_launch<1, 256>(descs, nd, maxm, bs, g, info, retire, st);
  if (maxm <= 512) return level_launch<1, 512>(descs, nd, maxm, bs, g, info, retire, st);
  if (maxm <= 1024) return level_launch<1, 1024>(descs, nd, maxm, bs, g, info, retire, st);
  return hipErrorInvalidValue;
}

// HPS_GJ_LEVEL=2: every strip of the level form retires right after its
// sweep, so gj_level_rest_kernel applies all later panels (same results;
// exercises the remainder path).
bool gj_level_force_retire() {
  const char *e = std::getenv("HPS_GJ_LEVEL");
  return e && e[0] == '2';
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
