// Descriptor records shared by the host planner and the HIP kernels.
//
// Every matrix is column-major.  A location is (buffer id, element offset);
// the kernels receive the buffer base pointers in a small by-value table, so
// one descriptor list serves any set of caller buffers.
#pragma once
#include <cstdint>

namespace hps {

enum BufId : int32_t {
  BUF_WS = 0,     // FP64 operator workspace (owned by the handle)
  BUF_SCR = 1,    // FP64 scratch (build temporaries, split-K partials)
  BUF_IN0 = 2,    // per-call inputs/outputs (coeffs, f, g, u, ...)
  BUF_IN1 = 3,
  BUF_IN2 = 4,
  BUF_VEC = 5,    // per-solve work vectors (h / w slots, global u, residuals)
  BUF_W32 = 6,    // FP32 operator copies
  BUF_AUX = 7,
  BUF_COEF = 8,   // the handle's copy of the nodal coefficients
  NBUF = 9
};

struct Bases {
  void *d[NBUF];
  const int32_t *imap;  // integer maps (gather/scatter lists)
  const int32_t *iota;  // iota[k] = k for every k an apply reads (unmapped operands)
};

struct Ref {
  int32_t buf;  // < 0: absent
  int32_t ld;
  int64_t off;
};

// C(i,j) = alpha * sum_k A(i,k) B(k,j) + beta * D(i,j), written at
// C[crow(i) + ccol(j) * ldc] (maps optional).  With msplit > 0 the rows of A
// from msplit on come from A2 (its row i - msplit), and D is block-diagonal:
// D(i,j) for i, j < msplit, D2(i - msplit, j - msplit) for i, j >= msplit,
// 0 elsewhere (the merge's T = blkdiag(T11a, T22b) + [T13a; T23b] S as one
// product).
struct GemmDesc {
  int32_t M, N, K, tn;
  int64_t tile0;
  Ref A, B, C, D;
  int64_t crow, ccol;   // offsets into imap, -1 = identity
  double alpha, beta;
  Ref A2, D2;
  int32_t msplit, pad;
};

// Leaf interior block: assemble A_ci,ci and A_ci,ce from the nodal
// coefficients, invert A_ci,ci in place (Gauss-Jordan, partial pivoting).
struct LeafDesc {
  int64_t coef;   // BUF_COEF offset of the leaf's [6][p*p] coefficients
  int64_t F;      // offset of F (mi x mi, ld mi) in buffer fbuf
  double sx, sy;  // 2/hx, 2/hy
  int32_t info;   // slot in the info array
  int32_t fbuf;   // buffer of F: BUF_WS (stored) or BUF_SCR (recomputed per chunk)
  // p = 16 kernel: H = D_ge,ci F formed in the same sweeps (hrows = 4q rows
  // of D_ge,ci at BUF_WS offset Dci and of H at offset H, both ld hrows);
  // hrows = 0: H is not formed here
  int64_t Dci, H;
  int32_t hrows, pad;
  // leaf_b_kernel: B = A_ci,ce L (mi x 4q, ld mi) at BUF_SCR offset Bout, from
  // the five products K_t L of the leaf's role (BUF_WS offset Mb, each
  // mi x 4q, ld mi)
  int64_t Bout, Mb;
};

// Interface block of a merge: X = (T33a - T33b)^-1.
struct MergeInvDesc {
  int64_t Ta, Tb;   // BUF_WS offsets of the T33 blocks
  int32_t lda, ldb;
  int32_t m, info;
  int64_t X;        // BUF_WS offset, ld m
  int64_t W;        // BUF_SCR offset of the blocked path's pivot-row panel
  int64_t ipiv;     // imap-independent int scratch offset (blocked path)
};

// Vector operand of the solve-stage applies.  With i = off + (map >= 0 ?
// imap[map + k] : k), element (k, r) is base[buf][i + r * stride] (RHS-major,
// stride >= 0) or base[buf][i * nrhs + r] (RHS-interleaved, stride < 0).
constexpr int64_t kInterleaved = -1;

struct VRef {
  int32_t buf;
  int32_t pad;
  int64_t off, map, stride;
};

// C(map(i), r) = alpha * sum_k A(i,k) B(k,r) + beta * D(i,r)
// (or A(k,i) for the transposed launch).  B rows k < K1 come from B1,
// k >= K1 from B2 (mode 0); in mode 1 B(k) = B1(k) - B2(k) (+ B3(k) if
// present); in mode 2 B(k) = B1(k) + B2(k); K = K1 in modes 1 and 2.
struct ApplyDesc {
  int32_t M, K1, K2, mode;
  int32_t ksl, rb;      // k-slices and 64-row blocks
  int64_t tile0;
  int32_t abuf, lda;
  int64_t aoff;
  VRef B1, B2, B3, C, D;
  double alpha, beta;
  int64_t part;         // split-K partials start at BUF_SCR[part * nrhs]
};

// dst(k, r) = ca * a(k, r) + cb * b(k, r) for k < n (absent operands are 0).
struct VecOpDesc {
  int32_t n, pad;
  VRef dst, a, b;
  double ca, cb;
};

}  // namespace hps
