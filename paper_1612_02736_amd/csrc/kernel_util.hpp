// Device helpers shared by the kernel translation units: XCD-aware tile
// order, pivot keys and wavefront reductions, vector operand addressing.
#pragma once
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

static inline unsigned grid_1d(int64_t n, int64_t cap = 65536) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return unsigned(b);
}

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


}  // namespace hps
