// Launchers of the HIP kernels (kernels_*.hip).  All launches are asynchronous
// on the given stream; descriptor arrays live in device memory.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "types.hpp"

namespace hps {

constexpr int kPanelNBMax = 32;   // widest panel of the blocked Gauss-Jordan
int panel_nb(int maxm);           // panel width used for a level of size maxm

// tmap[t] = index (into descs) of the descriptor that owns tile t
// leaves per chunk of the storage-economic build and solve
constexpr int kEconChunk = 1024;
// leaves of one role per workgroup of leaf_b_kernel
constexpr int kLeafBChunk = 16;
// info code of a leaf Gauss-Jordan whose flag-synchronised sweep gave up
// waiting (never in a correct run)
constexpr int kGjSyncTimeout = -0x7fffffff;
constexpr int kGemmVariants = 8;  // tile shapes of the grouped GEMM (see gemm_variant_tm/tn)
int gemm_variant_tm(int v);
int gemm_variant_tn(int v);
hipError_t launch_gemm(int variant, const GemmDesc *descs, const int32_t *tmap, int64_t ntiles,
                       const Bases &bs, hipStream_t st);
int gj_leaf_supported(int p);
// the leaf kernel of order p forms H = D_ge,ci F itself (4q rows fit in its
// padding rows)
inline bool leaf_kernel_forms_h(int p, int g4) { return p == 16 && 196 + g4 <= 256; }
hipError_t launch_gjb_leaf(const LeafDesc *descs, int nleaf, const Bases &bs, const double *Dh,
                           const double *Dh2, int32_t *info, hipStream_t st);
hipError_t launch_gj_leaf(int p, const LeafDesc *descs, int nleaf, const Bases &bs,
                          const double *Dh, const double *Dh2, int32_t *info, hipStream_t st);
// B = A_ci,ce L of every leaf (mi x g4), from the role's products K_t L;
// leaves in chunks of one role (chunks: [first, count] pairs into lidx, the
// leaf descriptor indices)
hipError_t launch_leaf_b(const LeafDesc *descs, const int32_t *chunks, int nchunks,
                         const int32_t *lidx, const Bases &bs, int p, int g4, hipStream_t st);
int gj_merge_class(int m);
hipError_t launch_gj_merge(int cls, const MergeInvDesc *descs, int nd, const Bases &bs,
                           int32_t *info, hipStream_t st);
hipError_t launch_zdiff(const MergeInvDesc *descs, int nd, int maxm, const Bases &bs,
                        hipStream_t st);
hipError_t launch_gj_panel(const MergeInvDesc *descs, int nd, int kb, int maxm,
                           const Bases &bs, int32_t *ipiv, int32_t *info, hipStream_t st);
// int scratch of one blocked inversion of an m x m block: pivrow[m],
// stepof[m], kGjLevelCtl control words of the level form (ready, ticket),
// progress[strips of 16]
constexpr int kGjLevelCtl = 32;
inline int64_t gj_int_scratch(int m) { return 2 * int64_t(m) + kGjLevelCtl + (m + 15) / 16; }
// One launch for the whole blocked inversion of a level, every strip resident
// (only where gj_level_fits(maxm, nd) holds for the current device).
bool gj_level_fits(int maxm, int nd);
bool gj_level_force_retire();
hipError_t launch_gj_level(const MergeInvDesc *descs, int nd, int maxm, const Bases &bs,
                           int32_t *ipiv, int32_t *info, int retire, hipStream_t st);
hipError_t launch_gj_ginit(const MergeInvDesc *descs, int nd, int maxm, int32_t *g,
                           hipStream_t st);
hipError_t launch_gj_colperm(const MergeInvDesc *descs, int nd, int maxm, const Bases &bs,
                             int32_t *ipiv, int32_t *src, hipStream_t st);
hipError_t launch_apply(int prec, const ApplyDesc *descs, const int32_t *tmap,
                        int64_t ntiles, const Bases &bs, int nrhs, hipStream_t st,
                        bool trans = false);
hipError_t launch_apply_finalize(const ApplyDesc *descs, const int32_t *list, int nlist,
                                 int64_t maxm, const Bases &bs, int nrhs, hipStream_t st);
hipError_t launch_copy_map(const Bases &bs, const VRef &dst, const VRef &src, int64_t n,
                           int nrhs, hipStream_t st);
hipError_t launch_vecop(const VecOpDesc *descs, int nd, int64_t maxn, const Bases &bs, int nrhs,
                        hipStream_t st);
hipError_t launch_cast_f32(const double *src, float *dst, int64_t n, hipStream_t st);
// *flag |= 1 if src[e] != src[e % per] for some e < n (flag cleared by the caller)
hipError_t launch_block_diff(const double *src, int64_t per, int64_t n, int32_t *flag,
                             hipStream_t st);
hipError_t launch_fill(double *dst, double v, int64_t n, hipStream_t st);

}  // namespace hps
