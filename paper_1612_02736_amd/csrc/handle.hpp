// Internal handle / tree objects behind the C ABI (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/hps.h"
#include "plan.hpp"
#include "types.hpp"

namespace hps {

inline thread_local std::string g_err;

inline int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                              \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess)                                                         \
      return hps::fail(HPS_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
struct DevArray {
  T *p = nullptr;
  size_t n = 0;
  bool owned = true;    // false: caller-owned memory (never freed here)
  ~DevArray() { reset(); }
  void reset() {
    if (p && owned) (void)hipFree(p);
    p = nullptr;
    n = 0;
    owned = true;
  }
  hipError_t alloc(size_t count) {
    reset();
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)&p, count * sizeof(T));
    if (e == hipSuccess) n = count;
    return e;
  }
  void borrow(T *q, size_t count) {
    reset();
    p = q;
    n = count;
    owned = false;
  }
  hipError_t upload(const std::vector<T> &v) {
    hipError_t e = alloc(v.size());
    if (e != hipSuccess) return e;
    if (!v.empty()) e = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
  }
};

enum StepKind {
  S_GEMM, S_GJ_LEAF, S_GJ_MERGE, S_ZDIFF, S_PANEL, S_COLPERM, S_APPLY, S_COPY_F, S_VECOP,
  S_LEAF_B
};

constexpr int kPanelLevel = -(1 << 30);
struct Step {
  StepKind kind;
  int cls = 0;
  int64_t d0 = 0, nd = 0;   // descriptor range
  int64_t ntiles = 0;
  int maxm = 0;
  int kb = 0;                 // PANEL: panel start, or kPanelLevel (one launch per level)
  int64_t fin0 = 0, nfin = 0;  // APPLY: finalize list range
  int64_t fin_maxm = 0;
  int64_t tmap0 = 0;          // GEMM / APPLY: start of the step's tile map
  bool trans = false;         // APPLY: transposed operator
  // GEMM: tile variant in use (set by the tuner) and, per variant, the
  // start of the step's tile map and its tile count
  int var = 0;
  int64_t vtmap0[8] = {}, vtiles[8] = {};
  // Algorithmic work of the launch: flops (GEMM, Gauss-Jordan, panel) or
  // operator elements read per right-hand side (APPLY).
  double work = 0.0;
};


struct SolveExt;
void solve_ext_free(SolveExt *);
struct SolveExtDeleter {
  void operator()(SolveExt *p) const { solve_ext_free(p); }
};

}  // namespace hps

struct hps_tree {
  hps::TreeDesc t;
};

struct hps_handle {
  hps::TreeDesc tree;
  hps::Plan pl;
  int p = 0, q = 0, mi = 0, me = 0, g4 = 0;
  int nleaf = 0;
  // device memory
  hps::DevArray<double> ws, scr, coef, vec, part, aux;
  hps::DevArray<float> ws32;
  hps::DevArray<int32_t> imap, info, ipiv, psrc;
  size_t solve_elems = 0;
  // descriptors
  // GEMM descriptors and tile maps, one copy per tile variant (the
  // descriptors differ only in their tiling fields)
  hps::DevArray<hps::GemmDesc> d_gemm_v[8];
  hps::DevArray<int32_t> d_gemm_tmap_v[8];
  hps::DevArray<int32_t> d_apply_tmap;   // tile -> descriptor (per step)
  hps::DevArray<hps::LeafDesc> d_leaf;
  hps::DevArray<hps::MergeInvDesc> d_minv;
  hps::DevArray<hps::ApplyDesc> d_apply;
  hps::DevArray<int32_t> d_finlist;
  std::vector<hps::Step> build_prog, up_prog, down_prog, adj_down_prog, adj_up_prog;
  std::vector<hps::Step> up_jump_prog, ext_prog;   // refinement-correction solve
  hps::DevArray<hps::VecOpDesc> d_vecop;
  // flux-jump residual maps (uniform trees): interior node id, flux index of
  // the west/south leaf and of the east/north leaf
  hps::DevArray<int32_t> d_jn, d_fa, d_fb, d_fp;
  int64_t iota_off = 0;            // imap offset of the identity map
  std::vector<int32_t> h_jn, h_fa, h_fb, h_fp;   // host copies, uploaded by hps_build
  std::vector<double> h_lloc;
  int64_t n_jump = 0;
  bool conforming = true;     // no refined interfaces
  hps::DevArray<double> d_lloc;   // q x p row-major Chebyshev -> Gauss
  int64_t map_fbar = -1;
  // offsets
  int64_t vec_per_rhs = 0;       // doubles per right-hand side in BUF_VEC
  int64_t ug_off = 0;            // global Gauss vector inside a RHS block
  int64_t part_per_rhs = 0;      // split-K partial doubles per RHS
  int64_t map_bdry = -1;
  int64_t n_bdry = 0;
  int64_t Dh_off = 0, Dh2_off = 0;  // in aux
  int64_t ice_map = -1, ici_map = -1;
  int n_info = 0;
  bool has_fp32 = false;
  // storage-economic build: leaf F not kept; the solve redoes the leaf
  // Gauss-Jordan in chunks of econ_chunk leaves (econ_chunk = nleaf otherwise)
  bool econ = false;
  int econ_chunk = 0;
  // translation-invariant build: boxes with identical operators share one copy
  bool dedup = false;
  hps::DevArray<int32_t> cflag;   // device flag of the constant-coefficient check
  std::vector<int64_t> off_T, off_X, off_S, off_LD, off_H;   // per box, -1 if absent
  int64_t scr_build = 0;          // scratch doubles the build needs
  // optional per-step timing (test hook): events around every launch step
  bool prof_on = false;
  bool tune_gemm = false;         // time the GEMM tile variants in the next build pass
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof_ev;
  std::vector<double> prof_work;
  std::vector<hipEvent_t> prof_pool;
  size_t prof_used = 0;
  std::unique_ptr<hps::SolveExt, hps::SolveExtDeleter> ext;
  // refactorization replays the build program as one HIP graph, captured on
  // the first refactor (and again if the scratch buffer has moved)
  hipGraphExec_t build_exec = nullptr;
  const void *build_exec_scr = nullptr;
  ~hps_handle() {
    for (hipEvent_t e : prof_pool) (void)hipEventDestroy(e);
    if (build_exec) (void)hipGraphExecDestroy(build_exec);
  }
};

