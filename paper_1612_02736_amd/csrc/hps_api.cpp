// C ABI of the HPS solver: trees, build (Algorithm 1), solve (Algorithm 2),
// adjoint sweeps and mixed-precision iterative refinement.
//
// The host planner turns the tree into fixed "programs": lists of kernel
// launches over descriptor arrays that are uploaded once per handle.  A build
// or solve is then a replay of its program on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/hps.h"
#include "handle.hpp"
#include "kernels.hpp"
#include "plan.hpp"
#include "solve_ext.hpp"
#include "spectral.hpp"
#include "types.hpp"

using namespace hps;

namespace {


// Host-side descriptor lists of one program, later uploaded.
struct GemmList {
  std::vector<GemmDesc> d;
  std::vector<int32_t> tmap;   // owning descriptor of each tile (index into d)
  int64_t tiles = 0;
  void add(const GemmDesc &g0, int TM = 64, int TN = 64) {   // TM x TN tiles
    GemmDesc g = g0;
    if (g.M <= 0 || g.N <= 0) return;
    g.tn = (g.N + TN - 1) / TN;
    const int64_t tm = (g.M + TM - 1) / TM;
    g.tile0 = tiles;
    tiles += tm * g.tn;
    tmap.insert(tmap.end(), size_t(tm * g.tn), int32_t(d.size()));
    d.push_back(g);
  }
};



Ref ref(int32_t buf, int64_t off, int32_t ld) { return Ref{buf, ld, off}; }
Ref noref() { return Ref{-1, 0, 0}; }
VRef vref(int32_t buf, int64_t off, int64_t map, int64_t stride) {
  return VRef{buf, 0, off, map, stride};
}
VRef novref() { return VRef{-1, 0, 0, -1, 0}; }

}  // namespace

extern "C" {

const char *hps_last_error(void) { return hps::g_err.c_str(); }

int hps_tree_uniform(double x0, double x1, double y0, double y1, int nx, int ny,
                     int n_problems, hps_tree **out) {
  if (!out) return fail(HPS_EINVAL, "out is NULL");
  *out = nullptr;
  if (nx <= 0 || ny <= 0 || n_problems <= 0 || !(x1 > x0) || !(y1 > y0))
    return fail(HPS_EINVAL, "empty rectangle or non-positive leaf count");
  hps_tree *t = new (std::nothrow) hps_tree;
  if (!t) return fail(HPS_ENOMEM, "host allocation");
  for (int k = 0; k < n_problems; ++k) {
    Problem P;
    P.X0 = x0; P.X1 = x1; P.Y0 = y0; P.Y1 = y1; P.nx = nx; P.ny = ny;
    for (int i = 0; i < nx; ++i)
      for (int j = 0; j < ny; ++j) P.leaves.insert({i * kUnit, j * kUnit, kUnit, kUnit, 0});
    t->t.probs.push_back(std::move(P));
  }
  *out = t;
  return HPS_OK;
}

int hps_tree_refine_point(hps_tree *tree, int problem, double px, double py, int n_ref,
                          double t) {
  if (!tree || n_ref < 0 || !(t >= 0.0)) return fail(HPS_EINVAL, "bad refinement arguments");
  if (n_ref > 20) return fail(HPS_EINVAL, "n_ref > 20");
  std::string e = refine_point(tree->t, problem, px, py, n_ref, t);
  if (!e.empty()) return fail(HPS_ETREE, e);
  return HPS_OK;
}

int hps_tree_set_bc(hps_tree *tree, int problem, const int *bc) {
  if (!tree || !bc) return fail(HPS_EINVAL, "NULL argument");
  std::string e = set_bc(tree->t, problem, bc);
  if (!e.empty()) return fail(HPS_EINVAL, e);
  return HPS_OK;
}

static int plan_tree(const TreeDesc &t, Plan &pl, int q) {
  std::string e = build_tree_boxes(t, pl);
  if (!e.empty()) return fail(HPS_ETREE, e);
  if (q > 0) {
    e = plan_gauss(t, pl, q);
    if (!e.empty()) return fail(HPS_ETREE, e);
  }
  return HPS_OK;
}

int hps_tree_info(const hps_tree *tree, hps_tree_info_t *info) {
  if (!tree || !info) return fail(HPS_EINVAL, "NULL argument");
  Plan pl;
  int rc = plan_tree(tree->t, pl, 0);
  if (rc) return rc;
  info->n_problems = (int)tree->t.probs.size();
  info->n_leaves = (int)pl.leaves.size();
  info->n_boxes = (int)pl.boxes.size();
  info->n_levels = pl.max_height;
  int md = 0;
  for (auto &P : tree->t.probs)
    for (auto &L : P.leaves) md = std::max(md, L.depth);
  info->max_depth = md;
  return HPS_OK;
}

int hps_tree_counts(const hps_tree *tree, int q, int64_t *n_gauss, int64_t *n_bdry) {
  if (!tree || q < 1) return fail(HPS_EINVAL, "bad arguments");
  Plan pl;
  int rc = plan_tree(tree->t, pl, q);
  if (rc) return rc;
  if (n_gauss) *n_gauss = pl.n_gauss;
  if (n_bdry) *n_bdry = (int64_t)pl.bdry.size();
  return HPS_OK;
}

int hps_leaf_cheb_nodes(const hps_tree *tree, int p, double *xy) {
  if (!tree || !xy || p < 2) return fail(HPS_EINVAL, "bad arguments");
  Plan pl;
  int rc = plan_tree(tree->t, pl, 0);
  if (rc) return rc;
  std::vector<double> xc = cheb_points(p);
  size_t o = 0;
  for (int li : pl.leaves) {
    double x0, x1, y0, y1;
    leaf_phys(tree->t, pl.boxes[li], x0, x1, y0, y1);
    for (int iy = 0; iy < p; ++iy)
      for (int ix = 0; ix < p; ++ix) {
        xy[o++] = x0 + (x1 - x0) * (xc[ix] + 1.0) * 0.5;
        xy[o++] = y0 + (y1 - y0) * (xc[iy] + 1.0) * 0.5;
      }
  }
  return HPS_OK;
}

int hps_leaf_boxes(const hps_tree *tree, double *boxes) {
  if (!tree || !boxes) return fail(HPS_EINVAL, "bad arguments");
  Plan pl;
  int rc = plan_tree(tree->t, pl, 0);
  if (rc) return rc;
  size_t o = 0;
  for (int li : pl.leaves) {
    double x0, x1, y0, y1;
    leaf_phys(tree->t, pl.boxes[li], x0, x1, y0, y1);
    boxes[o++] = x0; boxes[o++] = x1; boxes[o++] = y0; boxes[o++] = y1;
  }
  return HPS_OK;
}

int hps_bdry_gauss_nodes(const hps_tree *tree, int q, double *xy) {
  if (!tree || !xy || q < 1) return fail(HPS_EINVAL, "bad arguments");
  Plan pl;
  int rc = plan_tree(tree->t, pl, q);
  if (rc) return rc;
  for (size_t i = 0; i < pl.bdry.size(); ++i) {
    xy[2 * i] = pl.node_xy[2 * pl.bdry[i]];
    xy[2 * i + 1] = pl.node_xy[2 * pl.bdry[i] + 1];
  }
  return HPS_OK;
}

int hps_gauss_nodes(const hps_tree *tree, int q, double *xy) {
  if (!tree || !xy || q < 1) return fail(HPS_EINVAL, "bad arguments");
  Plan pl;
  int rc = plan_tree(tree->t, pl, q);
  if (rc) return rc;
  std::memcpy(xy, pl.node_xy.data(), pl.node_xy.size() * sizeof(double));
  return HPS_OK;
}

void hps_tree_free(hps_tree *tree) { delete tree; }

}  // extern "C"

// ---------------------------------------------------------------------------
// planning of the device layout and the programs
// ---------------------------------------------------------------------------
namespace {

struct Layout {
  // per box offsets (ws unless noted)
  std::vector<int64_t> T, X, S, LD, H, Pup, Pdn, Pups;   // -1 if absent
  std::vector<int64_t> Tn_scr, Tmp_scr, B_scr, W_scr, ipiv;
  std::vector<int64_t> h, w, hn;                          // vec offsets
  std::vector<int64_t> Ub, Ubn, wb, hb, hbn;              // adjoint vec offsets
  std::vector<int64_t> map_fin, map_nat, map_gi, map_pi, map_slave;  // imap offsets
  std::vector<int64_t> Z0, map_psi;   // Neumann closure: zero sibling T (ws), data positions
  std::vector<int64_t> L_role;                 // ws, per role (5)
  std::vector<int64_t> Mb_role;                // ws, per role: K_t L, t = 1..5 (build only)
  std::vector<int64_t> Dci, T0;                // ws, per (class*5 + role)
  int64_t ws = 0, scr = 0, vec = 0, imap = 0, ipiv_n = 0, solve_ws = 0;
};

// Reference matrices of one leaf class/role, column-major where stored.
struct LeafRef {
  std::vector<double> Dh, Dh2;     // p x p row-major
  std::vector<double> Lnat;        // me x 4q, column-major
  std::vector<int> ice, ici;       // exterior / interior grid indices
};

LeafRef leaf_reference(int p, int q) {
  LeafRef R;
  std::vector<double> xc = cheb_points(p), xg = legendre_roots(q);
  R.Dh = diff_matrix(xc);
  R.Dh2.assign(size_t(p) * p, 0.0);
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < p; ++j) {
      double s = 0.0;
      for (int k = 0; k < p; ++k) s += R.Dh[i * p + k] * R.Dh[k * p + j];
      R.Dh2[i * p + j] = s;
    }
  for (int g = 0; g < p * p; ++g) {
    int iy = g / p, ix = g % p;
    bool in = iy > 0 && iy < p - 1 && ix > 0 && ix < p - 1;
    (in ? R.ici : R.ice).push_back(g);
  }
  std::vector<double> G2C = interp_matrix(xg, xc);   // p x q row-major
  const int me = (int)R.ice.size();
  R.Lnat.assign(size_t(me) * 4 * q, 0.0);
  auto put = [&](int r, int side, int t, double w) {
    for (int k = 0; k < q; ++k) R.Lnat[r + size_t(me) * (side * q + k)] += w * G2C[t * q + k];
  };
  for (int r = 0; r < me; ++r) {
    int g = R.ice[r], iy = g / p, ix = g % p;
    bool cx = ix == 0 || ix == p - 1, cy = iy == 0 || iy == p - 1;
    if (cx && cy) {
      put(r, iy == 0 ? 0 : 2, ix, 0.5);
      put(r, ix == 0 ? 3 : 1, iy, 0.5);
    } else if (iy == 0) put(r, 0, ix, 1.0);
    else if (iy == p - 1) put(r, 2, ix, 1.0);
    else if (ix == 0) put(r, 3, iy, 1.0);
    else put(r, 1, iy, 1.0);
  }
  return R;
}

// The five fixed products M_t = K_t L (each mi x g4, column-major, ld mi;
// stacked t = 1..5) with which leaf_b_kernel forms B = A_ci,ce L: restricted
// to an interior row a = (iy, ix) and an exterior node b = (jy, jx), the
// collocated operator is cxy(a) Dh(iy,jy) Dh(ix,jx) + [iy = jy] (cxx(a)
// Dh2(ix,jx) + cx(a) Dh(ix,jx)) + [ix = jx] (cyy(a) Dh2(iy,jy) + cy(a)
// Dh(iy,jy)) (Sec. 3.3), so K_1..K_5 are those five coefficient-free terms.
std::vector<double> leaf_b_factors(const LeafRef &R, int p, const std::vector<double> &L,
                                   int g4) {
  const int mi = (int)R.ici.size(), me = (int)R.ice.size();
  std::vector<double> M(size_t(5) * mi * g4, 0.0), K(size_t(5) * me);
  for (int a = 0; a < mi; ++a) {
    const int ga = R.ici[a], iy = ga / p, ix = ga % p;
    for (int e = 0; e < me; ++e) {
      const int gb = R.ice[e], jy = gb / p, jx = gb % p;
      K[0 * me + e] = R.Dh[iy * p + jy] * R.Dh[ix * p + jx];
      K[1 * me + e] = iy == jy ? R.Dh2[ix * p + jx] : 0.0;
      K[2 * me + e] = iy == jy ? R.Dh[ix * p + jx] : 0.0;
      K[3 * me + e] = ix == jx ? R.Dh2[iy * p + jy] : 0.0;
      K[4 * me + e] = ix == jx ? R.Dh[iy * p + jy] : 0.0;
    }
    for (int t = 0; t < 5; ++t)
      for (int j = 0; j < g4; ++j) {
        double v = 0.0;
        for (int e = 0; e < me; ++e) v += K[size_t(t) * me + e] * L[e + size_t(j) * me];
        M[size_t(t) * mi * g4 + a + size_t(j) * mi] = v;
      }
  }
  return M;
}

// side order of a leaf with role r: the three kept sides, then the shared one
void role_sides(int role, int so[4]) {
  int k = 0;
  for (int s = 0; s < 4; ++s)
    if (s != role) so[k++] = s;
  if (role < 4) so[3] = role;
}

// D_ge,c of a leaf with sides in role order (4q x p^2, row-major)
std::vector<double> leaf_dge(int p, int q, double hx, double hy, int role) {
  std::vector<double> xc = cheb_points(p), xg = legendre_roots(q);
  std::vector<double> D = diff_matrix(xc), Lloc = interp_matrix(xc, xg);  // q x p
  const double sx = 2.0 / hx, sy = 2.0 / hy;
  std::vector<double> nat(size_t(4) * q * p * p, 0.0);
  for (int k = 0; k < q; ++k)
    for (int jy = 0; jy < p; ++jy)
      for (int jx = 0; jx < p; ++jx) {
        const int c = jy * p + jx;
        nat[size_t(0 * q + k) * p * p + c] = Lloc[k * p + jx] * sy * D[0 * p + jy];
        nat[size_t(1 * q + k) * p * p + c] = Lloc[k * p + jy] * sx * D[(p - 1) * p + jx];
        nat[size_t(2 * q + k) * p * p + c] = Lloc[k * p + jx] * sy * D[(p - 1) * p + jy];
        nat[size_t(3 * q + k) * p * p + c] = Lloc[k * p + jy] * sx * D[0 * p + jx];
      }
  int so[4];
  role_sides(role, so);
  std::vector<double> out(nat.size());
  for (int j = 0; j < 4; ++j)
    std::memcpy(&out[size_t(j) * q * p * p], &nat[size_t(so[j]) * q * p * p],
                sizeof(double) * q * p * p);
  return out;
}

void gemm_step(GemmList &gl, GemmList &tmp, std::vector<Step> &prog) {
  if (tmp.d.empty()) return;
  Step s{S_GEMM};
  s.d0 = (int64_t)gl.d.size();
  s.nd = (int64_t)tmp.d.size();
  s.ntiles = tmp.tiles;
  s.tmap0 = (int64_t)gl.tmap.size();
  for (auto &g : tmp.d) gl.d.push_back(g);
  gl.tmap.insert(gl.tmap.end(), tmp.tmap.begin(), tmp.tmap.end());   // relative to d0
  prog.push_back(s);
}

// Launch steps that invert the interface blocks of one level: the
// register-resident kernel per size class, the blocked path above it.
void emit_inverse_steps(const std::vector<MergeInvDesc> &lev, std::vector<MergeInvDesc> &minv,
                        std::vector<Step> &prog) {
  std::vector<MergeInvDesc> cls_d[4], big;
  int bigmax = 0;
  for (const MergeInvDesc &d : lev) {
    int cls = gj_merge_class(d.m);
    if (cls >= 0) cls_d[cls].push_back(d);
    else { big.push_back(d); bigmax = std::max(bigmax, d.m); }
  }
  for (int c = 0; c < 4; ++c) {
    if (cls_d[c].empty()) continue;
    Step s{S_GJ_MERGE};
    s.cls = c;
    s.d0 = (int64_t)minv.size();
    s.nd = (int64_t)cls_d[c].size();
    minv.insert(minv.end(), cls_d[c].begin(), cls_d[c].end());
    prog.push_back(s);
  }
  if (big.empty()) return;
  const int NBp = panel_nb(bigmax);
  const int64_t d0 = (int64_t)minv.size();
  minv.insert(minv.end(), big.begin(), big.end());
  Step z{S_ZDIFF};
  z.d0 = d0; z.nd = (int64_t)big.size(); z.maxm = bigmax;
  prog.push_back(z);
  if (gj_level_fits(bigmax, (int)big.size())) {
    // one launch for the level, strips resident
    Step s{S_PANEL};
    s.d0 = d0; s.nd = (int64_t)big.size(); s.kb = kPanelLevel; s.maxm = bigmax;
    s.cls = gj_level_force_retire() ? 1 : 0;
    prog.push_back(s);
  } else
  // launch kb applies panel kb's update to the other columns and sweeps
  // panel kb + NB (kb = -NB: only the sweep of panel 0)
  for (int kb = -NBp; kb < bigmax; kb += NBp) {
    Step s{S_PANEL};
    s.d0 = d0; s.nd = (int64_t)big.size(); s.kb = kb; s.maxm = bigmax;
    prog.push_back(s);
  }
  Step cp{S_COLPERM};
  cp.d0 = d0; cp.nd = (int64_t)big.size(); cp.maxm = bigmax;
  prog.push_back(cp);
}

}  // namespace

// State shared by the planning stages of one handle.
struct PlanCtx {
  hps_handle *H;
  Layout &Lo;
  std::vector<double> &ws_init;
  std::vector<std::pair<int64_t, std::vector<double>>> &ws_blocks;
  std::vector<int32_t> &imap;
  GemmList &gl;
  std::vector<LeafDesc> &leafd;
  std::vector<MergeInvDesc> &minv;
  std::vector<ApplyDesc> &appl;
  std::vector<int32_t> &appl_tmap;
  std::vector<int32_t> &finlist;
  std::vector<VecOpDesc> &vops;
  std::vector<int> rep;     // the box whose operators a box shares (itself unless deduplicated)
  int64_t f_scr = -1;       // economic build: scratch of one chunk's F
  bool own(int b) const { return rep[size_t(b)] == b; }
  int64_t imap_put(const std::vector<int32_t> &v) {
    const int64_t o = (int64_t)imap.size();
    imap.insert(imap.end(), v.begin(), v.end());
    return o;
  }
  Ref f_ref(int i) const {   // where leaf i's F lives
    const int mi = H->mi;
    if (H->econ) return ref(BUF_SCR, f_scr + int64_t(i % H->econ_chunk) * mi * mi, mi);
    return ref(BUF_WS, Lo.LD[H->pl.leaves[i]] + int64_t(H->g4) * mi, mi);
  }
};

// Stage 1: operator and scratch layout, reference matrices, integer maps.
static int plan_layout(PlanCtx &C) {
  hps_handle *H = C.H;
  Layout &Lo = C.Lo;
  Plan &pl = H->pl;
  const int p = H->p, q = H->q, mi = H->mi, me = H->me, g4 = H->g4;
  const int nb = (int)pl.boxes.size();
  const int nleaf = H->nleaf;
  (void)p; (void)q; (void)mi; (void)me; (void)g4; (void)nb; (void)nleaf;
  auto &ws_init = C.ws_init;
  auto &ws_blocks = C.ws_blocks;
  Lo.T.assign(nb, -1); Lo.X.assign(nb, -1); Lo.S.assign(nb, -1); Lo.LD.assign(nb, -1);
  Lo.H.assign(nb, -1); Lo.Pup.assign(nb, -1); Lo.Pdn.assign(nb, -1); Lo.Pups.assign(nb, -1);
  Lo.Tn_scr.assign(nb, -1); Lo.Tmp_scr.assign(nb, -1);
  Lo.B_scr.assign(nb, -1); Lo.W_scr.assign(nb, -1); Lo.ipiv.assign(nb, -1);
  Lo.h.assign(nb, -1); Lo.w.assign(nb, -1); Lo.hn.assign(nb, -1);
  Lo.Ub.assign(nb, -1); Lo.Ubn.assign(nb, -1); Lo.wb.assign(nb, -1); Lo.hb.assign(nb, -1);
  Lo.hbn.assign(nb, -1);
  Lo.map_fin.assign(nb, -1); Lo.map_nat.assign(nb, -1); Lo.map_gi.assign(nb, -1);
  Lo.map_pi.assign(nb, -1); Lo.map_slave.assign(nb, -1);
  auto ws_take = [&](int64_t n) { int64_t o = Lo.ws; Lo.ws += (n + 31) / 32 * 32; return o; };
  auto scr_take = [&](int64_t n) { int64_t o = Lo.scr; Lo.scr += (n + 31) / 32 * 32; return o; };
  auto vec_take = [&](int64_t n) { int64_t o = Lo.vec; Lo.vec += n; return o; };
  auto imap_put = [&](const std::vector<int32_t> &v) { return C.imap_put(v); };
  auto imap_put64 = [&](const std::vector<int64_t> &v) {
    std::vector<int32_t> w(v.begin(), v.end());
    return imap_put(w);
  };
  // Translation-invariant operators (constant coefficients, the remark after
  // the timings of Sec. 7.1): boxes with the same key -- a leaf's size class
  // and role, a merge's children's keys, cut, role and final order -- have
  // identical operators, stored once at the key's first box (rep).
  std::vector<int> &rep = C.rep;
  rep.assign(nb, 0);
  for (int b = 0; b < nb; ++b) rep[b] = b;
  if (H->dedup) {
    std::map<std::vector<int64_t>, int> first;
    std::vector<int64_t> kid(nb, -1);
    for (int b = nb - 1; b >= 0; --b) {       // children come after their parent
      const Box &B = pl.boxes[b];
      std::vector<int64_t> k;
      if (B.leaf) {
        k = {0, pl.leaf_class[B.leaf_index], B.role};
      } else if (B.kind == 3) {        // Neumann closure: its root and its size
        k = {3, kid[B.alpha], (int64_t)B.gi.size()};
      } else {
        k = {1, kid[B.alpha], kid[B.beta], B.cut, B.role, B.n_shared, (int64_t)B.gi.size()};
        k.insert(k.end(), B.pi.begin(), B.pi.end());
      }
      auto it = first.find(k);
      if (it == first.end()) {
        kid[b] = (int64_t)first.size();
        first.emplace(k, b);
      } else {
        kid[b] = kid[it->second];
        rep[b] = it->second;
      }
    }
  }
  auto own = [&](int b) { return C.own(b); };
  // --- solve-stage operators first (they are the FP32-copied prefix) ---
  Lo.vec = pl.n_gauss;   // global u at the start of each RHS block
  H->ug_off = 0;
  for (int li : pl.leaves) {
    if (!own(li)) continue;
    // [S_ci | F]; the economic build keeps S_ci only
    Lo.LD[li] = ws_take(int64_t(mi) * (g4 + (H->econ ? 0 : mi)));
    Lo.H[li] = ws_take(int64_t(g4) * mi);
  }
  for (int b = 0; b < nb; ++b) {
    const Box &B = pl.boxes[b];
    const int ef = (int)B.fin.size();
    if (!own(b)) continue;
    if (B.parent >= 0) Lo.T[b] = ws_take(int64_t(ef) * ef);
    if (!B.leaf) {
      const int m = (int)B.gi.size(), en = (int)B.nat.size();
      Lo.X[b] = ws_take(int64_t(m) * m);
      Lo.S[b] = ws_take(int64_t(m) * en);
      if (B.coarsened) {
        Lo.Pdn[b] = ws_take(int64_t(ef) * en);
        Lo.Pups[b] = ws_take(int64_t(B.slave_rows.size()) * ef);
        Lo.Pup[b] = ws_take(int64_t(en) * ef);
      }
    }
  }
  for (int b = 0; b < nb; ++b)
    if (!own(b)) {
      const int r = rep[b];
      Lo.LD[b] = Lo.LD[r]; Lo.H[b] = Lo.H[r]; Lo.T[b] = Lo.T[r];
      Lo.X[b] = Lo.X[r]; Lo.S[b] = Lo.S[r];
    }
  // reference matrices per role / size class
  LeafRef R = leaf_reference(p, q);
  Lo.L_role.assign(5, -1);
  std::vector<std::vector<double>> role_L(5);
  for (int r = 0; r < 5; ++r) {
    int so[4];
    role_sides(r, so);
    std::vector<double> &L = role_L[r];
    L.assign(size_t(me) * g4, 0.0);
    for (int j = 0; j < 4; ++j)
      std::memcpy(&L[size_t(me) * j * q], &R.Lnat[size_t(me) * so[j] * q],
                  sizeof(double) * me * q);
    Lo.L_role[r] = ws_take(int64_t(me) * g4);
    ws_blocks.push_back({Lo.L_role[r], L});
  }
  Lo.solve_ws = Lo.ws;
  // the five fixed products K_t L of each role for B = A_ci,ce L (build only)
  Lo.Mb_role.assign(5, -1);
  for (int r = 0; r < 5; ++r) {
    Lo.Mb_role[r] = ws_take(5 * int64_t(mi) * g4);
    ws_blocks.push_back({Lo.Mb_role[r], leaf_b_factors(R, p, role_L[r], g4)});
  }
  // Neumann closure boxes merge with a sibling whose T is zero
  Lo.Z0.assign(nb, -1);
  for (int b = 0; b < nb; ++b)
    if (pl.boxes[b].kind == 3) {
      const int64_t m = (int64_t)pl.boxes[b].gi.size();
      Lo.Z0[b] = ws_take(m * m);
      ws_blocks.push_back({Lo.Z0[b], std::vector<double>(size_t(m * m), 0.0)});
    }
  const int ncls = (int)pl.size_class.size();
  Lo.Dci.assign(size_t(ncls) * 5, -1);
  Lo.T0.assign(size_t(ncls) * 5, -1);
  std::vector<char> need(size_t(ncls) * 5, 0);
  for (int i = 0; i < nleaf; ++i) need[size_t(pl.leaf_class[i]) * 5 + pl.boxes[pl.leaves[i]].role] = 1;
  for (int c = 0; c < ncls; ++c)
    for (int r = 0; r < 5; ++r) {
      if (!need[size_t(c) * 5 + r]) continue;
      std::vector<double> Dg = leaf_dge(p, q, pl.size_class[c].first, pl.size_class[c].second, r);
      std::vector<double> Dci(size_t(g4) * mi), T0(size_t(g4) * g4, 0.0);
      for (int a = 0; a < mi; ++a)
        for (int k = 0; k < g4; ++k) Dci[k + size_t(g4) * a] = Dg[size_t(k) * p * p + R.ici[a]];
      // T0 = D_ge,ce L (role order)
      int so[4];
      role_sides(r, so);
      for (int k = 0; k < g4; ++k)
        for (int j = 0; j < g4; ++j) {
          const int js = so[j / q] * q + j % q;   // natural column of L
          double s = 0.0;
          for (int e = 0; e < me; ++e)
            s += Dg[size_t(k) * p * p + R.ice[e]] * R.Lnat[e + size_t(me) * js];
          T0[k + size_t(g4) * j] = s;
        }
      Lo.Dci[size_t(c) * 5 + r] = ws_take(int64_t(g4) * mi);
      Lo.T0[size_t(c) * 5 + r] = ws_take(int64_t(g4) * g4);
      ws_blocks.push_back({Lo.Dci[size_t(c) * 5 + r], Dci});
      ws_blocks.push_back({Lo.T0[size_t(c) * 5 + r], T0});
    }
  // P_up / P_down of coarsened boxes
  for (int b = 0; b < nb; ++b) {
    const Box &B = pl.boxes[b];
    if (!B.coarsened) continue;
    const int ef = (int)B.fin.size(), en = (int)B.nat.size();
    ws_blocks.push_back({Lo.Pup[b], B.Pup});
    ws_blocks.push_back({Lo.Pdn[b], B.Pdn});
    std::vector<double> Ps(size_t(B.slave_rows.size()) * ef);
    const int ns = (int)B.slave_rows.size();
    for (int j = 0; j < ef; ++j)
      for (int a = 0; a < ns; ++a) Ps[a + size_t(ns) * j] = B.Pup[B.slave_rows[a] + size_t(en) * j];
    ws_blocks.push_back({Lo.Pups[b], Ps});
  }
  // leaf temporaries and T
  for (int i = 0; i < nleaf; ++i) {
    const int li = pl.leaves[i];
    if (!own(li)) continue;
    if (Lo.T[li] < 0) Lo.T[li] = ws_take(int64_t(g4) * g4);   // single-leaf root
    Lo.B_scr[li] = scr_take(int64_t(mi) * g4);
  }
  for (int li : pl.leaves)
    if (!own(li)) Lo.T[li] = Lo.T[rep[li]];
  // economic build: F of one chunk of leaves at a time (build and solve)
  H->econ_chunk = H->econ ? std::min(nleaf, kEconChunk) : nleaf;
  C.f_scr = H->econ ? scr_take(int64_t(H->econ_chunk) * mi * mi) : -1;
  for (int b = 0; b < nb; ++b) {
    const Box &B = pl.boxes[b];
    if (B.leaf || !own(b)) continue;
    const int m = (int)B.gi.size(), en = (int)B.nat.size(), ef = (int)B.fin.size();
    if (gj_merge_class(m) < 0) {
      Lo.W_scr[b] = scr_take(std::max<int64_t>(int64_t(kPanelNBMax) * m, int64_t(m) * m));
      Lo.ipiv[b] = Lo.ipiv_n;          // pivrow[m], stepof[m], level control
      Lo.ipiv_n += gj_int_scratch(m);
    }
    if (B.coarsened && B.parent >= 0) {
      Lo.Tn_scr[b] = scr_take(int64_t(en) * en);
      Lo.Tmp_scr[b] = scr_take(int64_t(en) * ef);
    }
  }
  // --- vectors (per RHS) ---
  for (int b = 0; b < nb; ++b) {
    const Box &B = pl.boxes[b];
    Lo.h[b] = vec_take((int64_t)B.fin.size());
    if (!B.leaf) {
      Lo.w[b] = vec_take((int64_t)B.gi.size());
      if (B.coarsened) Lo.hn[b] = vec_take((int64_t)B.nat.size());
    }
  }
  for (int b = 0; b < nb; ++b) {      // adjoint sweeps
    const Box &B = pl.boxes[b];
    Lo.Ub[b] = vec_take((int64_t)B.fin.size());
    Lo.hb[b] = vec_take((int64_t)B.fin.size());
    if (!B.leaf) {
      Lo.wb[b] = vec_take((int64_t)B.gi.size());
      if (B.coarsened) {
        Lo.Ubn[b] = vec_take((int64_t)B.nat.size());
        Lo.hbn[b] = vec_take((int64_t)B.nat.size());
      }
    }
  }
  // --- integer maps ---
  for (int b = 0; b < nb; ++b) {
    const Box &B = pl.boxes[b];
    Lo.map_fin[b] = imap_put64(B.fin);
    if (!B.leaf) {
      Lo.map_nat[b] = imap_put64(B.nat);
      Lo.map_gi[b] = imap_put64(B.gi);
      if (!B.coarsened) {
        std::vector<int32_t> pi(B.pi.begin(), B.pi.end());
        Lo.map_pi[b] = imap_put(pi);
      } else {
        std::vector<int32_t> sl;
        for (int a : B.slave_rows) sl.push_back((int32_t)B.nat[a]);
        Lo.map_slave[b] = imap_put(sl);
      }
    }
  }
  {
    std::vector<int32_t> v(R.ice.begin(), R.ice.end());
    H->ice_map = imap_put(v);
    std::vector<int32_t> w(R.ici.begin(), R.ici.end());
    H->ici_map = imap_put(w);
    H->map_bdry = imap_put64(pl.bdry);
    H->n_bdry = (int64_t)pl.bdry.size();
    // position of each Neumann node's data in the boundary vector
    std::unordered_map<int64_t, int32_t> npos;
    for (size_t k = 0; k < pl.bdry.size(); ++k)
      if (pl.bdry_kind[k] == kBcNeumann) npos[pl.bdry[k]] = (int32_t)k;
    Lo.map_psi.assign(nb, -1);
    for (int b = 0; b < nb; ++b) {
      const Box &B = pl.boxes[b];
      if (B.kind != 3) continue;
      std::vector<int32_t> v;
      for (int64_t j : B.gi) {
        auto it = npos.find(j);
        if (it == npos.end()) return fail(HPS_ETREE, "closure node without Neumann data");
        v.push_back(it->second);
      }
      Lo.map_psi[b] = imap_put(v);
    }
  }
  // aux: Dh, Dh2
  ws_init.clear();
  ws_init.insert(ws_init.end(), R.Dh.begin(), R.Dh.end());
  ws_init.insert(ws_init.end(), R.Dh2.begin(), R.Dh2.end());
  H->Dh_off = 0;
  H->Dh2_off = int64_t(p) * p;

  return HPS_OK;
}

// Stage 2: the build program (Algorithm 1): leaf Gauss-Jordan and products,
// then the merges level by level.
static int plan_build_program(PlanCtx &C) {
  hps_handle *H = C.H;
  Layout &Lo = C.Lo;
  Plan &pl = H->pl;
  const int p = H->p, q = H->q, mi = H->mi, me = H->me, g4 = H->g4;
  const int nb = (int)pl.boxes.size();
  const int nleaf = H->nleaf;
  (void)p; (void)q; (void)mi; (void)me; (void)g4; (void)nb; (void)nleaf;
  auto &gl = C.gl;
  auto &leafd = C.leafd;
  auto &minv = C.minv;
  auto own = [&](int b) { return C.own(b); };
  auto f_ref = [&](int i) { return C.f_ref(i); };
  auto &prog = H->build_prog;
  prog.clear();
  // leaves: Gauss-Jordan, then the leaf products, one chunk of leaves at a
  // time (a single chunk unless the build is economic)
  for (int i = 0; i < nleaf; ++i) {
    const int li = pl.leaves[i];
    const auto &sc = pl.size_class[pl.leaf_class[i]];
    LeafDesc d{};
    d.coef = int64_t(i) * 6 * p * p;
    const Ref fr = f_ref(i);
    d.F = fr.off;
    d.fbuf = fr.buf;
    d.sx = 2.0 / sc.first;
    d.sy = 2.0 / sc.second;
    d.info = i;
    // the p = 16 leaf kernel forms H itself (its padding rows hold D_ge,ci)
    d.hrows = leaf_kernel_forms_h(p, g4) ? g4 : 0;
    d.Dci = Lo.Dci[size_t(pl.leaf_class[i]) * 5 + pl.boxes[li].role];
    d.H = Lo.H[li];
    d.Bout = Lo.B_scr[li];
    d.Mb = Lo.Mb_role[pl.boxes[li].role];
    leafd.push_back(d);
  }
  // the leaves whose operators the build computes (all but deduplicated
  // ones); their descriptors follow the per-leaf list when that is a subset
  std::vector<int> bl;
  for (int i = 0; i < nleaf; ++i)
    if (own(pl.leaves[i])) bl.push_back(i);
  const int nbl = (int)bl.size();
  int64_t bl0 = 0;
  if (nbl < nleaf) {
    bl0 = (int64_t)leafd.size();
    for (int i : bl) leafd.push_back(leafd[i]);
  }
  for (int c0 = 0; c0 < nbl; c0 += H->econ_chunk) {
    const int c1 = std::min(nbl, c0 + H->econ_chunk);
    Step s{S_GJ_LEAF};
    s.d0 = bl0 + c0;
    s.nd = c1 - c0;
    prog.push_back(s);
    {
      // B = A_ci,ce L: the step's leaves grouped by role in chunks of up to
      // kLeafBChunk; imap holds the leaf descriptor indices (lidx) and the
      // chunks' [first, count] pairs
      std::vector<int32_t> lidx, chunks;
      for (int r = 0; r < 5; ++r) {
        int n = 0;
        for (int ci = c0; ci < c1; ++ci) {
          if (pl.boxes[pl.leaves[bl[ci]]].role != r) continue;
          if (n % kLeafBChunk == 0) { chunks.push_back((int32_t)lidx.size()); chunks.push_back(0); }
          lidx.push_back(int32_t(bl0 + ci));
          ++chunks.back();
          ++n;
        }
      }
      Step sb{S_LEAF_B};
      sb.d0 = C.imap_put(lidx);
      sb.tmap0 = C.imap_put(chunks);
      sb.nd = c1 - c0;
      sb.ntiles = (int64_t)chunks.size() / 2;
      prog.push_back(sb);
    }
    GemmList a, b2, c;
    for (int ci = c0; ci < c1; ++ci) {
      const int i = bl[ci];
      const int li = pl.leaves[i];
      const int role = pl.boxes[li].role, cls = pl.leaf_class[i];
      const Ref F = f_ref(i);
      const int64_t Dci = Lo.Dci[size_t(cls) * 5 + role], T0 = Lo.T0[size_t(cls) * 5 + role];
      GemmDesc g{};
      // H = D_ge,ci F (unless the leaf kernel formed it)
      if (!leaf_kernel_forms_h(p, g4)) {
        g = GemmDesc{};
        g.M = g4; g.N = mi; g.K = mi;
        g.A = ref(BUF_WS, Dci, g4); g.B = F;
        g.C = ref(BUF_WS, Lo.H[li], g4); g.D = noref();
        g.crow = g.ccol = -1; g.alpha = 1.0; g.beta = 0.0;
        a.add(g);
      }
      // S_ci = -F B
      g = GemmDesc{};
      g.M = mi; g.N = g4; g.K = mi;
      g.A = F; g.B = ref(BUF_SCR, Lo.B_scr[li], mi);
      g.C = ref(BUF_WS, Lo.LD[li], mi); g.D = noref();
      g.crow = g.ccol = -1; g.alpha = -1.0; g.beta = 0.0;
      b2.add(g);
      // T = T0 + D_ge,ci S_ci
      g = GemmDesc{};
      g.M = g4; g.N = g4; g.K = mi;
      g.A = ref(BUF_WS, Dci, g4); g.B = ref(BUF_WS, Lo.LD[li], mi);
      g.C = ref(BUF_WS, Lo.T[li], g4); g.D = ref(BUF_WS, T0, g4);
      g.crow = g.ccol = -1; g.alpha = 1.0; g.beta = 1.0;
      c.add(g);
    }
    gemm_step(gl, a, prog);
    gemm_step(gl, b2, prog);
    gemm_step(gl, c, prog);
  }
  // merges, level by level
  int info_slot = nleaf;
  for (int h = 1; h <= pl.max_height; ++h) {
    std::vector<int> lev;
    for (int b = 0; b < nb; ++b)
      if (!pl.boxes[b].leaf && pl.boxes[b].height == h && own(b)) lev.push_back(b);
    if (lev.empty()) continue;
    std::vector<MergeInvDesc> levd;
    for (int b : lev) {
      const Box &B = pl.boxes[b];
      const Box &A = pl.boxes[B.alpha];
      const int m = (int)B.gi.size();
      const int ea = (int)A.fin.size();
      const int n1 = ea - m;
      MergeInvDesc d{};
      d.Ta = Lo.T[B.alpha] + n1 + int64_t(n1) * ea;
      d.lda = ea; d.m = m; d.info = info_slot++;
      if (B.kind == 3) {               // closure: the sibling's T is zero
        d.Tb = Lo.Z0[b];
        d.ldb = m;
      } else {
        const Box &C = pl.boxes[B.beta];
        const int eb = (int)C.fin.size(), n2 = eb - m;
        d.Tb = Lo.T[B.beta] + n2 + int64_t(n2) * eb;
        d.ldb = eb;
      }
      d.X = Lo.X[b];
      d.W = Lo.W_scr[b];
      d.ipiv = Lo.ipiv[b];
      levd.push_back(d);
    }
    emit_inverse_steps(levd, minv, prog);
    // S = X [-T31a | T32b]
    GemmList sg, tg, c1, c2;
    for (int b : lev) {
      const Box &B = pl.boxes[b];
      const Box &A = pl.boxes[B.alpha];
      const int m = (int)B.gi.size();
      const int ea = (int)A.fin.size();
      const int n1 = ea - m;
      GemmDesc g{};
      g.M = m; g.N = n1; g.K = m;
      g.A = ref(BUF_WS, Lo.X[b], m); g.B = ref(BUF_WS, Lo.T[B.alpha] + n1, ea);
      g.C = ref(BUF_WS, Lo.S[b], m); g.D = noref(); g.crow = g.ccol = -1;
      g.alpha = -1.0; g.beta = 0.0;
      if (n1 > 0) sg.add(g);
      if (B.kind == 3) continue;      // closure: S = -X T31a only, no T above
      const Box &C = pl.boxes[B.beta];
      const int eb = (int)C.fin.size();
      const int n2 = eb - m, en = n1 + n2, ef = (int)B.fin.size();
      g = GemmDesc{};
      g.M = m; g.N = n2; g.K = m;
      g.A = ref(BUF_WS, Lo.X[b], m); g.B = ref(BUF_WS, Lo.T[B.beta] + n2, eb);
      g.C = ref(BUF_WS, Lo.S[b] + int64_t(n1) * m, m); g.D = noref(); g.crow = g.ccol = -1;
      g.alpha = 1.0; g.beta = 0.0;
      sg.add(g);
      if (B.parent < 0) continue;   // the root's T is never used
      // T = blkdiag(T11a, T22b) + [T13a; T23b] S, written in final order
      Ref Cout;
      int64_t pr = -1;
      if (B.coarsened) Cout = ref(BUF_SCR, Lo.Tn_scr[b], en);
      else { Cout = ref(BUF_WS, Lo.T[b], ef); pr = Lo.map_pi[b]; }
      const int64_t Ta = Lo.T[B.alpha], Tb = Lo.T[B.beta];
      // one product: rows 0..n1-1 of [T13a; T23b] from T_alpha, the rest
      // from T_beta, and the block-diagonal part from both
      GemmDesc t{};
      t.M = en; t.N = en; t.K = m;
      const Ref a1 = ref(BUF_WS, Ta + int64_t(n1) * ea, ea), a2 = ref(BUF_WS, Tb + int64_t(n2) * eb, eb);
      const Ref d1 = ref(BUF_WS, Ta, ea), d2 = ref(BUF_WS, Tb, eb);
      if (n1 == 0) { t.A = a2; t.D = d2; }
      else if (n2 == 0) { t.A = a1; t.D = d1; }
      else { t.A = a1; t.D = d1; t.A2 = a2; t.D2 = d2; t.msplit = n1; }
      t.B = ref(BUF_WS, Lo.S[b], m);
      t.alpha = 1.0; t.beta = 1.0;
      if (pr >= 0) {
        t.C = Cout; t.crow = pr; t.ccol = pr;
      } else {
        t.C = ref(Cout.buf, Cout.off, en);
        t.crow = t.ccol = -1;
      }
      tg.add(t);
      if (B.coarsened) {
        GemmDesc u{};
        u.M = en; u.N = ef; u.K = en;
        u.A = ref(BUF_SCR, Lo.Tn_scr[b], en); u.B = ref(BUF_WS, Lo.Pup[b], en);
        u.C = ref(BUF_SCR, Lo.Tmp_scr[b], en); u.D = noref(); u.crow = u.ccol = -1;
        u.alpha = 1.0; u.beta = 0.0;
        c1.add(u);
        GemmDesc v{};
        v.M = ef; v.N = ef; v.K = en;
        v.A = ref(BUF_WS, Lo.Pdn[b], ef); v.B = ref(BUF_SCR, Lo.Tmp_scr[b], en);
        v.C = ref(BUF_WS, Lo.T[b], ef); v.D = noref(); v.crow = v.ccol = -1;
        v.alpha = 1.0; v.beta = 0.0;
        c2.add(v);
      }
    }
    gemm_step(gl, sg, prog);
    gemm_step(gl, tg, prog);
    gemm_step(gl, c1, prog);
    gemm_step(gl, c2, prog);
  }
  H->n_info = info_slot;

  return HPS_OK;
}

// Stage 3: the solve programs (Algorithm 2 and its extensions): upward and
// downward passes, the refinement-correction and adjoint variants.
static int plan_solve_programs(PlanCtx &C) {
  hps_handle *H = C.H;
  Layout &Lo = C.Lo;
  Plan &pl = H->pl;
  const int p = H->p, q = H->q, mi = H->mi, me = H->me, g4 = H->g4;
  const int nb = (int)pl.boxes.size();
  const int nleaf = H->nleaf;
  (void)p; (void)q; (void)mi; (void)me; (void)g4; (void)nb; (void)nleaf;
  auto &leafd = C.leafd;
  auto &appl = C.appl;
  auto &appl_tmap = C.appl_tmap;
  auto &finlist = C.finlist;
  auto &vops = C.vops;
  auto imap_put = [&](const std::vector<int32_t> &v) { return C.imap_put(v); };
  auto f_ref = [&](int i) { return C.f_ref(i); };
  H->vec_per_rhs = Lo.vec;
  const int64_t gstride = int64_t(nleaf) * mi, ustride = int64_t(nleaf) * p * p;
  int64_t part_off = 0;
  auto apply_step = [&](std::vector<ApplyDesc> &tmp, std::vector<Step> &prg) {
    if (tmp.empty()) return;
    Step s{S_APPLY};
    s.d0 = (int64_t)appl.size();
    s.nd = (int64_t)tmp.size();
    s.tmap0 = (int64_t)appl_tmap.size();
    int64_t tiles = 0;
    s.fin0 = (int64_t)finlist.size();
    // k-slices: at most 512 k per tile, and enough tiles in the launch to
    // fill the chip (about 1024 workgroups), with at least 64 k per slice
    int64_t sum_rb = 0;
    for (auto &a : tmp) sum_rb += (a.M + 63) / 64;
    const int want = int(std::max<int64_t>(1, (1024 + sum_rb - 1) / std::max<int64_t>(1, sum_rb)));
    for (auto &a : tmp) {
      const int K = a.K1 + (a.mode == 0 ? a.K2 : 0);
      a.rb = (a.M + 63) / 64;
      a.ksl = std::max(1, std::min(64, (K + 511) / 512));
      a.ksl = std::max(a.ksl, std::min(want, std::max(1, K / 64)));
      a.ksl = std::min(a.ksl, 64);
      if (a.abuf == BUF_SCR) a.ksl = 1;   // split-K partials live in BUF_SCR too
      a.tile0 = tiles;
      tiles += int64_t(a.rb) * a.ksl;
      appl_tmap.insert(appl_tmap.end(), size_t(int64_t(a.rb) * a.ksl),
                       int32_t(appl.size() - s.d0));
      if (a.ksl > 1) {
        a.part = part_off;
        part_off += int64_t(a.ksl) * a.M;
        finlist.push_back((int32_t)appl.size());
        s.fin_maxm = std::max<int64_t>(s.fin_maxm, a.M);
      }
      appl.push_back(a);
    }
    s.ntiles = tiles;
    s.nfin = (int64_t)finlist.size() - s.fin0;
    prg.push_back(s);
    tmp.clear();
  };
  auto ad = [&](int M, int K1, int K2, int mode, int64_t aoff, int lda) {
    ApplyDesc a{};
    a.M = M; a.K1 = K1; a.K2 = K2; a.mode = mode;
    a.abuf = BUF_WS; a.aoff = aoff; a.lda = lda;
    a.B1 = novref(); a.B2 = novref(); a.B3 = novref(); a.C = novref(); a.D = novref();
    a.alpha = 1.0; a.beta = 0.0;
    return a;
  };
  auto vecop_step = [&](std::vector<VecOpDesc> &tmp, std::vector<Step> &prg) {
    if (tmp.empty()) return;
    Step s{S_VECOP};
    s.d0 = (int64_t)vops.size();
    s.nd = (int64_t)tmp.size();
    for (auto &v : tmp) s.maxm = std::max(s.maxm, v.n);
    vops.insert(vops.end(), tmp.begin(), tmp.end());
    prg.push_back(s);
    tmp.clear();
  };
  auto vop = [&](int n, VRef dst, VRef a, double ca, VRef b, double cb) {
    VecOpDesc v{};
    v.n = n; v.dst = dst; v.a = a; v.b = b; v.ca = ca; v.cb = cb;
    return v;
  };
  // up pass
  {
    auto &up = H->up_prog;
    up.clear();
    std::vector<ApplyDesc> tmp;
    for (int i = 0; i < nleaf; ++i) {
      const int li = pl.leaves[i];
      ApplyDesc a = ad(g4, mi, 0, 0, Lo.H[li], g4);
      a.B1 = vref(BUF_IN1, int64_t(i) * mi, -1, gstride);
      a.C = vref(BUF_VEC, Lo.h[li], -1, kInterleaved);
      tmp.push_back(a);
    }
    apply_step(tmp, up);
    for (int h = 1; h <= pl.max_height; ++h) {
      std::vector<int> lev;
      for (int b = 0; b < nb; ++b)
        if (!pl.boxes[b].leaf && pl.boxes[b].height == h) lev.push_back(b);
      if (lev.empty()) continue;
      std::vector<ApplyDesc> wst, hst, cst;
      for (int b : lev) {
        const Box &B = pl.boxes[b];
        const Box &A = pl.boxes[B.alpha];
        const int m = (int)B.gi.size();
        if (B.kind == 3) {
          // Neumann closure: w = X (psi - h3a), psi read from the boundary data
          const int n1 = (int)A.fin.size() - m;
          ApplyDesc a = ad(m, m, 0, 1, Lo.X[b], m);
          a.B1 = vref(BUF_IN0, 0, Lo.map_psi[b], H->n_bdry);
          a.B2 = vref(BUF_VEC, Lo.h[B.alpha] + n1, -1, kInterleaved);
          a.B3 = vref(BUF_AUX, 0, Lo.map_gi[b], kInterleaved);  // Neumann-row residual
          a.B3.buf = -1;                                          // off unless enabled
          a.C = vref(BUF_VEC, Lo.w[b], -1, kInterleaved);
          wst.push_back(a);
          continue;
        }
        const Box &C = pl.boxes[B.beta];
        const int ea = (int)A.fin.size(), eb = (int)C.fin.size();
        const int n1 = ea - m, n2 = eb - m, en = n1 + n2, ef = (int)B.fin.size();
        ApplyDesc a = ad(m, m, 0, 1, Lo.X[b], m);
        a.B1 = vref(BUF_VEC, Lo.h[B.beta] + n2, -1, kInterleaved);
        a.B2 = vref(BUF_VEC, Lo.h[B.alpha] + n1, -1, kInterleaved);
        a.B3 = vref(BUF_AUX, 0, Lo.map_gi[b], kInterleaved);  // flux-jump source
        a.B3.buf = -1;                                          // off unless enabled
        a.C = vref(BUF_VEC, Lo.w[b], -1, kInterleaved);
        wst.push_back(a);
        if (B.parent < 0) continue;
        for (int part = 0; part < 2; ++part) {
          const int M = part == 0 ? n1 : n2;
          if (M == 0) continue;
          const int64_t Tsrc = part == 0 ? Lo.T[B.alpha] + int64_t(n1) * ea
                                         : Lo.T[B.beta] + int64_t(n2) * eb;
          ApplyDesc c = ad(M, m, 0, 0, Tsrc, part == 0 ? ea : eb);
          c.B1 = vref(BUF_VEC, Lo.w[b], -1, kInterleaved);
          c.D = vref(BUF_VEC, part == 0 ? Lo.h[B.alpha] : Lo.h[B.beta], -1, kInterleaved);
          c.beta = 1.0;
          if (B.coarsened) c.C = vref(BUF_VEC, Lo.hn[b] + (part == 0 ? 0 : n1), -1, kInterleaved);
          else c.C = vref(BUF_VEC, Lo.h[b], Lo.map_pi[b] + (part == 0 ? 0 : n1), kInterleaved);
          hst.push_back(c);
        }
        if (B.coarsened) {
          ApplyDesc c = ad(ef, en, 0, 0, Lo.Pdn[b], ef);
          c.B1 = vref(BUF_VEC, Lo.hn[b], -1, kInterleaved);
          c.C = vref(BUF_VEC, Lo.h[b], -1, kInterleaved);
          cst.push_back(c);
        }
      }
      apply_step(wst, up);
      apply_step(hst, up);
      apply_step(cst, up);
    }
  }
  // down pass
  {
    auto &dn = H->down_prog;
    dn.clear();
    std::vector<ApplyDesc> tmp;
    for (int h = pl.max_height; h >= 1; --h) {
      std::vector<int> lev;
      for (int b = 0; b < nb; ++b)
        if (!pl.boxes[b].leaf && pl.boxes[b].height == h) lev.push_back(b);
      if (lev.empty()) continue;
      std::vector<ApplyDesc> sl, ug;
      std::vector<VecOpDesc> cp;
      for (int b : lev) {
        const Box &B = pl.boxes[b];
        const int m = (int)B.gi.size(), en = (int)B.nat.size(), ef = (int)B.fin.size();
        if (en == 0) {                 // a closure with no Dirichlet side: u_gi = w
          VecOpDesc v = vop(m, vref(BUF_VEC, H->ug_off, Lo.map_gi[b], kInterleaved),
                            vref(BUF_VEC, Lo.w[b], -1, kInterleaved), 1.0, vref(-1, 0, -1, 0), 0.0);
          v.b.buf = -1;
          cp.push_back(v);
          continue;
        }
        if (B.coarsened && !B.slave_rows.empty()) {
          ApplyDesc a = ad((int)B.slave_rows.size(), ef, 0, 0, Lo.Pups[b], (int)B.slave_rows.size());
          a.B1 = vref(BUF_VEC, H->ug_off, Lo.map_fin[b], kInterleaved);
          a.C = vref(BUF_VEC, H->ug_off, Lo.map_slave[b], kInterleaved);
          sl.push_back(a);
        }
        ApplyDesc a = ad(m, en, 0, 0, Lo.S[b], m);
        a.B1 = vref(BUF_VEC, H->ug_off, Lo.map_nat[b], kInterleaved);
        a.D = vref(BUF_VEC, Lo.w[b], -1, kInterleaved);
        a.beta = 1.0;
        a.C = vref(BUF_VEC, H->ug_off, Lo.map_gi[b], kInterleaved);
        ug.push_back(a);
      }
      apply_step(sl, dn);
      apply_step(ug, dn);
      vecop_step(cp, dn);
    }
    for (int i = 0; i < nleaf; ++i) {
      const int li = pl.leaves[i];
      const int role = pl.boxes[li].role;
      // u_ci = [S_ci | F] [u_ge; g] (economic: S_ci u_ge, F g added below)
      ApplyDesc a = ad(mi, g4, H->econ ? 0 : mi, 0, Lo.LD[li], mi);
      a.B1 = vref(BUF_VEC, H->ug_off, Lo.map_fin[li], kInterleaved);
      if (!H->econ) a.B2 = vref(BUF_IN1, int64_t(i) * mi, -1, gstride);
      a.C = vref(BUF_IN2, int64_t(i) * p * p, H->ici_map, ustride);
      tmp.push_back(a);
      ApplyDesc e = ad(me, g4, 0, 0, Lo.L_role[role], me);
      e.B1 = vref(BUF_VEC, H->ug_off, Lo.map_fin[li], kInterleaved);
      e.C = vref(BUF_IN2, int64_t(i) * p * p, H->ice_map, ustride);
      tmp.push_back(e);
    }
    apply_step(tmp, dn);
    if (H->econ) {
      // the storage-economic solve: per chunk of leaves, the leaf
      // Gauss-Jordan again (F into the chunk scratch, A_ci,ce not written),
      // then u_ci += F g
      for (int i = 0; i < nleaf; ++i) {
        LeafDesc d = leafd[i];
        d.hrows = 0;                  // H is stored already
        leafd.push_back(d);
      }
      for (int c0 = 0; c0 < nleaf; c0 += H->econ_chunk) {
        const int c1 = std::min(nleaf, c0 + H->econ_chunk);
        Step s{S_GJ_LEAF};
        s.d0 = nleaf + c0;
        s.nd = c1 - c0;
        dn.push_back(s);
        for (int i = c0; i < c1; ++i) {
          const Ref F = f_ref(i);
          ApplyDesc a = ad(mi, mi, 0, 0, F.off, mi);
          a.abuf = F.buf;
          a.B1 = vref(BUF_IN1, int64_t(i) * mi, -1, gstride);
          a.C = vref(BUF_IN2, int64_t(i) * p * p, H->ici_map, ustride);
          a.D = a.C;
          a.beta = 1.0;
          tmp.push_back(a);
        }
        apply_step(tmp, dn);
      }
    }
  }
  // transposed applies of the adjoint use the same descriptor layout
  auto apply_step_t = [&](std::vector<ApplyDesc> &tmp, std::vector<Step> &prg) {
    if (tmp.empty()) return;
    apply_step(tmp, prg);
    prg.back().trans = true;
  };
  // solve with a flux-jump source: the up pass with the B3 operand enabled
  {
    H->up_jump_prog.clear();
    for (const Step &st : H->up_prog) {
      bool wstep = false;
      for (int64_t i = st.d0; i < st.d0 + st.nd; ++i)
        if (appl[i].mode == 1) wstep = true;
      if (!wstep) { H->up_jump_prog.push_back(st); continue; }
      std::vector<ApplyDesc> tmp(appl.begin() + st.d0, appl.begin() + st.d0 + st.nd);
      for (auto &a : tmp) a.B3.buf = BUF_AUX;
      apply_step(tmp, H->up_jump_prog);
    }
  }
  // exterior Chebyshev values u_c(I_ce) = L u_ge alone (FP64 recompute)
  {
    H->ext_prog.clear();
    std::vector<ApplyDesc> tmp;
    for (int i = 0; i < nleaf; ++i) {
      const int li = pl.leaves[i];
      ApplyDesc e = ad(me, g4, 0, 0, Lo.L_role[pl.boxes[li].role], me);
      e.B1 = vref(BUF_VEC, H->ug_off, Lo.map_fin[li], kInterleaved);
      e.C = vref(BUF_IN2, int64_t(i) * p * p, H->ice_map, ustride);
      tmp.push_back(e);
    }
    apply_step(tmp, H->ext_prog);
  }
  // adjoint, reverse of the downward pass (children before parents):
  // inputs ubar (BUF_IN0), outputs fbar (BUF_IN1) and gbar (BUF_IN2).  A
  // periodic seam is an ordinary merge here; a Neumann closure box has no
  // beta, and its w-step read psi, so psibar = X^T wbar goes to fbar at the
  // Neumann entries (in the reverse of the upward pass)
  H->adj_down_prog.clear();
  H->adj_up_prog.clear();
  {
    auto &P = H->adj_down_prog;
    P.clear();
    std::vector<ApplyDesc> t1, t2;
    for (int i = 0; i < nleaf; ++i) {
      const int li = pl.leaves[i];
      const int role = pl.boxes[li].role;
      ApplyDesc a = ad(g4, me, 0, 0, Lo.L_role[role], me);      // L^T ubar(I_ce)
      a.B1 = vref(BUF_IN0, int64_t(i) * p * p, H->ice_map, ustride);
      a.C = vref(BUF_VEC, Lo.Ub[li], -1, kInterleaved);
      t1.push_back(a);
      ApplyDesc b = ad(g4, mi, 0, 0, Lo.LD[li], mi);            // + S_ci^T ubar(I_ci)
      b.B1 = vref(BUF_IN0, int64_t(i) * p * p, H->ici_map, ustride);
      b.D = vref(BUF_VEC, Lo.Ub[li], -1, kInterleaved);
      b.beta = 1.0;
      b.C = vref(BUF_VEC, Lo.Ub[li], -1, kInterleaved);
      t2.push_back(b);
      if (!H->econ) {                 // the adjoint needs the stored F
        ApplyDesc c = ad(mi, mi, 0, 0, Lo.LD[li] + int64_t(g4) * mi, mi);   // F^T ubar(I_ci)
        c.B1 = vref(BUF_IN0, int64_t(i) * p * p, H->ici_map, ustride);
        c.C = vref(BUF_IN2, int64_t(i) * mi, -1, gstride);
        t2.push_back(c);
      }
    }
    apply_step_t(t1, P);
    apply_step_t(t2, P);
    for (int h = 1; h <= pl.max_height; ++h) {
      std::vector<int> lev;
      for (int b = 0; b < nb; ++b)
        if (!pl.boxes[b].leaf && pl.boxes[b].height == h) lev.push_back(b);
      if (lev.empty()) continue;
      std::vector<VecOpDesc> v1;
      std::vector<ApplyDesc> a2, a3;
      for (int b : lev) {
        const Box &B = pl.boxes[b];
        const bool clo = B.kind == 3;
        const Box &A = pl.boxes[B.alpha], &C = pl.boxes[clo ? B.alpha : B.beta];
        const int m = (int)B.gi.size();
        const int ea = (int)A.fin.size(), eb = clo ? m : (int)C.fin.size();
        const int n1 = ea - m, n2 = eb - m, en = n1 + n2, ef = (int)B.fin.size();
        // wbar = ubar at the interior edge, summed over both children
        VecOpDesc wv = vop(m, vref(BUF_VEC, Lo.wb[b], -1, kInterleaved),
                           vref(BUF_VEC, Lo.Ub[B.alpha] + n1, -1, kInterleaved), 1.0,
                           vref(BUF_VEC, clo ? 0 : Lo.Ub[B.beta] + n2, -1, kInterleaved), 1.0);
        if (clo) wv.b.buf = -1;          // the closure's outside sibling holds no unknowns
        v1.push_back(wv);
        for (int part = 0; part < 2; ++part) {
          const int M = part == 0 ? n1 : n2;
          if (M == 0) continue;
          ApplyDesc a = ad(M, m, 0, 0, Lo.S[b] + (part == 0 ? 0 : int64_t(n1) * m), m);
          a.B1 = vref(BUF_VEC, Lo.wb[b], -1, kInterleaved);
          a.D = vref(BUF_VEC, part == 0 ? Lo.Ub[B.alpha] : Lo.Ub[B.beta], -1, kInterleaved);
          a.beta = 1.0;
          if (B.coarsened) a.C = vref(BUF_VEC, Lo.Ubn[b] + (part == 0 ? 0 : n1), -1, kInterleaved);
          else a.C = vref(BUF_VEC, Lo.Ub[b], Lo.map_pi[b] + (part == 0 ? 0 : n1), kInterleaved);
          a2.push_back(a);
        }
        if (B.coarsened) {
          ApplyDesc c = ad(ef, en, 0, 0, Lo.Pup[b], en);        // P_up^T
          c.B1 = vref(BUF_VEC, Lo.Ubn[b], -1, kInterleaved);
          c.C = vref(BUF_VEC, Lo.Ub[b], -1, kInterleaved);
          a3.push_back(c);
        }
      }
      vecop_step(v1, P);
      apply_step_t(a2, P);
      apply_step_t(a3, P);
    }
    // fbar at the Dirichlet entries from the top boxes' boundary slots; zero
    // at periodic entries (their data is not used); Neumann entries are
    // written by the reverse of the upward pass
    std::vector<int32_t> fpos, fmap, zpos;
    {
      std::unordered_map<int64_t, int64_t> where;
      for (int b = 0; b < nb; ++b) {
        const Box &B = pl.boxes[b];
        if (B.parent >= 0) continue;
        for (size_t k = 0; k < B.fin.size(); ++k) where[B.fin[k]] = Lo.Ub[b] + (int64_t)k;
      }
      for (size_t k = 0; k < pl.bdry.size(); ++k) {
        if (pl.bdry_kind[k] == kBcDirichlet) {
          auto it = where.find(pl.bdry[k]);
          if (it == where.end()) return fail(HPS_ETREE, "Dirichlet node missing from the top box");
          fpos.push_back((int32_t)k);
          fmap.push_back((int32_t)it->second);
        } else if (pl.bdry_kind[k] == kBcPeriodic) {
          zpos.push_back((int32_t)k);
        }
      }
    }
    std::vector<VecOpDesc> fv;
    if (!fpos.empty()) {
      H->map_fbar = imap_put(fmap);
      const int64_t mpos = imap_put(fpos);
      VecOpDesc v = vop((int)fpos.size(), vref(BUF_IN1, 0, mpos, H->n_bdry),
                        vref(BUF_VEC, 0, H->map_fbar, kInterleaved), 1.0, vref(-1, 0, -1, 0), 0.0);
      v.b.buf = -1;
      fv.push_back(v);
    }
    if (!zpos.empty()) {
      VecOpDesc v = vop((int)zpos.size(), vref(BUF_IN1, 0, imap_put(zpos), H->n_bdry),
                        vref(-1, 0, -1, 0), 0.0, vref(-1, 0, -1, 0), 0.0);
      v.a.buf = -1;
      v.b.buf = -1;
      fv.push_back(v);
    }
    vecop_step(fv, P);
  }
  // adjoint, reverse of the upward pass (parents before children)
  {
    auto &P = H->adj_up_prog;
    P.clear();
    for (int h = pl.max_height; h >= 1; --h) {
      std::vector<int> lev;
      for (int b = 0; b < nb; ++b)
        if (!pl.boxes[b].leaf && pl.boxes[b].height == h) lev.push_back(b);
      if (lev.empty()) continue;
      std::vector<ApplyDesc> u1, u2, u3, u4;
      std::vector<VecOpDesc> u5;
      for (int b : lev) {
        const Box &B = pl.boxes[b];
        const bool clo = B.kind == 3;
        const Box &A = pl.boxes[B.alpha], &C = pl.boxes[clo ? B.alpha : B.beta];
        const int m = (int)B.gi.size();
        const int ea = (int)A.fin.size(), eb = clo ? m : (int)C.fin.size();
        const int n1 = ea - m, n2 = eb - m, en = n1 + n2, ef = (int)B.fin.size();
        const bool root = B.parent < 0;
        // hbar in natural order: P_down^T hbar, or hbar through the permutation
        auto hnat = [&](int off) {
          if (B.coarsened) return vref(BUF_VEC, Lo.hbn[b] + off, -1, kInterleaved);
          return vref(BUF_VEC, Lo.hb[b], Lo.map_pi[b] + off, kInterleaved);
        };
        if (!root && B.coarsened) {
          ApplyDesc a = ad(en, ef, 0, 0, Lo.Pdn[b], ef);
          a.B1 = vref(BUF_VEC, Lo.hb[b], -1, kInterleaved);
          a.C = vref(BUF_VEC, Lo.hbn[b], -1, kInterleaved);
          u1.push_back(a);
        }
        if (!root && n1 > 0) {                       // wbar += T13a^T hbar_1
          ApplyDesc a = ad(m, n1, 0, 0, Lo.T[B.alpha] + int64_t(n1) * ea, ea);
          a.B1 = hnat(0);
          a.D = vref(BUF_VEC, Lo.wb[b], -1, kInterleaved);
          a.beta = 1.0;
          a.C = vref(BUF_VEC, Lo.wb[b], -1, kInterleaved);
          u2.push_back(a);
        }
        if (!root && n2 > 0) {                       // wbar += T23b^T hbar_2
          ApplyDesc a = ad(m, n2, 0, 0, Lo.T[B.beta] + int64_t(n2) * eb, eb);
          a.B1 = hnat(n1);
          a.D = vref(BUF_VEC, Lo.wb[b], -1, kInterleaved);
          a.beta = 1.0;
          a.C = vref(BUF_VEC, Lo.wb[b], -1, kInterleaved);
          u3.push_back(a);
        }
        for (int side = 0; side < 2; ++side) {       // d = X^T wbar into h3a (-), h3b (+)
          ApplyDesc a = ad(m, m, 0, 0, Lo.X[b], m);
          a.B1 = vref(BUF_VEC, Lo.wb[b], -1, kInterleaved);
          a.alpha = side == 0 ? -1.0 : 1.0;
          a.C = side == 0 ? vref(BUF_VEC, Lo.hb[B.alpha] + n1, -1, kInterleaved)
                          : clo ? vref(BUF_IN1, 0, Lo.map_psi[b], H->n_bdry)   // psibar
                                : vref(BUF_VEC, Lo.hb[B.beta] + n2, -1, kInterleaved);
          u4.push_back(a);
        }
        for (int side = 0; side < 2; ++side) {       // kept parts pass through
          const int n = side == 0 ? n1 : n2;
          if (n == 0) continue;
          VecOpDesc v = vop(n, vref(BUF_VEC, side == 0 ? Lo.hb[B.alpha] : Lo.hb[B.beta], -1, kInterleaved),
                            hnat(side == 0 ? 0 : n1), 1.0, vref(-1, 0, -1, 0), 0.0);
          v.b.buf = -1;
          if (root) v.a.buf = -1;                    // the root's hbar is zero
          u5.push_back(v);
        }
      }
      apply_step_t(u1, P);
      apply_step_t(u2, P);
      apply_step_t(u3, P);
      apply_step_t(u4, P);
      vecop_step(u5, P);
    }
    std::vector<ApplyDesc> g;
    for (int i = 0; i < nleaf; ++i) {                // gbar += H^T hbar
      const int li = pl.leaves[i];
      ApplyDesc a = ad(mi, g4, 0, 0, Lo.H[li], g4);
      a.B1 = vref(BUF_VEC, Lo.hb[li], -1, kInterleaved);
      a.D = vref(BUF_IN2, int64_t(i) * mi, -1, gstride);
      a.beta = 1.0;
      a.C = vref(BUF_IN2, int64_t(i) * mi, -1, gstride);
      g.push_back(a);
    }
    if (pl.max_height == 0) {                        // a single leaf: hbar = 0
      g.clear();
    }
    apply_step_t(g, P);
  }
  // flux-jump maps of the refinement residual (conforming trees only)
  {
    bool conf = true;
    for (const Box &B : pl.boxes) if (B.coarsened) conf = false;
    H->conforming = conf;
    std::vector<int32_t> jn, fa, fb, fp;
    if (conf) {
      // owner (leaf index, natural position) of each node on each side
      std::vector<int64_t> own_a(pl.n_gauss, -1), own_b(pl.n_gauss, -1);
      for (int i = 0; i < nleaf; ++i) {
        const Box &B = pl.boxes[pl.leaves[i]];
        for (int k = 0; k < g4; ++k) {
          const int64_t j = B.nat[k];
          const int side = k / q;
          // west/south leaf sees the node on its E or N side: alpha side
          if (side == 1 || side == 2) own_a[j] = int64_t(i) * g4 + k;
          else own_b[j] = int64_t(i) * g4 + k;
        }
      }
      // a periodic seam is eliminated by a merge whose alpha lies on the
      // seam's west (south) side, where its leaves see the node on their W
      // (S) side: the two roles are swapped there
      for (int64_t j = 0; j < pl.n_gauss; ++j) {
        const Segment &S = pl.segs[j / q];
        const Problem &P = H->tree.probs[S.problem];
        const bool seam = S.fixed == 0 && ((S.orient == 'v' && P.bc[1] == kBcPeriodic) ||
                                           (S.orient == 'h' && P.bc[2] == kBcPeriodic));
        if (seam) std::swap(own_a[j], own_b[j]);
      }
      for (int64_t j = 0; j < pl.n_gauss; ++j)
        if (own_a[j] >= 0 && own_b[j] >= 0) {
          jn.push_back((int32_t)j);
          fa.push_back((int32_t)own_a[j]);
          fb.push_back((int32_t)own_b[j]);
          fp.push_back(-1);
        }
      // a Neumann node's row reads flux = psi: its residual is psi - flux
      for (size_t k = 0; k < pl.bdry.size(); ++k) {
        if (pl.bdry_kind[k] != kBcNeumann) continue;
        const int64_t j = pl.bdry[k];
        jn.push_back((int32_t)j);
        fa.push_back((int32_t)(own_a[j] >= 0 ? own_a[j] : own_b[j]));
        fb.push_back(-1);
        fp.push_back((int32_t)k);
      }
    }
    H->n_jump = (int64_t)jn.size();
    H->h_jn = std::move(jn);
    H->h_fa = std::move(fa);
    H->h_fb = std::move(fb);
    H->h_fp = std::move(fp);
    std::vector<double> xc = cheb_points(p), xg = legendre_roots(q);
    H->h_lloc = interp_matrix(xc, xg);
  }
  H->part_per_rhs = part_off;
  H->off_T = Lo.T; H->off_X = Lo.X; H->off_S = Lo.S; H->off_LD = Lo.LD; H->off_H = Lo.H;
  // identity map covering every k an apply reads from an unmapped operand
  int maxk = 1;
  for (const ApplyDesc &a : appl) maxk = std::max(maxk, std::max(a.K1, a.K2));
  std::vector<int32_t> iota(maxk);
  for (int k = 0; k < maxk; ++k) iota[k] = k;
  H->iota_off = imap_put(iota);
  return HPS_OK;
}

// Builds layout, uploads reference matrices and maps, generates programs.
static int plan_handle(hps_handle *H, Layout &Lo, std::vector<double> &ws_init,
                       std::vector<std::pair<int64_t, std::vector<double>>> &ws_blocks,
                       std::vector<int32_t> &imap, GemmList &gl, std::vector<LeafDesc> &leafd,
                       std::vector<MergeInvDesc> &minv, std::vector<ApplyDesc> &appl,
                       std::vector<int32_t> &appl_tmap, std::vector<int32_t> &finlist,
                       std::vector<VecOpDesc> &vops) {
  PlanCtx C{H, Lo, ws_init, ws_blocks, imap, gl, leafd, minv, appl, appl_tmap, finlist, vops,
            {}, -1};
  int rc = plan_layout(C);
  if (rc == HPS_OK) rc = plan_build_program(C);
  if (rc == HPS_OK) rc = plan_solve_programs(C);
  return rc;
}

Bases make_bases(hps_handle *H) {
  Bases b{};
  b.d[BUF_WS] = H->ws.p;
  b.d[BUF_SCR] = H->scr.p;
  b.d[BUF_VEC] = H->vec.p;
  b.d[BUF_W32] = H->ws32.p;
  b.d[BUF_AUX] = H->aux.p;
  b.d[BUF_COEF] = H->coef.p;
  b.imap = H->imap.p;
  b.iota = H->imap.p ? H->imap.p + H->iota_off : nullptr;
  return b;
}

// Algorithmic work of each launch step, from the host descriptor lists.
static void annotate_work(std::vector<Step> &prog, const GemmList &gl,
                          const std::vector<MergeInvDesc> &mv,
                          const std::vector<ApplyDesc> &ap, int mi, int p, int g4) {
  // the leaf kernel's work: the inverse, and H = D_ge,ci F where it forms H
  const double leaf_w = 2.0 * double(mi) * mi * mi +
                        (leaf_kernel_forms_h(p, g4) ? 2.0 * double(g4) * mi * mi : 0.0);
  for (Step &s : prog) {
    double w = 0.0;
    for (int64_t i = s.d0; i < s.d0 + s.nd; ++i) {
      switch (s.kind) {
        case S_GEMM: w += 2.0 * gl.d[i].M * double(gl.d[i].N) * gl.d[i].K; break;
        case S_GJ_LEAF: w += leaf_w; break;
        case S_LEAF_B: w += 10.0 * double(mi) * g4; break;
        case S_GJ_MERGE: w += 2.0 * double(mv[i].m) * mv[i].m * mv[i].m; break;
        case S_PANEL: {
          // update by panel kb of the other columns, sweep of panel kb + NB
          // (the level form: every kb)
          const int NBp = panel_nb(s.maxm), m = mv[i].m;
          const int k_lo = s.kb == kPanelLevel ? -NBp : s.kb;
          const int k_hi = s.kb == kPanelLevel ? m : s.kb + 1;
          for (int kb = k_lo; kb < k_hi; kb += NBp) {
            const double nu = kb >= 0 ? std::min(NBp, m - kb) : 0;
            const double ns = std::min(NBp, m - (kb + NBp));
            if (nu > 0) w += 2.0 * m * (m - nu) * nu;
            if (ns > 0) w += 2.0 * m * ns * ns;
          }
          break;
        }
        case S_APPLY:
          w += double(ap[i].M) * (ap[i].K1 + (ap[i].mode == 0 ? ap[i].K2 : 0));
          break;
        default: break;
      }
    }
    s.work = w;
  }
}

// Per tile variant: the GEMM descriptors re-tiled for that variant's
// TM x TN tiles and the tile maps of every GEMM step of every program (a
// step's tile0 and tile map are relative to its own first descriptor).
static_assert(kGemmVariants <= 8, "Step keeps at most eight tile variants");
static int upload_gemm_variants(hps_handle *H, const std::vector<GemmDesc> &d0,
                                std::vector<std::vector<Step> *> progs) {
  for (int v = 0; v < kGemmVariants; ++v) {
    const int TM = gemm_variant_tm(v), TN = gemm_variant_tn(v);
    std::vector<GemmDesc> dv = d0;
    std::vector<int32_t> tv;
    for (std::vector<Step> *prog : progs)
      for (Step &s : *prog) {
        if (s.kind != S_GEMM) continue;
        s.vtmap0[v] = (int64_t)tv.size();
        int64_t t = 0;
        for (int64_t i = s.d0; i < s.d0 + s.nd; ++i) {
          GemmDesc &g = dv[size_t(i)];
          g.tn = (g.N + TN - 1) / TN;
          const int64_t tm = (g.M + TM - 1) / TM;
          g.tile0 = t;
          t += tm * g.tn;
          tv.insert(tv.end(), size_t(tm * g.tn), int32_t(i - s.d0));
        }
        s.vtiles[v] = t;
      }
    HIPCHK(H->d_gemm_v[v].upload(dv));
    HIPCHK(H->d_gemm_tmap_v[v].upload(tv));
  }
  return HPS_OK;
}

// GEMM tile tuner.  The first build of a handle times every tile variant on
// each GEMM step of its program (two launches after a warm-up, HIP events)
// and keeps the fastest; all variants compute bitwise the same result, so
// the choice never changes the operators.  Winners are cached per process,
// keyed by the device architecture and the step's shape class (descriptor
// count, first descriptor's M x N x K, the step's 64 x 64 tile count), and,
// when HPS_GEMM_TUNE_CACHE names a file, read from and appended to it.
// HPS_GEMM_TUNE=0 switches tuning off (64 x 64 tiles everywhere).
namespace {
std::mutex g_tune_mu;
std::map<std::string, int> g_tune;
bool g_tune_loaded = false;

std::string tune_key(const Step &s, const GemmDesc &g0) {
  int dev = 0;
  hipDeviceProp_t prop{};
  std::string arch = "gpu";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    arch = prop.gcnArchName;
  const size_t c = arch.find(':');
  if (c != std::string::npos) arch.resize(c);
  return arch + " " + std::to_string(s.nd) + " " + std::to_string(g0.M) + "x" +
         std::to_string(g0.N) + "x" + std::to_string(g0.K) + " " + std::to_string(s.vtiles[0]);
}

void tune_cache_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char *path = std::getenv("HPS_GEMM_TUNE_CACHE");
  if (!path) return;
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    const size_t bar = line.rfind('|');
    if (bar == std::string::npos) continue;
    g_tune[line.substr(0, bar)] = std::atoi(line.c_str() + bar + 1);
  }
}

void tune_cache_store(const std::string &key, int v) {
  g_tune[key] = v;
  const char *path = std::getenv("HPS_GEMM_TUNE_CACHE");
  if (!path) return;
  std::ofstream out(path, std::ios::app);
  out << key << "|" << v << "\n";
}
}  // namespace

static bool gemm_tuning_enabled() {
  const char *e = std::getenv("HPS_GEMM_TUNE");
  return !(e && e[0] == '0');
}

static int tune_gemm_step(hps_handle *H, Step &s, const Bases &bs, hipStream_t st) {
  GemmDesc g0{};
  HIPCHK(hipMemcpy(&g0, H->d_gemm_v[0].p + s.d0, sizeof(GemmDesc), hipMemcpyDeviceToHost));
  const std::string key = tune_key(s, g0);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_cache_load();
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      s.var = it->second;
      return HPS_OK;
    }
  }
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  float best = 0.0f;
  int bv = 0;
  hipError_t err = hipSuccess;
  for (int v = 0; v < kGemmVariants && err == hipSuccess; ++v) {
    auto go = [&]() {
      return launch_gemm(v, H->d_gemm_v[v].p + s.d0, H->d_gemm_tmap_v[v].p + s.vtmap0[v],
                         s.vtiles[v], bs, st);
    };
    err = go();
    if (err == hipSuccess) err = hipEventRecord(e0, st);
    for (int r = 0; r < 2 && err == hipSuccess; ++r) err = go();
    if (err == hipSuccess) err = hipEventRecord(e1, st);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
    if (err == hipSuccess && (v == 0 || ms < best)) {
      best = ms;
      bv = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return fail(HPS_EHIP, std::string("GEMM tuning: ") + hipGetErrorString(err));
  s.var = bv;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_cache_store(key, bv);
  return HPS_OK;
}

static hipEvent_t prof_event(hps_handle *H) {
  if (H->prof_used == H->prof_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    H->prof_pool.push_back(e);
  }
  return H->prof_pool[H->prof_used++];
}

int run_prog(hps_handle *H, std::vector<Step> &prog, Bases bs, int nrhs, int prec,
             hipStream_t st) {
  for (Step &s : prog) {
    if (s.kind == S_GEMM && H->tune_gemm) {
      const int rc = tune_gemm_step(H, s, bs, st);
      if (rc) return rc;
    }
    hipError_t e = hipSuccess;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (H->prof_on) {
      e0 = prof_event(H);
      e1 = prof_event(H);
      if (e0 && e1) (void)hipEventRecord(e0, st);
    }
    switch (s.kind) {
      case S_GEMM:
        e = launch_gemm(s.var, H->d_gemm_v[s.var].p + s.d0,
                        H->d_gemm_tmap_v[s.var].p + s.vtmap0[s.var], s.vtiles[s.var], bs, st);
        break;
      case S_GJ_LEAF:
        e = launch_gj_leaf(H->p, H->d_leaf.p + s.d0, (int)s.nd, bs, H->aux.p + H->Dh_off,
                           H->aux.p + H->Dh2_off, H->info.p, st);
        break;
      case S_LEAF_B:
        e = launch_leaf_b(H->d_leaf.p, H->imap.p + s.tmap0, (int)s.ntiles, H->imap.p + s.d0, bs,
                          H->p, H->g4, st);
        break;
      case S_GJ_MERGE:
        e = launch_gj_merge(s.cls, H->d_minv.p + s.d0, (int)s.nd, bs, H->info.p, st);
        break;
      case S_ZDIFF:
        e = launch_zdiff(H->d_minv.p + s.d0, (int)s.nd, s.maxm, bs, st);
        if (e == hipSuccess) e = launch_gj_ginit(H->d_minv.p + s.d0, (int)s.nd, s.maxm, H->ipiv.p, st);
        break;
      case S_PANEL:
        if (s.kb == kPanelLevel)
          e = launch_gj_level(H->d_minv.p + s.d0, (int)s.nd, s.maxm, bs, H->ipiv.p, H->info.p,
                              s.cls, st);
        else
          e = launch_gj_panel(H->d_minv.p + s.d0, (int)s.nd, s.kb, s.maxm, bs, H->ipiv.p,
                              H->info.p, st);
        break;
      case S_COLPERM:
        e = launch_gj_colperm(H->d_minv.p + s.d0, (int)s.nd, s.maxm, bs, H->ipiv.p, H->psrc.p,
                              st);
        break;
      case S_APPLY:
        e = launch_apply(prec, H->d_apply.p + s.d0, H->d_apply_tmap.p + s.tmap0, s.ntiles,
                         bs, nrhs, st, s.trans);
        if (e == hipSuccess && s.nfin > 0)
          e = launch_apply_finalize(H->d_apply.p, H->d_finlist.p + s.fin0, (int)s.nfin,
                                    s.fin_maxm, bs, nrhs, st);
        break;
      case S_VECOP:
        e = launch_vecop(H->d_vecop.p + s.d0, (int)s.nd, s.maxm, bs, nrhs, st);
        break;
      default:
        break;
    }
    if (e != hipSuccess) return fail(HPS_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
    if (H->prof_on && e0 && e1) {
      (void)hipEventRecord(e1, st);
      int kind = int(s.kind) * 16 + (s.kind == S_GJ_MERGE ? s.cls : s.kind == S_GEMM ? s.var : 0);
      if (s.kind == S_APPLY) kind += prec;
      H->prof_ev.push_back({kind, {e0, e1}});
      H->prof_work.push_back(s.work);
    }
  }
  return HPS_OK;
}

extern "C" {

// Device check that every leaf has the coefficients of leaf 0 (translation
// invariant builds share operators between leaves); waits for the stream.
static int check_constant_coeffs(hps_handle *H, const double *coeffs, hipStream_t st) {
  if (!H->cflag.p) HIPCHK(H->cflag.alloc(1));
  const int64_t per = int64_t(6) * H->p * H->p;
  HIPCHK(hipMemsetAsync(H->cflag.p, 0, sizeof(int32_t), st));
  HIPCHK(launch_block_diff(coeffs, per, per * H->nleaf, H->cflag.p, st));
  int32_t f = 0;
  HIPCHK(hipMemcpyAsync(&f, H->cflag.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (f) return fail(HPS_EINVAL, "translation_invariant: the leaves' coefficients differ");
  return HPS_OK;
}

size_t hps_build_workspace_size(const hps_tree *tree, int p, const hps_build_opts *opts) {
  if (!tree || p < 4) return 0;
  int q = opts && opts->q > 0 ? opts->q : p - 1;
  const int economic = opts ? opts->economic : 0;
  const int translation_invariant = opts ? opts->translation_invariant : 0;
  hps_handle H;
  H.tree = tree->t;
  H.econ = economic != 0;
  H.dedup = translation_invariant != 0;
  if (H.econ && H.dedup) return 0;
  if (plan_tree(H.tree, H.pl, q)) return 0;
  if (H.dedup)
    for (const Box &b : H.pl.boxes)
      if (b.coarsened) return 0;
  H.p = p; H.q = q; H.mi = (p - 2) * (p - 2); H.me = 4 * (p - 1); H.g4 = 4 * q;
  H.nleaf = (int)H.pl.leaves.size();
  Layout Lo;
  std::vector<double> wi;
  std::vector<std::pair<int64_t, std::vector<double>>> blocks;
  std::vector<int32_t> imap;
  GemmList gl;
  std::vector<LeafDesc> ld;
  std::vector<MergeInvDesc> mv;
  std::vector<ApplyDesc> ap;
  std::vector<int32_t> at0;
  std::vector<int32_t> fl;
  std::vector<VecOpDesc> vo;
  if (plan_handle(&H, Lo, wi, blocks, imap, gl, ld, mv, ap, at0, fl, vo)) return 0;
  return size_t(Lo.ws) * sizeof(double);
}

int hps_build(const hps_tree *tree, const double *coeffs, int p, const hps_build_opts *opts,
              hps_handle **out) {
  if (!out) return fail(HPS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!tree || !coeffs) return fail(HPS_EINVAL, "NULL tree or coefficients");
  int q = opts && opts->q > 0 ? opts->q : p - 1;
  if (p < 4 || q < 2 || q >= p) return fail(HPS_EINVAL, "need p >= 4 and 2 <= q < p");
  if (!gj_leaf_supported(p)) return fail(HPS_EINVAL, "p must be one of 6, 8, 10, 12, 16");
  if (opts && opts->economic && opts->keep_fp32)
    return fail(HPS_EINVAL, "economic builds keep no leaf operators to copy to FP32");
  hipStream_t st = opts ? (hipStream_t)opts->stream : nullptr;
  std::unique_ptr<hps_handle> H(new (std::nothrow) hps_handle);
  if (!H) return fail(HPS_ENOMEM, "host allocation");
  H->tree = tree->t;
  H->econ = opts && opts->economic;
  H->dedup = opts && opts->translation_invariant;
  if (H->econ && H->dedup)
    return fail(HPS_EINVAL, "economic and translation_invariant builds do not combine");
  int rc = plan_tree(H->tree, H->pl, q);
  if (rc) return rc;
  H->p = p; H->q = q; H->mi = (p - 2) * (p - 2); H->me = 4 * (p - 1); H->g4 = 4 * q;
  H->nleaf = (int)H->pl.leaves.size();
  for (const Problem &P : H->tree.probs) {
    bool dirichlet = false;
    for (int s = 0; s < 4; ++s) dirichlet |= P.bc[s] == kBcDirichlet;
    // with q = p - 1 the leaf Gauss -> Chebyshev maps share a null vector
    // that only Dirichlet data removes
    if (!dirichlet && q > p - 2)
      return fail(HPS_EINVAL, "a problem without a Dirichlet side needs q <= p - 2");
  }
  for (const Box &b : H->pl.boxes) {
    if (!b.leaf && (int)b.gi.size() > 2048)
      return fail(HPS_EINVAL, "interface longer than 2048 nodes");
    if (H->dedup && b.coarsened)
      return fail(HPS_EINVAL, "translation_invariant builds need a tree without refined interfaces");
  }
  if (H->dedup) {
    rc = check_constant_coeffs(H.get(), coeffs, st);
    if (rc) return rc;
  }
  Layout Lo;
  std::vector<double> aux_init;
  std::vector<std::pair<int64_t, std::vector<double>>> blocks;
  std::vector<int32_t> imap;
  GemmList gl;
  std::vector<LeafDesc> leafd;
  std::vector<MergeInvDesc> minv;
  std::vector<ApplyDesc> appl;
  std::vector<int32_t> appl_tmap;
  std::vector<int32_t> finlist;
  std::vector<VecOpDesc> vops;
  rc = plan_handle(H.get(), Lo, aux_init, blocks, imap, gl, leafd, minv, appl, appl_tmap, finlist,
                   vops);
  if (rc) return rc;
  for (auto *prog : {&H->build_prog, &H->up_prog, &H->down_prog, &H->adj_down_prog,
                     &H->adj_up_prog, &H->up_jump_prog, &H->ext_prog})
    annotate_work(*prog, gl, minv, appl, H->mi, H->p, H->g4);
  H->solve_elems = (size_t)Lo.solve_ws;
  H->scr_build = Lo.scr + 64;
  if (opts && opts->workspace) {
    const size_t need = size_t(Lo.ws) * sizeof(double);
    if (opts->workspace_bytes < need)
      return fail(HPS_EINVAL, "workspace holds " + std::to_string(opts->workspace_bytes) +
                                  " bytes; the operators need " + std::to_string(need));
    if (reinterpret_cast<uintptr_t>(opts->workspace) % 256 != 0)
      return fail(HPS_EINVAL, "workspace must be 256-byte aligned");
    H->ws.borrow(static_cast<double *>(opts->workspace), size_t(Lo.ws));
  } else if (H->ws.alloc(Lo.ws) != hipSuccess) {
    return fail(HPS_ENOMEM, "device allocation of the operator workspace");
  }
  if (H->scr.alloc(Lo.scr + 64) != hipSuccess)
    return fail(HPS_ENOMEM, "device allocation of the build scratch");
  HIPCHK(H->imap.upload(imap));
  HIPCHK(H->aux.upload(aux_init));
  HIPCHK(H->info.alloc(H->n_info));
  HIPCHK(hipMemset(H->info.p, 0, sizeof(int32_t) * H->n_info));
  HIPCHK(H->ipiv.alloc(Lo.ipiv_n + 1));
  HIPCHK(H->psrc.alloc(Lo.ipiv_n + 1));
  for (auto &bl : blocks)
    HIPCHK(hipMemcpy(H->ws.p + bl.first, bl.second.data(), bl.second.size() * sizeof(double),
                     hipMemcpyHostToDevice));
  rc = upload_gemm_variants(H.get(), gl.d, {&H->build_prog, &H->up_prog, &H->down_prog,
                                            &H->adj_down_prog, &H->adj_up_prog,
                                            &H->up_jump_prog, &H->ext_prog});
  if (rc) return rc;
  HIPCHK(H->d_leaf.upload(leafd));
  HIPCHK(H->d_minv.upload(minv));
  HIPCHK(H->d_apply.upload(appl));
  HIPCHK(H->d_apply_tmap.upload(appl_tmap));
  HIPCHK(H->d_finlist.upload(finlist));
  HIPCHK(H->d_vecop.upload(vops));
  HIPCHK(H->d_jn.upload(H->h_jn));
  HIPCHK(H->d_fa.upload(H->h_fa));
  HIPCHK(H->d_fb.upload(H->h_fb));
  HIPCHK(H->d_fp.upload(H->h_fp));
  HIPCHK(H->d_lloc.upload(H->h_lloc));
  // keep the coefficients (residuals of mixed-precision solves use them)
  const size_t ncoef = size_t(H->nleaf) * 6 * p * p;
  HIPCHK(H->coef.alloc(ncoef));
  HIPCHK(hipMemcpyAsync(H->coef.p, coeffs, ncoef * sizeof(double), hipMemcpyDeviceToDevice, st));
  Bases bs = make_bases(H.get());
  H->tune_gemm = gemm_tuning_enabled();
  rc = run_prog(H.get(), H->build_prog, bs, 1, 0, st);
  H->tune_gemm = false;
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(st));
  std::vector<int32_t> info(H->n_info);
  HIPCHK(hipMemcpy(info.data(), H->info.p, sizeof(int32_t) * H->n_info, hipMemcpyDeviceToHost));
  for (int i = 0; i < H->n_info; ++i)
    if (info[i] != 0) {
      const bool leaf = i < H->nleaf;
      const std::string what = leaf ? "leaf " + std::to_string(i) : "merge " + std::to_string(i - H->nleaf);
      if (info[i] == kGjSyncTimeout)
        return fail(HPS_EHIP, "synchronisation wait timed out in the Gauss-Jordan of " + what);
      if (info[i] > 0)
        return fail(HPS_ESINGULAR, "zero pivot at step " + std::to_string(info[i]) + " of " + what);
      return fail(HPS_ENONFINITE, "non-finite pivot at step " + std::to_string(-info[i]) + " of " + what);
    }
  if (opts && opts->keep_fp32) {
    HIPCHK(H->ws32.alloc(H->solve_elems));
    HIPCHK(launch_cast_f32(H->ws.p, H->ws32.p, (int64_t)H->solve_elems, st));
    H->has_fp32 = true;
  }
  rc = solve_ext_init(H.get());
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(st));
  *out = H.release();
  return HPS_OK;
}

// Recompute every operator of an existing handle for new coefficients (same
// tree, p, q): Algorithm 1 again without any device allocation.
int hps_refactor(hps_handle *H, const double *coeffs, void *stream) {
  if (!H || !coeffs) return fail(HPS_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  if (H->dedup) {
    const int rc0 = check_constant_coeffs(H, coeffs, st);
    if (rc0) return rc0;
  }
  if (H->scr.n < size_t(H->scr_build)) HIPCHK(H->scr.alloc(H->scr_build));
  HIPCHK(hipMemsetAsync(H->info.p, 0, sizeof(int32_t) * H->n_info, st));
  const size_t ncoef = size_t(H->nleaf) * 6 * H->p * H->p;
  HIPCHK(hipMemcpyAsync(H->coef.p, coeffs, ncoef * sizeof(double), hipMemcpyDeviceToDevice, st));
  Bases bs = make_bases(H);           // coefficients: the handle's copy (fixed address)
  int rc = HPS_OK;
  if (H->prof_on) {
    rc = run_prog(H, H->build_prog, bs, 1, 0, st);   // per-launch events need eager launches
  } else {
    if (!H->build_exec || H->build_exec_scr != H->scr.p) {
      if (H->build_exec) HIPCHK(hipGraphExecDestroy(H->build_exec));
      H->build_exec = nullptr;
      hipStream_t cs;
      HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        rc = run_prog(H, H->build_prog, bs, 1, 0, cs);
        e = hipStreamEndCapture(cs, &g);
      }
      if (e == hipSuccess && rc == HPS_OK)
        e = hipGraphInstantiate(&H->build_exec, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      (void)hipStreamDestroy(cs);
      if (rc) return rc;
      if (e != hipSuccess) {
        H->build_exec = nullptr;
        return fail(HPS_EHIP, std::string("build graph: ") + hipGetErrorString(e));
      }
      H->build_exec_scr = H->scr.p;
    }
    HIPCHK(hipGraphLaunch(H->build_exec, st));
  }
  std::vector<int32_t> info(H->n_info);
  HIPCHK(hipMemcpyAsync(info.data(), H->info.p, sizeof(int32_t) * H->n_info,
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int i = 0; i < H->n_info; ++i)
    if (info[i] != 0) {
      const std::string what = i < H->nleaf ? "leaf " + std::to_string(i)
                                            : "merge " + std::to_string(i - H->nleaf);
      if (info[i] == kGjSyncTimeout)
        return fail(HPS_EHIP, "synchronisation wait timed out in the Gauss-Jordan of " + what);
      if (info[i] > 0)
        return fail(HPS_ESINGULAR, "zero pivot at step " + std::to_string(info[i]) + " of " + what);
      return fail(HPS_ENONFINITE, "non-finite pivot at step " + std::to_string(-info[i]) + " of " + what);
    }
  if (H->has_fp32) HIPCHK(launch_cast_f32(H->ws.p, H->ws32.p, (int64_t)H->solve_elems, st));
  HIPCHK(hipStreamSynchronize(st));
  return HPS_OK;
}

void hps_handle_free(hps_handle *h) { delete h; }

}  // extern "C"

// ---------------------------------------------------------------------------
// solve
// ---------------------------------------------------------------------------
int ensure_solve_buffers(hps_handle *H, int nrhs) {
  const size_t need_vec = size_t(H->vec_per_rhs) * nrhs;
  if (H->vec.n < need_vec) HIPCHK(H->vec.alloc(need_vec));
  const size_t need_part = size_t(H->part_per_rhs) * nrhs + 64;
  if (H->scr.n < need_part) HIPCHK(H->scr.alloc(std::max<size_t>(need_part, H->scr_build)));
  return HPS_OK;
}

// Doubles of per-solve work memory for nrhs right-hand sides: the work
// vectors (BUF_VEC) followed by the split-K partials (BUF_SCR).
int64_t solve_vec_elems(const hps_handle *H, int nrhs) { return H->vec_per_rhs * nrhs; }
int64_t solve_work_elems(const hps_handle *H, int nrhs) {
  return (H->vec_per_rhs + H->part_per_rhs) * nrhs + 64;
}

// One pass of Algorithm 2 in precision prec (0 FP64, 1 FP32 operators) on
// the given work memory (vec: solve_vec_elems doubles, scr: the split-K
// partials).  f, g, u are device arrays in the canonical layouts; jump
// (optional) adds a flux-jump source on interior Gauss nodes (the refinement
// correction).
int hps_solve_pass_on(hps_handle *H, const double *f, const double *g, int nrhs, double *u,
                      int prec, const double *jump, double *vec, double *scr, hipStream_t st) {
  Bases bs = make_bases(H);
  bs.d[BUF_VEC] = vec;
  bs.d[BUF_SCR] = scr;
  if (prec == 1) {
    if (!H->has_fp32) return fail(HPS_EINVAL, "handle was built without keep_fp32");
    bs.d[BUF_WS] = H->ws32.p;
  }
  bs.d[BUF_IN0] = (void *)f;
  bs.d[BUF_IN1] = (void *)g;
  bs.d[BUF_IN2] = (void *)u;
  bs.d[BUF_AUX] = (void *)jump;
  // with a flux-jump source the w-steps read it as their third operand
  int rc = run_prog(H, jump ? H->up_jump_prog : H->up_prog, bs, nrhs, prec, st);
  if (rc) return rc;
  HIPCHK(launch_copy_map(bs, vref(BUF_VEC, H->ug_off, H->map_bdry, kInterleaved),
                         vref(BUF_IN0, 0, -1, H->n_bdry), H->n_bdry, nrhs, st));
  return run_prog(H, H->down_prog, bs, nrhs, prec, st);
}

// The same on the handle's own work buffers (grown on demand).
int hps_solve_pass(hps_handle *H, const double *f, const double *g, int nrhs, double *u,
                   int prec, const double *jump, hipStream_t st) {
  int rc = ensure_solve_buffers(H, nrhs);
  if (rc) return rc;
  return hps_solve_pass_on(H, f, g, nrhs, u, prec, jump, H->vec.p, H->scr.p, st);
}

// hps_solve on caller-supplied work memory of `bytes` bytes (device): no
// allocation.  FP64 and FP32 sweeps of stored (not economic) builds only.
int hps_solve_on_scratch(hps_handle *h, const double *f, const double *g, int nrhs, double *u,
                         const hps_solve_opts *opts, double *work, size_t bytes) {
  if (!h || !f || !g || !u) return fail(HPS_EINVAL, "NULL argument");
  if (!work) return fail(HPS_EHIP, "no device address for the solve work array");
  if (nrhs <= 0) return fail(HPS_EINVAL, "nrhs must be positive");
  const int prec = opts ? opts->precision : HPS_PREC_FP64;
  if (prec != HPS_PREC_FP64 && prec != HPS_PREC_FP32)
    return fail(HPS_EINVAL, "the allocation-free solve runs FP64 or FP32 sweeps only");
  if (h->econ)
    return fail(HPS_EINVAL, "the allocation-free solve needs stored leaf operators (not economic)");
  if (h->prof_on)
    return fail(HPS_EINVAL, "per-launch profiling creates events; switch it off first");
  const size_t need = size_t(solve_work_elems(h, nrhs)) * sizeof(double);
  if (need > bytes)
    return fail(HPS_EINVAL, "the solve needs " + std::to_string(need) + " bytes of work memory for " +
                                std::to_string(nrhs) + " right-hand sides; the fixed array holds " +
                                std::to_string(bytes));
  hipStream_t st = opts ? (hipStream_t)opts->stream : nullptr;
  double *vec = work, *scr = work + solve_vec_elems(h, nrhs);
  int rc = hps_solve_pass_on(h, f, g, nrhs, u, prec == HPS_PREC_FP32 ? 1 : 0, nullptr, vec, scr, st);
  if (rc) return rc;
  if (opts && opts->u_gauss) {
    Bases bs = make_bases(h);
    bs.d[BUF_VEC] = vec;
    bs.d[BUF_IN0] = opts->u_gauss;
    HIPCHK(launch_copy_map(bs, vref(BUF_IN0, 0, -1, h->pl.n_gauss),
                           vref(BUF_VEC, h->ug_off, -1, kInterleaved), h->pl.n_gauss, nrhs, st));
  }
  if (opts && opts->iters_out) *opts->iters_out = 0;
  if (opts && opts->resid_out) *opts->resid_out = 0.0;
  HIPCHK(hipStreamSynchronize(st));
  return HPS_OK;
}

int hps_set_error(int code, const char *msg) { return fail(code, msg); }

extern "C" int hps_solve(hps_handle *h, const double *f, const double *g, int nrhs, double *u,
                         const hps_solve_opts *opts) {
  if (!h || !f || !g || !u) return fail(HPS_EINVAL, "NULL argument");
  if (nrhs <= 0) return fail(HPS_EINVAL, "nrhs must be positive");
  hipStream_t st = opts ? (hipStream_t)opts->stream : nullptr;
  const int prec = opts ? opts->precision : HPS_PREC_FP64;
  int rc;
  if (prec == HPS_PREC_MIXED) {
    rc = solve_ext_mixed(h, f, g, nrhs, u, opts, st);
  } else {
    rc = hps_solve_pass(h, f, g, nrhs, u, prec == HPS_PREC_FP32 ? 1 : 0, nullptr, st);
  }
  if (rc) return rc;
  if (opts && opts->u_gauss) {
    Bases bs = make_bases(h);
    bs.d[BUF_IN0] = opts->u_gauss;
    HIPCHK(launch_copy_map(bs, vref(BUF_IN0, 0, -1, h->pl.n_gauss),
                           vref(BUF_VEC, h->ug_off, -1, kInterleaved), h->pl.n_gauss, nrhs, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  return HPS_OK;
}

// ---------------------------------------------------------------------------
// test hooks (include/hps_debug.h)
// ---------------------------------------------------------------------------
extern "C" int hps_debug_gemm_variant(int variant, int M, int N, int K, double alpha,
                                      const double *A, int lda, const double *B, int ldb,
                                      double *C, int ldc, void *stream) {
  if (M <= 0 || N <= 0 || K < 0 || !A || !B || !C) return fail(HPS_EINVAL, "bad gemm arguments");
  if (variant < 0 || variant >= kGemmVariants) return fail(HPS_EINVAL, "no such GEMM variant");
  hipStream_t st = (hipStream_t)stream;
  GemmList gl;
  GemmDesc g{};
  g.M = M; g.N = N; g.K = K;
  g.A = ref(BUF_IN0, 0, lda); g.B = ref(BUF_IN1, 0, ldb); g.C = ref(BUF_IN2, 0, ldc);
  g.D = noref(); g.crow = g.ccol = -1; g.alpha = alpha; g.beta = 0.0;
  gl.add(g, gemm_variant_tm(variant), gemm_variant_tn(variant));
  DevArray<GemmDesc> dd;
  DevArray<int32_t> dt;
  HIPCHK(dd.upload(gl.d));
  HIPCHK(dt.upload(gl.tmap));
  Bases bs{};
  bs.d[BUF_IN0] = (void *)A; bs.d[BUF_IN1] = (void *)B; bs.d[BUF_IN2] = (void *)C;
  HIPCHK(launch_gemm(variant, dd.p, dt.p, gl.tiles, bs, st));
  HIPCHK(hipStreamSynchronize(st));
  return HPS_OK;
}

extern "C" int hps_debug_gemm(int M, int N, int K, double alpha, const double *A, int lda,
                              const double *B, int ldb, double *C, int ldc, void *stream) {
  return hps_debug_gemm_variant(0, M, N, K, alpha, A, lda, B, ldb, C, ldc, stream);
}

extern "C" int hps_debug_invert(int n, int batch, const double *A, double *X, void *stream) {
  if (n <= 0 || batch <= 0 || !A || !X) return fail(HPS_EINVAL, "bad invert arguments");
  if (n > 2048) return fail(HPS_EINVAL, "n > 2048");
  hipStream_t st = (hipStream_t)stream;
  hps_handle H;
  const int64_t nn = int64_t(n) * n;
  // ws: [A copies][zero block][X]
  HIPCHK(H.ws.alloc(size_t(nn) * (2 * batch + 1)));
  HIPCHK(hipMemcpyAsync(H.ws.p, A, sizeof(double) * nn * batch, hipMemcpyDeviceToDevice, st));
  HIPCHK(launch_fill(H.ws.p + nn * batch, 0.0, nn, st));
  const int64_t wsz = std::max<int64_t>(int64_t(kPanelNBMax) * n, nn);
  HIPCHK(H.scr.alloc(size_t(wsz) * batch + 64));
  HIPCHK(H.ipiv.alloc(size_t(gj_int_scratch(n)) * batch));
  HIPCHK(H.psrc.alloc(size_t(n) * batch));
  HIPCHK(H.info.alloc(batch));
  HIPCHK(hipMemsetAsync(H.info.p, 0, sizeof(int32_t) * batch, st));
  std::vector<MergeInvDesc> lev, minv;
  for (int b = 0; b < batch; ++b) {
    MergeInvDesc d{};
    d.Ta = nn * b; d.Tb = nn * batch; d.lda = n; d.ldb = n; d.m = n; d.info = b;
    d.X = nn * (batch + 1 + b); d.W = wsz * b; d.ipiv = gj_int_scratch(n) * b;
    lev.push_back(d);
  }
  GemmList gl;
  std::vector<Step> prog;
  emit_inverse_steps(lev, minv, prog);
  HIPCHK(H.d_minv.upload(minv));

  Bases bs = make_bases(&H);
  int rc = run_prog(&H, prog, bs, 1, 0, st);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(X, H.ws.p + nn * (batch + 1), sizeof(double) * nn * batch,
                        hipMemcpyDeviceToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  std::vector<int32_t> info(batch);
  HIPCHK(hipMemcpy(info.data(), H.info.p, sizeof(int32_t) * batch, hipMemcpyDeviceToHost));
  for (int b = 0; b < batch; ++b) {
    if (info[b] > 0) return fail(HPS_ESINGULAR, "zero pivot in matrix " + std::to_string(b));
    if (info[b] < 0) return fail(HPS_ENONFINITE, "non-finite pivot in matrix " + std::to_string(b));
  }
  return HPS_OK;
}

extern "C" int hps_debug_gemm_choices(const hps_handle *h, int *out, int max_n, int *count) {
  if (!h || !count) return fail(HPS_EINVAL, "NULL argument");
  int n = 0;
  for (const Step &s : h->build_prog)
    if (s.kind == S_GEMM) {
      if (out && n < max_n) out[n] = s.var;
      ++n;
    }
  *count = n;
  return HPS_OK;
}

extern "C" size_t hps_debug_solve_work_bytes(const hps_handle *h, int nrhs) {
  if (!h || nrhs <= 0) return 0;
  return size_t(solve_work_elems(h, nrhs)) * sizeof(double);
}

extern "C" int hps_debug_boxes(const hps_handle *h, int *n_boxes, int32_t *out) {
  if (!h || !n_boxes) return fail(HPS_EINVAL, "NULL argument");
  *n_boxes = (int)h->pl.boxes.size();
  if (!out) return HPS_OK;
  for (size_t i = 0; i < h->pl.boxes.size(); ++i) {
    const Box &b = h->pl.boxes[i];
    int32_t *o = out + 8 * i;
    o[0] = b.leaf; o[1] = b.leaf_index; o[2] = b.parent; o[3] = b.alpha; o[4] = b.beta;
    o[5] = (int32_t)b.fin.size(); o[6] = (int32_t)b.nat.size(); o[7] = (int32_t)b.gi.size();
  }
  return HPS_OK;
}

extern "C" int hps_debug_box_nodes(const hps_handle *h, int box, int which, int64_t *out) {
  if (!h || !out || box < 0 || box >= (int)h->pl.boxes.size()) return fail(HPS_EINVAL, "bad box");
  const Box &b = h->pl.boxes[box];
  const std::vector<int64_t> &v = which == 0 ? b.fin : which == 1 ? b.nat : b.gi;
  std::copy(v.begin(), v.end(), out);
  return HPS_OK;
}

extern "C" int hps_debug_box_op(const hps_handle *h, int box, int which, double *out,
                                int64_t *count) {
  if (!h || box < 0 || box >= (int)h->pl.boxes.size()) return fail(HPS_EINVAL, "bad box");
  const Box &b = h->pl.boxes[box];
  const int64_t ef = (int64_t)b.fin.size(), en = (int64_t)b.nat.size(), m = (int64_t)b.gi.size();
  const int64_t mi = h->mi, g4 = h->g4;
  int64_t off = -1, n = 0;
  switch (which) {
    case 0: off = h->off_T[box]; n = ef * ef; break;
    case 1: off = h->off_X[box]; n = m * m; break;
    case 2:
      if (b.leaf) { off = h->off_LD[box]; n = mi * g4; }
      else { off = h->off_S[box]; n = m * en; }
      break;
    case 3: if (b.leaf) { off = h->off_LD[box] + g4 * mi; n = mi * mi; } break;
    case 4: if (b.leaf) { off = h->off_H[box]; n = g4 * mi; } break;
    default: break;
  }
  if (off < 0) return fail(HPS_EINVAL, "operator not stored for this box");
  if (count) *count = n;
  if (out) HIPCHK(hipMemcpy(out, h->ws.p + off, sizeof(double) * n, hipMemcpyDeviceToHost));
  return HPS_OK;
}

extern "C" int hps_debug_profile(hps_handle *h, int enable) {
  if (!h) return fail(HPS_EINVAL, "NULL handle");
  h->prof_on = enable != 0;
  h->prof_ev.clear();
  h->prof_work.clear();
  h->prof_used = 0;
  return HPS_OK;
}

extern "C" int hps_debug_profile_read(hps_handle *h, int *kinds, double *ms, double *work,
                                      int max_n, int *count) {
  if (!h || !count) return fail(HPS_EINVAL, "NULL argument");
  HIPCHK(hipDeviceSynchronize());
  const int n = std::min<int>(max_n, (int)h->prof_ev.size());
  for (int i = 0; i < n; ++i) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, h->prof_ev[i].second.first, h->prof_ev[i].second.second));
    kinds[i] = h->prof_ev[i].first;
    ms[i] = t;
    if (work) work[i] = h->prof_work[i];
  }
  *count = (int)h->prof_ev.size();
  h->prof_ev.clear();
  h->prof_work.clear();
  h->prof_used = 0;
  return HPS_OK;
}
