#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <functional>
#include <map>
#include <unordered_map>

#include "spectral.hpp"

namespace hps {

namespace {

struct SideRef {
  char orient;
  int64_t fixed, lo, hi;
};

// side s of a box: 0 S, 1 E, 2 N, 3 W
SideRef box_side(const Box &b, int s) {
  switch (s) {
    case 0: return {'h', b.iy0, b.ix0, b.ix1};
    case 1: return {'v', b.ix1, b.iy0, b.iy1};
    case 2: return {'h', b.iy1, b.ix0, b.ix1};
    default: return {'v', b.ix0, b.iy0, b.iy1};
  }
}

using SegKey = std::tuple<int, char, int64_t, int64_t, int64_t>;

}  // namespace

void leaf_phys(const TreeDesc &t, const Box &b, double &x0, double &x1,
               double &y0, double &y1) {
  const Problem &P = t.probs[b.problem];
  const double W = double(P.nx) * double(kUnit), H = double(P.ny) * double(kUnit);
  x0 = P.X0 + (P.X1 - P.X0) * (double(b.ix0) / W);
  x1 = P.X0 + (P.X1 - P.X0) * (double(b.ix1) / W);
  y0 = P.Y0 + (P.Y1 - P.Y0) * (double(b.iy0) / H);
  y1 = P.Y0 + (P.Y1 - P.Y0) * (double(b.iy1) / H);
}

std::string refine_point(TreeDesc &t, int problem, double px, double py,
                         int n_ref, double tfac) {
  if (problem < 0 || problem >= (int)t.probs.size()) return "bad problem index";
  Problem &P = t.probs[problem];
  const double sx = (P.X1 - P.X0) / (double(P.nx) * double(kUnit));
  const double sy = (P.Y1 - P.Y0) / (double(P.ny) * double(kUnit));
  for (int r = 0; r < n_ref; ++r) {
    std::set<QuadLeaf> nw;
    for (const QuadLeaf &L : P.leaves) {
      double x0 = P.X0 + L.ix * sx, x1 = P.X0 + (L.ix + L.w) * sx;
      double y0 = P.Y0 + L.iy * sy, y1 = P.Y0 + (L.iy + L.h) * sy;
      double dx = std::max({x0 - px, 0.0, px - x1});
      double dy = std::max({y0 - py, 0.0, py - y1});
      double dist = std::hypot(dx, dy);
      double half = 0.5 * std::max(x1 - x0, y1 - y0);
      if (dist <= tfac * half && L.w >= 2 && L.h >= 2) {
        int64_t hw = L.w / 2, hh = L.h / 2;
        nw.insert({L.ix, L.iy, hw, hh, L.depth + 1});
        nw.insert({L.ix + hw, L.iy, hw, hh, L.depth + 1});
        nw.insert({L.ix, L.iy + hh, hw, hh, L.depth + 1});
        nw.insert({L.ix + hw, L.iy + hh, hw, hh, L.depth + 1});
      } else {
        nw.insert(L);
      }
    }
    P.leaves.swap(nw);
  }
  return "";
}

std::string set_bc(TreeDesc &t, int problem, const int bc[4]) {
  for (int s = 0; s < 4; ++s)
    if (bc[s] < kBcDirichlet || bc[s] > kBcPeriodic) return "unknown side condition";
  if ((bc[1] == kBcPeriodic) != (bc[3] == kBcPeriodic) ||
      (bc[0] == kBcPeriodic) != (bc[2] == kBcPeriodic))
    return "periodic sides come in opposite pairs";
  if (problem < -1 || problem >= (int)t.probs.size()) return "bad problem index";
  for (int k = 0; k < (int)t.probs.size(); ++k)
    if (problem < 0 || k == problem)
      for (int s = 0; s < 4; ++s) t.probs[k].bc[s] = bc[s];
  return "";
}

std::string build_tree_boxes(const TreeDesc &t, Plan &pl) {
  pl.boxes.clear();
  pl.general_bc = false;
  for (const Problem &P : t.probs) {
    const int64_t W = int64_t(P.nx) * kUnit, H = int64_t(P.ny) * kUnit;
    for (int s = 0; s < 4; ++s) pl.general_bc |= P.bc[s] != kBcDirichlet;
    // the box that closes a periodic seam must have two children that are
    // not leaves (a leaf has one shared side)
    if ((P.bc[1] == kBcPeriodic && P.nx < 4) || (P.bc[0] == kBcPeriodic && P.ny < 4))
      return "a periodic direction needs at least 4 leaves";
    for (const QuadLeaf &L : P.leaves)
      if (L.depth > 0 && ((P.bc[1] == kBcPeriodic && (L.ix == 0 || L.ix + L.w == W)) ||
                          (P.bc[0] == kBcPeriodic && (L.iy == 0 || L.iy + L.h == H))))
        return "refined leaves on a periodic side";
  }
  std::function<int(int, int64_t, int64_t, int64_t, int64_t, int, int)> make =
      [&](int prob, int64_t ix0, int64_t ix1, int64_t iy0, int64_t iy1,
          int kind, int depth) -> int {
    int id = (int)pl.boxes.size();
    pl.boxes.emplace_back();
    {
      Box &b = pl.boxes[id];
      b.problem = prob;
      b.ix0 = ix0; b.ix1 = ix1; b.iy0 = iy0; b.iy1 = iy1;
      b.kind = kind; b.depth = depth;
    }
    const int64_t w = ix1 - ix0, h = iy1 - iy0;
    const auto &lv = t.probs[prob].leaves;
    if (kind != 2 && lv.count(QuadLeaf{ix0, iy0, w, h, depth})) {
      pl.boxes[id].leaf = true;
      return id;
    }
    int a, c;
    if (kind == 0 && (w > kUnit || h > kUnit)) {
      int64_t bx = w / kUnit, by = h / kUnit;
      if (bx >= by && bx > 1) {
        int64_t xm = ix0 + (bx / 2) * kUnit;
        pl.boxes[id].cut = 'x';
        a = make(prob, ix0, xm, iy0, iy1, 0, 0);
        c = make(prob, xm, ix1, iy0, iy1, 0, 0);
      } else {
        int64_t ym = iy0 + (by / 2) * kUnit;
        pl.boxes[id].cut = 'y';
        a = make(prob, ix0, ix1, iy0, ym, 0, 0);
        c = make(prob, ix0, ix1, ym, iy1, 0, 0);
      }
    } else if (kind != 2) {
      if (w < 2 || h < 2) return -1;
      int64_t xm = ix0 + w / 2;
      pl.boxes[id].cut = 'x';
      a = make(prob, ix0, xm, iy0, iy1, 2, depth);
      c = make(prob, xm, ix1, iy0, iy1, 2, depth);
    } else {
      int64_t ym = iy0 + h / 2;
      pl.boxes[id].cut = 'y';
      a = make(prob, ix0, ix1, iy0, ym, 1, depth + 1);
      c = make(prob, ix0, ix1, ym, iy1, 1, depth + 1);
    }
    if (a < 0 || c < 0) return -1;
    pl.boxes[id].alpha = a;
    pl.boxes[id].beta = c;
    pl.boxes[a].parent = id;
    pl.boxes[c].parent = id;
    return id;
  };
  for (int pi = 0; pi < (int)t.probs.size(); ++pi) {
    const Problem &P = t.probs[pi];
    const int64_t W = int64_t(P.nx) * kUnit, H = int64_t(P.ny) * kUnit;
    bool neumann = false;
    for (int s = 0; s < 4; ++s) neumann |= P.bc[s] == kBcNeumann;
    int clo = -1;
    if (neumann) {                      // the closure box precedes its root
      clo = (int)pl.boxes.size();
      pl.boxes.emplace_back();
      Box &c = pl.boxes[clo];
      c.problem = pi;
      c.ix1 = W; c.iy1 = H;
      c.kind = 3;
    }
    const int r = make(pi, 0, W, 0, H, 0, 0);
    if (r < 0) return "tree construction failed";
    if (clo >= 0) {
      if (pl.boxes[r].leaf) return "a problem with a Neumann side needs at least two leaves";
      pl.boxes[clo].alpha = r;
      pl.boxes[r].parent = clo;
    }
  }
  // canonical leaves
  pl.leaves.clear();
  for (int i = 0; i < (int)pl.boxes.size(); ++i)
    if (pl.boxes[i].leaf) pl.leaves.push_back(i);
  std::sort(pl.leaves.begin(), pl.leaves.end(), [&](int a, int b) {
    const Box &A = pl.boxes[a], &B = pl.boxes[b];
    return std::tie(A.problem, A.iy0, A.ix0) < std::tie(B.problem, B.iy0, B.ix0);
  });
  for (int i = 0; i < (int)pl.leaves.size(); ++i)
    pl.boxes[pl.leaves[i]].leaf_index = i;
  // heights
  pl.max_height = 0;
  for (int i = (int)pl.boxes.size() - 1; i >= 0; --i) {
    Box &b = pl.boxes[i];
    b.height = b.leaf ? 0
                      : 1 + std::max(pl.boxes[b.alpha].height,
                                     b.beta >= 0 ? pl.boxes[b.beta].height : 0);
    pl.max_height = std::max(pl.max_height, b.height);
  }
  return "";
}

std::string plan_gauss(const TreeDesc &t, Plan &pl, int q) {
  pl.q = q;
  const std::vector<double> g = legendre_roots(q);
  std::map<SegKey, int> seg_id;
  pl.segs.clear();
  // a periodic pair is one set of nodes: east sides onto west, north onto south
  auto norm = [&](int prob, SideRef s) {
    const Problem &P = t.probs[prob];
    if (s.orient == 'v' && P.bc[1] == kBcPeriodic && s.fixed == int64_t(P.nx) * kUnit) s.fixed = 0;
    if (s.orient == 'h' && P.bc[2] == kBcPeriodic && s.fixed == int64_t(P.ny) * kUnit) s.fixed = 0;
    return s;
  };
  auto seg = [&](int prob, SideRef s) {
    s = norm(prob, s);
    SegKey k{prob, s.orient, s.fixed, s.lo, s.hi};
    auto it = seg_id.find(k);
    if (it != seg_id.end()) return it->second;
    int id = (int)pl.segs.size();
    seg_id[k] = id;
    pl.segs.push_back({prob, s.orient, s.fixed, s.lo, s.hi});
    return id;
  };
  for (int li : pl.leaves)
    for (int s = 0; s < 4; ++s) seg(pl.boxes[li].problem, box_side(pl.boxes[li], s));
  pl.n_gauss = int64_t(pl.segs.size()) * q;
  auto node_t = [&](int64_t j) {
    const Segment &S = pl.segs[j / q];
    return double(S.s0) + double(S.s1 - S.s0) * (g[j % q] + 1.0) / 2.0;
  };
  auto on_side = [&](int64_t j, int prob, SideRef s) {
    s = norm(prob, s);
    const Segment &S = pl.segs[j / q];
    return S.problem == prob && S.orient == s.orient && S.fixed == s.fixed &&
           S.s0 >= s.lo && S.s1 <= s.hi;
  };
  pl.node_xy.assign(size_t(pl.n_gauss) * 2, 0.0);
  for (int64_t j = 0; j < pl.n_gauss; ++j) {
    const Segment &S = pl.segs[j / q];
    const Problem &P = t.probs[S.problem];
    const double W = double(P.nx) * double(kUnit), H = double(P.ny) * double(kUnit);
    double tt = node_t(j);
    double x, y;
    if (S.orient == 'h') {
      x = P.X0 + (P.X1 - P.X0) * (tt / W);
      y = P.Y0 + (P.Y1 - P.Y0) * (double(S.fixed) / H);
    } else {
      x = P.X0 + (P.X1 - P.X0) * (double(S.fixed) / W);
      y = P.Y0 + (P.Y1 - P.Y0) * (tt / H);
    }
    pl.node_xy[2 * j] = x;
    pl.node_xy[2 * j + 1] = y;
  }
  // unrefined leaves of every problem, by position and size
  std::vector<std::set<std::tuple<int64_t, int64_t, int64_t, int64_t>>> quads(t.probs.size());
  for (size_t pi = 0; pi < t.probs.size(); ++pi)
    for (const QuadLeaf &L : t.probs[pi].leaves) quads[pi].insert({L.ix, L.iy, L.w, L.h});

  // sides whose nodes a box shares with its sibling, in block order: the
  // side facing the sibling, then the periodic seam when the parent spans the
  // whole periodic width across its cut; below a closure box, the Neumann
  // sides in the order S, E, N, W
  auto shared_sides = [&](int id) -> std::vector<int> {
    const Box &b = pl.boxes[id];
    if (b.parent < 0) return {};
    const Box &P = pl.boxes[b.parent];
    const Problem &Pr = t.probs[b.problem];
    std::vector<int> v;
    if (P.kind == 3) {
      for (int s = 0; s < 4; ++s)
        if (Pr.bc[s] == kBcNeumann) v.push_back(s);
      return v;
    }
    const bool is_a = P.alpha == id;
    if (P.cut == 'x') {
      v.push_back(is_a ? 1 : 3);
      if (Pr.bc[1] == kBcPeriodic && P.ix0 == 0 && P.ix1 == int64_t(Pr.nx) * kUnit)
        v.push_back(is_a ? 3 : 1);
    } else {
      v.push_back(is_a ? 2 : 0);
      if (Pr.bc[2] == kBcPeriodic && P.iy0 == 0 && P.iy1 == int64_t(Pr.ny) * kUnit)
        v.push_back(is_a ? 0 : 2);
    }
    return v;
  };
  // split cur into the kept nodes and the shared block (each side's nodes
  // sorted along it)
  auto split_shared = [&](int id, const std::vector<int64_t> &cur, std::vector<int64_t> &keep,
                          std::vector<int64_t> &sh) {
    const Box &b = pl.boxes[id];
    const std::vector<int> sides = shared_sides(id);
    keep.clear();
    sh.clear();
    std::vector<char> taken(cur.size(), 0);
    for (int sd : sides) {
      SideRef sr = box_side(b, sd);
      std::vector<int64_t> part;
      for (size_t a = 0; a < cur.size(); ++a)
        if (!taken[a] && on_side(cur[a], b.problem, sr)) {
          part.push_back(cur[a]);
          taken[a] = 1;
        }
      std::sort(part.begin(), part.end(), [&](int64_t a, int64_t c) { return node_t(a) < node_t(c); });
      sh.insert(sh.end(), part.begin(), part.end());
    }
    for (size_t a = 0; a < cur.size(); ++a)
      if (!taken[a]) keep.push_back(cur[a]);
    return (int)sides.size();
  };

  for (int id = (int)pl.boxes.size() - 1; id >= 0; --id) {
    Box &b = pl.boxes[id];
    std::vector<int64_t> cur;
    if (b.leaf) {
      for (int s = 0; s < 4; ++s) {
        int sg = seg(b.problem, box_side(b, s));
        for (int k = 0; k < q; ++k) cur.push_back(int64_t(sg) * q + k);
      }
      b.nat = cur;
    } else if (b.kind == 3) {
      // Neumann closure: the root's shared block (its Neumann nodes) is
      // interior, the rest of its boundary stays exterior
      const Box &A = pl.boxes[b.alpha];
      const int m = A.n_shared;
      if (m == 0) return "closure box without Neumann nodes";
      b.gi.assign(A.fin.end() - m, A.fin.end());
      cur.assign(A.fin.begin(), A.fin.end() - m);
      b.nat = cur;
    } else {
      const Box &A = pl.boxes[b.alpha], &B = pl.boxes[b.beta];
      if (A.n_shared != B.n_shared || A.n_shared == 0)
        return "merge with mismatched interface";
      const int m = A.n_shared;
      const size_t ea = A.fin.size(), eb = B.fin.size();
      for (int k = 0; k < m; ++k)
        if (A.fin[ea - m + k] != B.fin[eb - m + k])
          return "merge interface nodes do not match";
      b.gi.assign(A.fin.end() - m, A.fin.end());
      cur.assign(A.fin.begin(), A.fin.end() - m);
      cur.insert(cur.end(), B.fin.begin(), B.fin.end() - m);
      b.nat = cur;
      // Sec. 6.3: coarsen sides facing an unrefined same-size leaf
      const bool quadbox = b.kind == 1 ||
                           (b.kind == 0 && b.ix1 - b.ix0 == kUnit && b.iy1 - b.iy0 == kUnit);
      if (quadbox) {
        const int64_t w = b.ix1 - b.ix0, h = b.iy1 - b.iy0;
        const int64_t nb[4][2] = {{b.ix0, b.iy0 - h}, {b.ix1, b.iy0},
                                  {b.ix0, b.iy1}, {b.ix0 - w, b.iy0}};
        struct Blk { std::vector<int64_t> on, coarse; std::vector<double> pu, pd; };
        std::vector<Blk> blocks;
        for (int s = 0; s < 4; ++s) {
          if (!quads[b.problem].count({nb[s][0], nb[s][1], w, h})) continue;
          SideRef sr = norm(b.problem, box_side(b, s));
          auto it = seg_id.find(SegKey{b.problem, sr.orient, sr.fixed, sr.lo, sr.hi});
          if (it == seg_id.end()) continue;
          Blk bl;
          for (int64_t j : cur)
            if (on_side(j, b.problem, sr)) bl.on.push_back(j);
          for (int k = 0; k < q; ++k) bl.coarse.push_back(int64_t(it->second) * q + k);
          if (bl.on == bl.coarse) continue;
          const double lo = double(sr.lo), hi = double(sr.hi);
          std::vector<double> xf;
          for (int64_t j : bl.on) xf.push_back(2.0 * (node_t(j) - lo) / (hi - lo) - 1.0);
          std::vector<double> Pu = interp_matrix(g, xf);  // |on| x q row-major
          bl.pu = Pu;
          std::vector<int> panels;
          for (int64_t j : bl.on)
            if (panels.empty() || panels.back() != int(j / q)) panels.push_back(int(j / q));
          std::sort(panels.begin(), panels.end(), [&](int a, int c) {
            return pl.segs[a].s0 < pl.segs[c].s0;
          });
          panels.erase(std::unique(panels.begin(), panels.end()), panels.end());
          std::unordered_map<int64_t, int> col;
          for (size_t a = 0; a < bl.on.size(); ++a) col[bl.on[a]] = (int)a;
          bl.pd.assign(size_t(q) * bl.on.size(), 0.0);  // q x |on| row-major
          for (int k = 0; k < q; ++k) {
            double tc = lo + (hi - lo) * (g[k] + 1.0) / 2.0;
            double tol = 1e-12 * (hi - lo);
            std::vector<int> hits;
            for (int sg : panels)
              if (double(pl.segs[sg].s0) - tol <= tc && tc <= double(pl.segs[sg].s1) + tol)
                hits.push_back(sg);
            for (int sg : hits) {
              double s0 = double(pl.segs[sg].s0), s1 = double(pl.segs[sg].s1);
              std::vector<double> xi{2.0 * (tc - s0) / (s1 - s0) - 1.0};
              std::vector<double> row = interp_matrix(g, xi);
              for (int kk = 0; kk < q; ++kk)
                bl.pd[size_t(k) * bl.on.size() + col[int64_t(sg) * q + kk]] +=
                    row[kk] / double(hits.size());
            }
          }
          // replace the fine nodes by the coarse ones at the first position
          auto pos = std::find(cur.begin(), cur.end(), bl.on[0]) - cur.begin();
          std::set<int64_t> onset(bl.on.begin(), bl.on.end());
          std::vector<int64_t> nw;
          for (size_t a = 0; a < cur.size(); ++a) {
            if ((int64_t)a == pos) nw.insert(nw.end(), bl.coarse.begin(), bl.coarse.end());
            if (!onset.count(cur[a])) nw.push_back(cur[a]);
          }
          cur.swap(nw);
          blocks.push_back(std::move(bl));
        }
        if (!blocks.empty()) {
          b.coarsened = true;
          // final order, then P_up (nat x fin) and P_down (fin x nat)
          std::vector<int64_t> keep, sh;
          split_shared(id, cur, keep, sh);
          b.fin = keep;
          b.fin.insert(b.fin.end(), sh.begin(), sh.end());
          b.n_shared = (int)sh.size();
          const size_t en = b.nat.size(), ef = b.fin.size();
          std::unordered_map<int64_t, int> npos, fpos;
          for (size_t a = 0; a < en; ++a) npos[b.nat[a]] = (int)a;
          for (size_t a = 0; a < ef; ++a) fpos[b.fin[a]] = (int)a;
          b.Pup.assign(en * ef, 0.0);
          b.Pdn.assign(ef * en, 0.0);
          std::set<int64_t> slave, coarse;
          for (const Blk &bl : blocks) {
            for (size_t a = 0; a < bl.on.size(); ++a) {
              slave.insert(bl.on[a]);
              for (int k = 0; k < q; ++k)
                b.Pup[npos[bl.on[a]] + en * size_t(fpos[bl.coarse[k]])] = bl.pu[a * q + k];
            }
            for (int k = 0; k < q; ++k) {
              coarse.insert(bl.coarse[k]);
              for (size_t a = 0; a < bl.on.size(); ++a)
                b.Pdn[fpos[bl.coarse[k]] + ef * size_t(npos[bl.on[a]])] =
                    bl.pd[size_t(k) * bl.on.size() + a];
            }
          }
          for (size_t a = 0; a < en; ++a)
            if (!slave.count(b.nat[a])) b.Pup[a + en * size_t(fpos[b.nat[a]])] = 1.0;
            else b.slave_rows.push_back((int)a);
          for (size_t a = 0; a < ef; ++a)
            if (!coarse.count(b.fin[a])) b.Pdn[a + ef * size_t(npos[b.fin[a]])] = 1.0;
          continue;
        }
      }
    }
    // final order: kept nodes, then the side(s) shared with the sibling
    std::vector<int64_t> keep, sh;
    const int nsides = split_shared(id, cur, keep, sh);
    b.fin = keep;
    b.fin.insert(b.fin.end(), sh.begin(), sh.end());
    b.n_shared = (int)sh.size();
    if (b.leaf) {
      if (nsides > 1) return "a leaf would share two sides (a periodic direction needs 4 leaves)";
      b.role = nsides == 0 ? 4 : shared_sides(id)[0];
    }
    std::unordered_map<int64_t, int> fpos;
    for (size_t a = 0; a < b.fin.size(); ++a) fpos[b.fin[a]] = (int)a;
    b.pi.resize(b.nat.size());
    for (size_t a = 0; a < b.nat.size(); ++a) b.pi[a] = fpos[b.nat[a]];
  }
  // canonical domain boundary nodes (a periodic side lists the seam nodes
  // it shares with its partner)
  pl.bdry.clear();
  pl.bdry_kind.clear();
  for (int pi = 0; pi < (int)t.probs.size(); ++pi) {
    const Problem &P = t.probs[pi];
    const int64_t W = int64_t(P.nx) * kUnit, H = int64_t(P.ny) * kUnit;
    const std::pair<char, int64_t> sides[4] = {{'h', 0},
                                               {'v', P.bc[1] == kBcPeriodic ? 0 : W},
                                               {'h', P.bc[2] == kBcPeriodic ? 0 : H},
                                               {'v', 0}};
    for (int side = 0; side < 4; ++side) {
      const auto &sd = sides[side];
      std::vector<int> ss;
      for (int s = 0; s < (int)pl.segs.size(); ++s)
        if (pl.segs[s].problem == pi && pl.segs[s].orient == sd.first &&
            pl.segs[s].fixed == sd.second)
          ss.push_back(s);
      std::sort(ss.begin(), ss.end(), [&](int a, int c) { return pl.segs[a].s0 < pl.segs[c].s0; });
      for (int s : ss)
        for (int k = 0; k < q; ++k) {
          pl.bdry.push_back(int64_t(s) * q + k);
          pl.bdry_kind.push_back((int8_t)P.bc[side]);
        }
    }
  }
  // leaf size classes
  std::map<std::tuple<int, int64_t, int64_t>, int> cls;
  pl.size_class.clear();
  pl.leaf_class.assign(pl.leaves.size(), 0);
  for (size_t i = 0; i < pl.leaves.size(); ++i) {
    const Box &b = pl.boxes[pl.leaves[i]];
    auto key = std::make_tuple(b.problem, b.ix1 - b.ix0, b.iy1 - b.iy0);
    auto it = cls.find(key);
    if (it == cls.end()) {
      double x0, x1, y0, y1;
      leaf_phys(t, b, x0, x1, y0, y1);
      int c = (int)pl.size_class.size();
      cls[key] = c;
      pl.size_class.push_back({x1 - x0, y1 - y0});
      pl.leaf_class[i] = c;
    } else {
      pl.leaf_class[i] = it->second;
    }
  }
  return "";
}

}  // namespace hps
