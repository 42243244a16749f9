// Host planner: box tree, Gauss node numbering, merge index maps, refined
// interface operators and the device workspace layout.
//
// Paper: Sec. 2 / Fig. 1 (binary tree, parent before child), Sec. 4 and its
// figure (J1, J2, J3), Sec. 5.1 (global Gauss vector), Sec. 6.1 (refinement
// criterion), Sec. 6.2-6.4 (neighbours, P_up / P_down).
//
// Side conditions (Sec. 7.6): every side of a problem is Dirichlet, Neumann
// or periodic (opposite pairs).  A periodic pair shares one set of Gauss
// nodes (the east / north segments are stored as the west / south ones), so
// the seam is eliminated by the merge whose children meet across it: the box
// spanning the whole periodic width, cut across it, whose children then each
// carry two shared blocks (the cut, then the seam).  A problem with Neumann
// sides gets one more box above its root (kind 3, no beta) whose interior
// nodes are the Neumann nodes: its "merge" with a zero-T sibling solves the
// root's flux relation on them.
//
// Orders used on the device (all matrices column-major):
//  * a box's "natural" boundary order: leaf S,E,N,W; parent J1 then J2;
//  * its "final" order: the nodes it keeps after its parent's merge first,
//    then the nodes it shares with its sibling, sorted along the shared side.
//    A child's shared block is exactly J3 of the parent, so every merge block
//    T11, T13, T31, T33 is a contiguous sub-matrix.
#pragma once
#include <cstdint>
#include <map>
#include <set>
#include <string>
#include <tuple>
#include <vector>

namespace hps {

constexpr int64_t kUnit = int64_t(1) << 24;  // integer units per base-leaf side

struct QuadLeaf {
  int64_t ix, iy, w, h;
  int depth;
  bool operator<(const QuadLeaf &o) const {
    return std::tie(ix, iy, w, h, depth) < std::tie(o.ix, o.iy, o.w, o.h, o.depth);
  }
};

enum { kBcDirichlet = 0, kBcNeumann = 1, kBcPeriodic = 2 };

struct Problem {
  double X0, X1, Y0, Y1;
  int nx, ny;
  std::set<QuadLeaf> leaves;
  int bc[4] = {kBcDirichlet, kBcDirichlet, kBcDirichlet, kBcDirichlet};  // S, E, N, W
};

struct TreeDesc {
  std::vector<Problem> probs;
};

struct Box {
  int problem = 0;
  int64_t ix0 = 0, ix1 = 0, iy0 = 0, iy1 = 0;
  int kind = 0;  // 0 base region, 1 refined quad box, 2 half of a quad box,
                 // 3 Neumann closure above a root (alpha = root, no beta)
  int depth = 0;
  int parent = -1, alpha = -1, beta = -1;
  char cut = 0;
  bool leaf = false;
  int height = 0;
  int leaf_index = -1;   // canonical index for leaves
  int role = 4;          // leaf: the side shared with the sibling (0..3) or 4
  // Gauss bookkeeping
  std::vector<int64_t> nat;   // natural order (fine)
  std::vector<int64_t> fin;   // final order (coarse when coarsened)
  std::vector<int64_t> gi;    // parent: interior nodes, sorted along the edge
  int n_shared = 0;           // shared block length at the end of fin
  bool coarsened = false;
  std::vector<int> pi;        // natural index -> final index (not coarsened)
  std::vector<double> Pup;    // coarsened: col-major nat x fin
  std::vector<double> Pdn;    // coarsened: col-major fin x nat
  std::vector<int> slave_rows;  // rows of nat replaced by P_up
};

struct Segment {
  int problem;
  char orient;  // 'h' (y fixed) or 'v' (x fixed)
  int64_t fixed, s0, s1;
};

// Everything the device needs, derived from the tree for a given (p, q).
struct Plan {
  int p = 0, q = 0, mi = 0, me = 0, g4 = 0;
  std::vector<Box> boxes;           // pre-order numbering
  std::vector<int> leaves;          // canonical leaf order -> box id
  std::vector<Segment> segs;
  int64_t n_gauss = 0;
  std::vector<int64_t> bdry;        // canonical boundary node ids
  std::vector<int8_t> bdry_kind;    // kBc* of each canonical boundary entry
  bool general_bc = false;          // some side is not Dirichlet
  std::vector<double> node_xy;      // [n_gauss][2]
  int max_height = 0;
  // leaf size classes
  std::vector<std::pair<double, double>> size_class;  // (hx, hy)
  std::vector<int> leaf_class;      // per canonical leaf
};

std::string build_tree_boxes(const TreeDesc &t, Plan &pl);
std::string plan_gauss(const TreeDesc &t, Plan &pl, int q);
void leaf_phys(const TreeDesc &t, const Box &b, double &x0, double &x1,
               double &y0, double &y1);
std::string refine_point(TreeDesc &t, int problem, double px, double py,
                         int n_ref, double tfac);
std::string set_bc(TreeDesc &t, int problem, const int bc[4]);

}  // namespace hps
