// Host planner under AddressSanitizer / UndefinedBehaviorSanitizer: builds the
// boxes and Gauss bookkeeping of uniform, rectangular, multi-problem and
// refined trees and checks their invariants.  Built with g++ by
// test_planner_sanitized.py (host code only, no device code).
#include <cstdio>
#include <cstdlib>
#include <set>
#include <string>

#include "../paper_1612_02736_amd/csrc/plan.hpp"

using namespace hps;

static int fails = 0;
#define CHECK(c, ...)                                        \
  do {                                                       \
    if (!(c)) {                                              \
      std::fprintf(stderr, "check failed: %s: ", #c);        \
      std::fprintf(stderr, __VA_ARGS__);                     \
      std::fprintf(stderr, "\n");                            \
      ++fails;                                               \
    }                                                        \
  } while (0)

static TreeDesc uniform(int nx, int ny, int nprob) {
  TreeDesc t;
  for (int k = 0; k < nprob; ++k) {
    Problem P;
    P.X0 = 0.0; P.X1 = 1.0; P.Y0 = 0.0; P.Y1 = 1.0; P.nx = nx; P.ny = ny;
    for (int i = 0; i < nx; ++i)
      for (int j = 0; j < ny; ++j) P.leaves.insert({i * kUnit, j * kUnit, kUnit, kUnit, 0});
    t.probs.push_back(P);
  }
  return t;
}

// expect_leaves / expect_bdry: the leaf and boundary node counts the tree must
// have (-1: not checked)
static void check_plan(const char *name, const TreeDesc &t, int q, int expect_leaves = -1,
                       long expect_bdry = -1) {
  Plan pl;
  std::string e = build_tree_boxes(t, pl);
  CHECK(e.empty(), "%s: build_tree_boxes: %s", name, e.c_str());
  e = plan_gauss(t, pl, q);
  CHECK(e.empty(), "%s: plan_gauss: %s", name, e.c_str());
  if (!e.empty()) return;
  const int nb = (int)pl.boxes.size();
  int nleaf = 0;
  for (int b = 0; b < nb; ++b) {
    const Box &B = pl.boxes[b];
    if (B.leaf) {
      ++nleaf;
      CHECK(B.nat.size() == size_t(4 * q), "%s: leaf %d has %zu Gauss nodes", name, b,
            B.nat.size());
      continue;
    }
    CHECK(B.alpha > b && B.beta > b, "%s: children of %d come after it", name, b);
    const Box &A = pl.boxes[B.alpha], &C = pl.boxes[B.beta];
    CHECK(A.parent == b && C.parent == b, "%s: parent links of %d", name, b);
    // a merge's nodes: its children's minus the shared interface, once each
    const size_t m = B.gi.size();
    CHECK(m > 0, "%s: merge %d has an empty interface", name, b);
    CHECK(A.fin.size() >= m && C.fin.size() >= m, "%s: interface of %d too long", name, b);
    std::set<int64_t> gi(B.gi.begin(), B.gi.end());
    CHECK(gi.size() == m, "%s: repeated interface nodes at %d", name, b);
    for (int64_t v : B.nat) {
      CHECK(v >= 0 && v < pl.n_gauss, "%s: node id out of range at %d", name, b);
      CHECK(!gi.count(v), "%s: interface node %lld also exterior at %d", name, (long long)v, b);
    }
    CHECK(B.height == 1 + std::max(A.height, C.height), "%s: height of %d", name, b);
  }
  CHECK(nleaf == (int)pl.leaves.size(), "%s: leaf list", name);
  CHECK(expect_leaves < 0 || nleaf == expect_leaves, "%s: %d leaves, expected %d", name, nleaf,
        expect_leaves);
  CHECK(expect_bdry < 0 || (long)pl.bdry.size() == expect_bdry,
        "%s: %zu boundary nodes, expected %ld", name, pl.bdry.size(), expect_bdry);
  std::set<int64_t> bd(pl.bdry.begin(), pl.bdry.end());
  CHECK(bd.size() == pl.bdry.size(), "%s: repeated boundary nodes", name);
  CHECK(pl.node_xy.size() == size_t(2 * pl.n_gauss), "%s: node coordinates", name);
  std::printf("%s: %d boxes, %d leaves, %lld Gauss nodes, %zu on the boundary\n", name, nb,
              nleaf, (long long)pl.n_gauss, pl.bdry.size());
}

int main() {
  // a uniform nx x ny grid has 2 (nx + ny) q boundary Gauss nodes per problem
  check_plan("1x1", uniform(1, 1, 1), 7, 1, 4 * 7);
  check_plan("4x4", uniform(4, 4, 1), 15, 16, 16 * 15);
  check_plan("3x5", uniform(3, 5, 1), 9, 15, 16 * 9);
  check_plan("64x64", uniform(64, 64, 1), 15, 4096, 256 * 15);
  check_plan("forest 8 of 2x3", uniform(2, 3, 8), 11, 48, 8 * 10 * 11);
  {
    TreeDesc t = uniform(4, 4, 1);
    std::string e = refine_point(t, 0, 0.25, 0.75, 1, 1.4142135623730951);
    CHECK(e.empty(), "refine: %s", e.c_str());
    // the 4 leaves touching the vertex split into 4 each: 12 + 16 = 28 leaves
    // (the leaf count of the concentrated-load experiment, Sec. 7.3)
    check_plan("4x4 refined once at a vertex", t, 15, 28);
  }
  {
    TreeDesc t = uniform(4, 4, 3);
    for (int k = 0; k < 3; ++k) {
      std::string e = refine_point(t, k, 0.1 + 0.3 * k, 0.8 - 0.25 * k, 2 + 2 * k,
                                   1.4142135623730951);
      CHECK(e.empty(), "refine %d: %s", k, e.c_str());
    }
    check_plan("forest of 3, refined 2, 4, 6 levels", t, 13);
  }
  {
    TreeDesc t = uniform(4, 4, 1);
    std::string e = refine_point(t, 0, 0.3, 0.6, 8, 1.4142135623730951);
    CHECK(e.empty(), "refine: %s", e.c_str());
    check_plan("4x4 refined 8 levels", t, 14);
  }
  {
    TreeDesc t = uniform(2, 2, 1);
    std::string e = refine_point(t, 5, 0.5, 0.5, 1, 1.0);
    CHECK(!e.empty(), "refining a problem that does not exist must fail");
  }
  if (fails) std::fprintf(stderr, "%d checks failed\n", fails);
  else std::printf("all checks passed\n");
  return fails ? 1 : 0;
}
