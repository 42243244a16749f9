// Host planner under AddressSanitizer / UndefinedBehaviorSanitizer: builds the
// boxes and Gauss bookkeeping of uniform, rectangular, multi-problem and
// refined trees and checks their invariants.  Built with g++ by
// test_planner_sanitized.py (host code only, no device code).
#include <cstdio>
#include <cstdlib>
#include <map>
#include <set>
#include <string>
#include <vector>

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
  std::map<int64_t, int> elim;     // times each node is interior to a box
  std::set<int64_t> slave;         // fine nodes replaced on refined sides
  for (int b = 0; b < nb; ++b) {
    const Box &B = pl.boxes[b];
    for (int64_t v : B.gi) ++elim[v];
    for (int a : B.slave_rows) slave.insert(B.nat[a]);
    if (B.leaf) {
      ++nleaf;
      CHECK(B.nat.size() == size_t(4 * q), "%s: leaf %d has %zu Gauss nodes", name, b,
            B.nat.size());
      std::set<int64_t> own(B.nat.begin(), B.nat.end());
      CHECK(own.size() == B.nat.size(), "%s: leaf %d lists a node twice", name, b);
      continue;
    }
    if (B.kind == 3) {             // Neumann closure above a root
      CHECK(B.alpha > b && B.beta < 0 && B.parent < 0, "%s: closure links at %d", name, b);
      const Box &A = pl.boxes[B.alpha];
      CHECK(A.parent == b && A.n_shared > 0 && B.gi.size() == size_t(A.n_shared),
            "%s: closure interface at %d", name, b);
      CHECK(B.height == 1 + A.height, "%s: closure height at %d", name, b);
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
  // every node is eliminated once, unless it is Dirichlet data or a fine node
  // replaced on a refined side
  std::set<int64_t> dir;
  for (size_t k = 0; k < pl.bdry.size(); ++k)
    if (pl.bdry_kind[k] == kBcDirichlet) dir.insert(pl.bdry[k]);
  for (int li : pl.leaves)
    for (int64_t v : pl.boxes[li].nat) {
      const int want = (dir.count(v) || slave.count(v)) ? 0 : 1;
      CHECK(elim[v] == want, "%s: node %lld eliminated %d times", name, (long long)v, elim[v]);
    }
  CHECK(expect_leaves < 0 || nleaf == expect_leaves, "%s: %d leaves, expected %d", name, nleaf,
        expect_leaves);
  CHECK(expect_bdry < 0 || (long)pl.bdry.size() == expect_bdry,
        "%s: %zu boundary nodes, expected %ld", name, pl.bdry.size(), expect_bdry);
  // boundary entries name distinct nodes, except that the two sides of a
  // periodic pair name the same seam nodes
  std::set<int64_t> bd;
  size_t nonper = 0;
  std::map<int64_t, int> per;
  for (size_t k = 0; k < pl.bdry.size(); ++k) {
    if (pl.bdry_kind[k] == kBcPeriodic) {
      ++per[pl.bdry[k]];
      continue;
    }
    bd.insert(pl.bdry[k]);
    ++nonper;
  }
  CHECK(bd.size() == nonper, "%s: repeated boundary nodes", name);
  for (const auto &kv : per)
    CHECK(kv.second == 2 && !bd.count(kv.first), "%s: seam node %lld listed %d times", name,
          (long long)kv.first, kv.second);
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
  // side conditions: Neumann closures and periodic seams
  const int NPNP[4] = {kBcNeumann, kBcPeriodic, kBcNeumann, kBcPeriodic};
  const int PPPP[4] = {kBcPeriodic, kBcPeriodic, kBcPeriodic, kBcPeriodic};
  const int NNNN[4] = {kBcNeumann, kBcNeumann, kBcNeumann, kBcNeumann};
  const int DNDN[4] = {kBcDirichlet, kBcNeumann, kBcDirichlet, kBcNeumann};
  const int PDPD[4] = {kBcPeriodic, kBcDirichlet, kBcPeriodic, kBcDirichlet};
  const struct { const char *name; const int *bc; int nx, ny, q; } cases[] = {
      {"NPNP 4x4", NPNP, 4, 4, 14}, {"NPNP 16x16", NPNP, 16, 16, 14},
      {"NPNP 64x64", NPNP, 64, 64, 14}, {"PPPP 4x4", PPPP, 4, 4, 10},
      {"PPPP 5x7", PPPP, 5, 7, 9}, {"NNNN 3x5", NNNN, 3, 5, 9},
      {"DNDN 6x4", DNDN, 6, 4, 11}, {"PDPD 3x9", PDPD, 3, 9, 11}};
  for (const auto &c : cases) {
    TreeDesc t = uniform(c.nx, c.ny, 1);
    CHECK(set_bc(t, -1, c.bc).empty(), "%s: set_bc", c.name);
    check_plan(c.name, t, c.q, c.nx * c.ny, 2L * (c.nx + c.ny) * c.q);
  }
  {
    TreeDesc t = uniform(4, 4, 3);
    CHECK(set_bc(t, 0, NPNP).empty() && set_bc(t, 2, NNNN).empty(), "forest set_bc");
    std::string e = refine_point(t, 1, 0.3, 0.6, 3, 1.4142135623730951);
    e += refine_point(t, 2, 0.5, 0.5, 2, 1.4142135623730951);
    e += refine_point(t, 0, 0.5, 0.5, 1, 1.4142135623730951);   // away from the seam
    CHECK(e.empty(), "forest refine: %s", e.c_str());
    check_plan("forest NPNP / DDDD / NNNN, refined", t, 12);
  }
  {
    const int bad[4] = {kBcPeriodic, kBcDirichlet, kBcDirichlet, kBcDirichlet};
    TreeDesc t = uniform(4, 4, 1);
    CHECK(!set_bc(t, -1, bad).empty(), "an unpaired periodic side must be refused");
    TreeDesc t2 = uniform(3, 4, 1);
    set_bc(t2, -1, NPNP);
    Plan pl;
    CHECK(!build_tree_boxes(t2, pl).empty(), "3 leaves across a periodic direction must fail");
    TreeDesc t3 = uniform(4, 4, 1);
    set_bc(t3, -1, NPNP);
    refine_point(t3, 0, 0.01, 0.5, 1, 1.4142135623730951);
    CHECK(!build_tree_boxes(t3, pl).empty(), "refinement on a periodic side must fail");
  }
  if (fails) std::fprintf(stderr, "%d checks failed\n", fails);
  else std::printf("all checks passed\n");
  return fails ? 1 : 0;
}
