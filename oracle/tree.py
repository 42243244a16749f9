"""Box tree, Gauss node numbering and refinement (oracle; test infrastructure).

Paper: Sec. 2 and Fig. 1 (binary tree of boxes, parent numbered before its
children), Sec. 5.1 notation (global Gauss vector, I_ge / I_gi index vectors,
J1/J2/J3 of the merge, Sec. 4 figure), Sec. 6.1 (refinement criterion) and
Sec. 6.2-6.3 (neighbours, non-matching interfaces, P_up / P_down).

Readings where the paper is silent:

* Split order: a box covering several base leaves is cut across the direction
  with more leaves; on a tie it is cut in x (a vertical cut).  A refined
  (2x2-split) box is cut in x first, then each half in y.  The x-cut gives
  alpha = west, beta = east; the y-cut alpha = south, beta = north.
* Leaf boundary order: sides S, E, N, W, each with q Gauss nodes in increasing
  coordinate (the row order of D_ge,c in Sec. 3.4).
* Parent boundary order: J1 (alpha's kept nodes, alpha's order) followed by J2.
* Canonical leaf order for inputs and outputs: by (problem, y0, x0).
* Canonical domain boundary order: sides S, E, N, W, increasing coordinate.
* Refinement: a leaf splits into 2x2 when the distance from the target point
  to the closed box is <= t * l, with 2l its side (Sec. 6.1).  A refined box
  whose same-size neighbour across a side is an unrefined leaf gets P_up /
  P_down on that side (Sec. 6.3); a side with no same-size neighbour keeps its
  nodes.  P_up evaluates the coarse side's Gauss interpolant at every fine
  node; P_down evaluates, at each coarse node, the interpolant of the one fine
  panel containing it (the average of two panels on an exact junction).  With
  two equal panels this is the paper's pair of q -> q/2 blocks.

* Side conditions (Sec. 7.6 uses zero Neumann data on two sides and
  periodicity on the other two, and states that the algorithm is unchanged):
  each side of a problem is Dirichlet ('D'), Neumann ('N') or periodic ('P',
  in opposite pairs).  A periodic pair is one set of Gauss nodes: the east
  (north) side's segments are the west (south) side's, so the seam is an
  interface like any other and the merge whose children meet across it
  eliminates it.  On Neumann sides the data is the boundary flux in the
  convention of Sec. 3.1 (+d/dx on vertical sides, +d/dy on horizontal
  sides); the nodes stay unknowns of the root.  The canonical boundary list
  keeps all four sides; entries of a periodic side name the seam nodes and
  carry no data.

Geometry is kept in integers: one base leaf spans ``U`` units per direction,
so every refined box, edge and junction is exact.
"""

import numpy as np

from .spectral import gauss_nodes, interp_matrix

U = 1 << 24          # integer units per base-leaf side


class Box:
    __slots__ = ("id", "problem", "ix0", "ix1", "iy0", "iy1", "parent",
                 "alpha", "beta", "cut", "kind", "depth", "is_leaf",
                 "ge", "gi", "ge_fine", "Pup", "Pdown", "cblocks")

    def __init__(self, problem, ix0, ix1, iy0, iy1, kind, depth):
        self.problem = problem
        self.ix0, self.ix1, self.iy0, self.iy1 = ix0, ix1, iy0, iy1
        self.kind = kind          # 'base' | 'quad' | 'half'
        self.depth = depth        # refinement depth of quad / half boxes
        self.parent = None
        self.alpha = self.beta = None
        self.cut = None
        self.is_leaf = False
        self.ge = self.gi = self.ge_fine = None
        self.Pup = self.Pdown = None
        self.cblocks = None
        self.id = -1


class Tree:
    """A forest of independent problems, each a rectangle split into boxes."""

    def __init__(self, tie="x"):
        self.tie = tie            # cut direction for a square base region
        self.problems = []        # dicts: X0, X1, Y0, Y1, nx, ny
        self.quad_leaves = []     # per problem: set of (ix0, iy0, w, h, depth)
        self._boxes = None
        self._q = None

    # -- construction -----------------------------------------------------
    @classmethod
    def uniform(cls, x0, x1, y0, y1, nx, ny, n_problems=1, tie="x"):
        t = cls(tie)
        for _ in range(n_problems):
            t.problems.append(dict(X0=float(x0), X1=float(x1), Y0=float(y0),
                                   Y1=float(y1), nx=int(nx), ny=int(ny),
                                   bc=("D", "D", "D", "D")))
            t.quad_leaves.append({(i * U, j * U, U, U, 0)
                                  for i in range(nx) for j in range(ny)})
        return t

    def _phys(self, prob, ix, iy):
        P = self.problems[prob]
        x = P["X0"] + (P["X1"] - P["X0"]) * (ix / (P["nx"] * U))
        y = P["Y0"] + (P["Y1"] - P["Y0"]) * (iy / (P["ny"] * U))
        return x, y

    def set_bc(self, bc, problem=None):
        """Side conditions (S, E, N, W), each 'D', 'N' or 'P'; periodic
        sides come in opposite pairs.  problem=None: every problem."""
        bc = tuple(bc)
        if len(bc) != 4 or any(k not in ("D", "N", "P") for k in bc):
            raise ValueError("bc must be four of 'D', 'N', 'P'")
        if (bc[1] == "P") != (bc[3] == "P") or (bc[0] == "P") != (bc[2] == "P"):
            raise ValueError("periodic sides come in opposite pairs")
        for k in (range(len(self.problems)) if problem is None else [problem]):
            self.problems[k]["bc"] = bc
        self._boxes = None

    def refine_point(self, problem, px, py, n_ref, t=np.sqrt(2.0)):
        """Sec. 6.1: n_ref rounds of splitting every close leaf into 2x2."""
        P = self.problems[problem]
        sx = (P["X1"] - P["X0"]) / (P["nx"] * U)
        sy = (P["Y1"] - P["Y0"]) / (P["ny"] * U)
        for _ in range(n_ref):
            new = set()
            for (ix, iy, w, h, d) in self.quad_leaves[problem]:
                x0 = P["X0"] + ix * sx
                x1 = P["X0"] + (ix + w) * sx
                y0 = P["Y0"] + iy * sy
                y1 = P["Y0"] + (iy + h) * sy
                dx = max(x0 - px, 0.0, px - x1)
                dy = max(y0 - py, 0.0, py - y1)
                dist = np.hypot(dx, dy)
                half = 0.5 * max(x1 - x0, y1 - y0)
                if dist <= t * half and w >= 2 and h >= 2:
                    hw, hh = w // 2, h // 2
                    new |= {(ix, iy, hw, hh, d + 1), (ix + hw, iy, hw, hh, d + 1),
                            (ix, iy + hh, hw, hh, d + 1),
                            (ix + hw, iy + hh, hw, hh, d + 1)}
                else:
                    new.add((ix, iy, w, h, d))
            self.quad_leaves[problem] = new
        self._boxes = None

    # -- binary tree --------------------------------------------------------
    def _make(self, prob, ix0, ix1, iy0, iy1, kind, depth, out):
        b = Box(prob, ix0, ix1, iy0, iy1, kind, depth)
        out.append(b)
        w, h = ix1 - ix0, iy1 - iy0
        leaf_key = (ix0, iy0, w, h, depth)
        if kind in ("base", "quad") and leaf_key in self.quad_leaves[prob]:
            b.is_leaf = True
            return b
        if kind == "base" and (w > U or h > U):
            bx, by = w // U, h // U
            if bx > by or (bx == by and bx > 1 and self.tie == "x"):
                xm = ix0 + (bx // 2) * U
                kids = ((ix0, xm, iy0, iy1), (xm, ix1, iy0, iy1))
                b.cut = "x"
            else:
                ym = iy0 + (by // 2) * U
                kids = ((ix0, ix1, iy0, ym), (ix0, ix1, ym, iy1))
                b.cut = "y"
            kk = []
            for (a0, a1, c0, c1) in kids:
                sub_kind = "base"
                if a1 - a0 == U and c1 - c0 == U:
                    sub_kind = "base"    # a single base leaf (maybe refined)
                kk.append(self._make(prob, a0, a1, c0, c1, sub_kind, 0, out))
        elif kind in ("base", "quad"):
            # a refined quad box: x-cut into two halves
            xm = ix0 + w // 2
            b.cut = "x"
            kk = [self._make(prob, ix0, xm, iy0, iy1, "half", depth, out),
                  self._make(prob, xm, ix1, iy0, iy1, "half", depth, out)]
        else:
            # half of a refined quad box: y-cut into two quad boxes
            ym = iy0 + h // 2
            b.cut = "y"
            kk = [self._make(prob, ix0, ix1, iy0, ym, "quad", depth + 1, out),
                  self._make(prob, ix0, ix1, ym, iy1, "quad", depth + 1, out)]
        b.alpha, b.beta = kk
        kk[0].parent = b
        kk[1].parent = b
        return b

    @property
    def boxes(self):
        if self._boxes is None:
            out = []
            self.roots = []
            for prob, P in enumerate(self.problems):
                r = self._make(prob, 0, P["nx"] * U, 0, P["ny"] * U, "base", 0, out)
                self.roots.append(r)
            for i, b in enumerate(out):      # pre-order: parent < child
                b.id = i
            self._boxes = out
            self._q = None
        return self._boxes

    @property
    def leaves(self):
        """Leaf boxes in canonical order (problem, y0, x0)."""
        lv = [b for b in self.boxes if b.is_leaf]
        lv.sort(key=lambda b: (b.problem, b.iy0, b.ix0))
        return lv

    def box_phys(self, b):
        x0, y0 = self._phys(b.problem, b.ix0, b.iy0)
        x1, y1 = self._phys(b.problem, b.ix1, b.iy1)
        return x0, x1, y0, y1

    # -- Gauss nodes --------------------------------------------------------
    def gauss(self, q):
        """Number the Gauss nodes and fill ge/gi (and P_up/P_down) of each box.

        Each leaf edge (a segment) carries q nodes with consecutive ids.
        Returns (node_xy [N, 2], boundary node ids in canonical order).
        """
        boxes = self.boxes
        if self._q == q:
            return self._node_xy, self._bdry
        g = gauss_nodes(q)
        seg_id = {}
        segs = []
        for p, P in enumerate(self.problems):
            bc = P["bc"]
            if bc[1] == "P" and P["nx"] < 2 or bc[0] == "P" and P["ny"] < 2:
                raise ValueError("a periodic direction needs at least two leaves")
            for (ix, iy, w, h, d) in self.quad_leaves[p]:
                if d > 0 and (bc[1] == "P" and (ix == 0 or ix + w == P["nx"] * U) or
                              bc[0] == "P" and (iy == 0 or iy + h == P["ny"] * U)):
                    raise ValueError("refined leaves on a periodic side")

        def seg(key):
            # a periodic pair is one set of nodes: east onto west, north onto
            # south
            p, o, fx = key[0], key[1], key[2]
            P = self.problems[p]
            if o == "v" and P["bc"][1] == "P" and fx == P["nx"] * U:
                key = (p, o, 0) + key[3:]
            if o == "h" and P["bc"][0] == "P" and fx == P["ny"] * U:
                key = (p, o, 0) + key[3:]
            if key not in seg_id:
                seg_id[key] = len(segs)
                segs.append(key)
            return seg_id[key]

        def leaf_sides(b):
            p = b.problem
            return [seg((p, "h", b.iy0, b.ix0, b.ix1)),
                    seg((p, "v", b.ix1, b.iy0, b.iy1)),
                    seg((p, "h", b.iy1, b.ix0, b.ix1)),
                    seg((p, "v", b.ix0, b.iy0, b.iy1))]

        for b in self.leaves:
            leaf_sides(b)
        # node coordinates
        xy = np.empty((len(segs) * q, 2))
        for s, (p, o, fixed, s0, s1) in enumerate(segs):
            for k in range(q):
                t = s0 + (s1 - s0) * (g[k] + 1.0) / 2.0
                if o == "h":
                    xy[s * q + k] = self._phys(p, t, fixed)
                else:
                    xy[s * q + k] = self._phys(p, fixed, t)
        self._segs = segs
        self._seg_id = seg_id

        def nodes_of(s):
            return list(range(s * q, (s + 1) * q))

        quad_set = [set((a, c, w, h) for (a, c, w, h, d) in ql)
                    for ql in self.quad_leaves]

        for b in reversed(boxes):            # children before parents
            if b.is_leaf:
                ge = []
                for s in leaf_sides(b):
                    ge += nodes_of(s)
                b.ge = ge
                continue
            a, c = b.alpha, b.beta
            sa = set(a.ge)
            sb = set(c.ge)
            J3 = [j for j in a.ge if j in sb]
            J1 = [j for j in a.ge if j not in sb]
            J2 = [j for j in c.ge if j not in sa]
            b.gi = J3
            b.ge = J1 + J2
            if b.kind == "quad" or (b.kind == "base" and b.ix1 - b.ix0 == U
                                    and b.iy1 - b.iy0 == U):
                self._coarsen(b, q, g, quad_set[b.problem], nodes_of)
        # canonical boundary nodes of each problem: S, E, N, W (a periodic
        # side lists the seam nodes it shares with its partner)
        bd, kinds = [], []
        for p, P in enumerate(self.problems):
            W, H = P["nx"] * U, P["ny"] * U
            bc = P["bc"]
            sides = [("h", 0), ("v", 0 if bc[1] == "P" else W),
                     ("h", 0 if bc[2] == "P" else H), ("v", 0)]
            for side, (o, fx) in enumerate(sides):
                ss = [s for s, k in enumerate(segs)
                      if k[0] == p and k[1] == o and k[2] == fx]
                ss.sort(key=lambda s: segs[s][3])
                for s in ss:
                    bd += nodes_of(s)
                    kinds += [bc[side]] * q
        self._node_xy = xy
        self._bdry = np.array(bd, dtype=np.int64)
        self._bdry_kind = np.array(kinds)
        self._q = q
        return xy, self._bdry

    def bdry_kind(self, q):
        """'D', 'N' or 'P' for every canonical boundary entry."""
        self.gauss(q)
        return self._bdry_kind

    def _coarsen(self, b, q, g, quads, nodes_of):
        """Sec. 6.3: replace fine nodes on each side that faces an unrefined
        same-size neighbour by that neighbour's q nodes; record P_up/P_down."""
        w, h = b.ix1 - b.ix0, b.iy1 - b.iy0
        segs = self._segs
        p = b.problem
        # side: (orientation, fixed coord, lo, hi, neighbour lower-left corner)
        sides = [("h", b.iy0, b.ix0, b.ix1, (b.ix0, b.iy0 - h)),
                 ("v", b.ix1, b.iy0, b.iy1, (b.ix1, b.iy0)),
                 ("h", b.iy1, b.ix0, b.ix1, (b.ix0, b.iy1)),
                 ("v", b.ix0, b.iy0, b.iy1, (b.ix0 - w, b.iy0))]
        fine = list(b.ge)
        new = list(fine)
        blocks = []     # (fine node ids, coarse node ids, Pup block, Pdown block)
        for (o, fx, lo, hi, (nx0, ny0)) in sides:
            if (nx0, ny0, w, h) not in quads:
                continue          # no unrefined same-size neighbour there
            key = (p, o, fx, lo, hi)
            if key not in self._seg_id:
                continue
            cs = self._seg_id[key]
            on = [j for j in fine
                  if segs[j // q][1] == o and segs[j // q][2] == fx
                  and segs[j // q][3] >= lo and segs[j // q][4] <= hi]
            if on == nodes_of(cs):
                continue          # already aligned
            coarse = nodes_of(cs)
            # P_up: coarse interpolant evaluated at each fine node
            xi_f = []
            for j in on:
                (_, _, _, s0, s1) = segs[j // q]
                t = s0 + (s1 - s0) * (g[j % q] + 1.0) / 2.0
                xi_f.append(2.0 * (t - lo) / (hi - lo) - 1.0)
            Pup = interp_matrix(g, np.array(xi_f))
            # P_down: each coarse node from the fine panel that holds it
            panels = sorted(set(j // q for j in on), key=lambda s: segs[s][3])
            Pdn = np.zeros((q, len(on)))
            col = {j: i for i, j in enumerate(on)}
            for k in range(q):
                t = lo + (hi - lo) * (g[k] + 1.0) / 2.0
                hits = []
                for s in panels:
                    s0, s1 = segs[s][3], segs[s][4]
                    tol = 1e-12 * (hi - lo)
                    if s0 - tol <= t <= s1 + tol:
                        hits.append(s)
                for s in hits:
                    s0, s1 = segs[s][3], segs[s][4]
                    xi = 2.0 * (t - s0) / (s1 - s0) - 1.0
                    row = interp_matrix(g, np.array([xi]))[0]
                    for kk in range(q):
                        Pdn[k, col[s * q + kk]] += row[kk] / len(hits)
            blocks.append((on, coarse, Pup, Pdn))
            pos = new.index(on[0])
            new = [j for j in new if j not in set(on)]
            new[pos:pos] = coarse
        if not blocks:
            return
        ef, ec = len(fine), len(new)
        Pup = np.zeros((ef, ec))
        Pdn = np.zeros((ec, ef))
        fi = {j: i for i, j in enumerate(fine)}
        ci = {j: i for i, j in enumerate(new)}
        touched = set()
        for (on, coarse, pu, pd) in blocks:
            for a_, j in enumerate(on):
                for b_, c in enumerate(coarse):
                    Pup[fi[j], ci[c]] = pu[a_, b_]
                    Pdn[ci[c], fi[j]] = pd[b_, a_]
                touched.add(j)
        for j in fine:
            if j not in touched:
                Pup[fi[j], ci[j]] = 1.0
                Pdn[ci[j], fi[j]] = 1.0
        b.ge_fine = fine
        b.ge = new
        b.Pup = Pup
        b.Pdown = Pdn
        b.cblocks = blocks
