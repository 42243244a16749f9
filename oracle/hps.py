"""Algorithms 1 and 2 with explicit per-box loops (oracle; test infrastructure).

* ``build``  -- Algorithm 1 (Sec. 5.2): leaves by Sec. 3; parents by the merge
  of Sec. 4: X = (T33a - T33b)^-1, S = X [-T31a | T32b],
  T = blkdiag(T11a, T22b) + [T13a; T23b] S.  A refined box whose side faces an
  unrefined same-size leaf gets T <- P_down T P_up (Sec. 6.3); S is kept and
  P_up applied in the solve (S_new = S P_up).
* ``solve``  -- Algorithm 2 (Sec. 5.3): upward pass h = H g at leaves,
  w = X(h3b - h3a), h = [h1a; h2b] + [T13a; T23b] w at parents (h <- P_down h
  on coarsened boxes, Sec. 6.4); downward pass u(root boundary) = f,
  u_gi = S u_ge + w at parents (u_ge,fine = P_up u_ge first, Sec. 6.4),
  u_c = S u_ge + F g at leaves.
* Neumann sides (Sec. 7.6 states that the algorithm is unchanged; the
  closure is our reading): the root's own relation flux = T u + h holds on
  its boundary, so on the Neumann nodes N, with the Dirichlet nodes D known,
  T_NN u_N = psi - h_N - T_ND f_D.  This is the merge formula of Sec. 4 with
  the outside as a sibling whose T is zero and whose flux is the data psi.
  Periodic sides need nothing here: the tree identifies their nodes and the
  ordinary merges eliminate them.
* ``solve_adjoint`` -- the transpose of the linear map (f, g) -> u_c of
  Algorithm 2, taken step by step in reverse order (not in the paper).
* ``coeff_gradient`` -- dL/dc for the nodal coefficients: with lambda the
  adjoint of the collocation system, only the PDE rows depend on c, so
  dL/dc_k(i) = -gbar(i) * (B_k u)(i) at interior nodes, with B_k the operator
  multiplying c_k in A (Sec. 3.2); zero at exterior nodes.

Explicit inverses use LAPACK getrf/getrs (scipy.linalg.lu_factor/lu_solve).
"""

import numpy as np
import scipy.linalg as sla

from .leaf import leaf_operators


class Ops:
    pass


def _inv(Z):
    lu = sla.lu_factor(Z)
    if np.any(np.diag(lu[0]) == 0.0):
        raise np.linalg.LinAlgError("singular interface block")
    return sla.lu_solve(lu, np.eye(Z.shape[0]))


def _merge_index(tau):
    a, b = tau.alpha, tau.beta
    pa = {j: i for i, j in enumerate(a.ge)}
    pb = {j: i for i, j in enumerate(b.ge)}
    sb = set(b.ge)
    sa = set(a.ge)
    p3a = [pa[j] for j in tau.gi]
    p3b = [pb[j] for j in tau.gi]
    p1a = [pa[j] for j in a.ge if j not in sb]
    p2b = [pb[j] for j in b.ge if j not in sa]
    return np.array(p1a, int), np.array(p2b, int), np.array(p3a, int), np.array(p3b, int)


def build(tree, coeffs, p, q=None):
    """Algorithm 1.  coeffs: [n_leaves, 6, p*p] in canonical leaf order."""
    if q is None:
        q = p - 1
    for P in tree.problems:
        if "D" not in P["bc"] and q > p - 2:
            # with q = p - 1 the Gauss -> Chebyshev map of every leaf has a
            # null vector (phi on horizontal edges, -phi on vertical edges,
            # phi vanishing at an edge's p - 2 inner Chebyshev nodes); only
            # Dirichlet data removes it, so the global system is singular
            raise ValueError("a problem without a Dirichlet side needs q <= p - 2")
    tree.gauss(q)
    leaves = tree.leaves
    leaf_pos = {b.id: i for i, b in enumerate(leaves)}
    ops = Ops()
    ops.tree, ops.p, ops.q = tree, p, q
    ops.box = {}
    for tau in reversed(tree.boxes):                 # tau = N_boxes, ..., 1
        if tau.is_leaf:
            o = leaf_operators(tree.box_phys(tau), coeffs[leaf_pos[tau.id]], p, q)
            ops.box[tau.id] = o
            continue
        oa, ob = ops.box[tau.alpha.id], ops.box[tau.beta.id]
        p1a, p2b, p3a, p3b = _merge_index(tau)
        Ta, Tb = oa["T"], ob["T"]
        X = _inv(Ta[np.ix_(p3a, p3a)] - Tb[np.ix_(p3b, p3b)])
        R = np.hstack([-Ta[np.ix_(p3a, p1a)], Tb[np.ix_(p3b, p2b)]])
        S = X @ R
        n1, n2 = p1a.size, p2b.size
        T = np.zeros((n1 + n2, n1 + n2))
        T[:n1, :n1] = Ta[np.ix_(p1a, p1a)]
        T[n1:, n1:] = Tb[np.ix_(p2b, p2b)]
        Q = np.vstack([Ta[np.ix_(p1a, p3a)], Tb[np.ix_(p2b, p3b)]])
        T = T + Q @ S
        o = dict(X=X, S=S, Q=Q, T_fine=T, idx=(p1a, p2b, p3a, p3b))
        if tau.Pup is not None:
            o["T"] = tau.Pdown @ T @ tau.Pup
        else:
            o["T"] = T
        ops.box[tau.id] = o
    ops.leaf_pos = leaf_pos
    # Neumann closure of each root: LU of T_NN and the block T_ND
    _, bdry = tree.gauss(q)
    kind = tree.bdry_kind(q)
    neu = set(int(j) for j in bdry[kind == "N"])
    ops.closure = {}
    for r in tree.roots:
        iN = [i for i, j in enumerate(r.ge) if j in neu]
        if not iN:
            continue
        iD = [i for i, j in enumerate(r.ge) if j not in neu]
        T = ops.box[r.id]["T"]
        lu = sla.lu_factor(T[np.ix_(iN, iN)])
        if np.any(np.diag(lu[0]) == 0.0):
            raise np.linalg.LinAlgError("singular Neumann closure")
        ops.closure[r.id] = dict(iN=np.array(iN, int), iD=np.array(iD, int), lu=lu,
                                 TND=T[np.ix_(iN, iD)])
    return ops


def solve(ops, f, g):
    """Algorithm 2 for one right-hand side.

    f: [n_bdry] boundary data at the canonical boundary Gauss nodes (u on
    Dirichlet sides, the flux on Neumann sides, ignored on periodic sides);
    g: [n_leaves, (p-2)^2] body load at leaf interior Chebyshev nodes.
    Returns (u_c [n_leaves, p*p], u [N] at every Gauss node).
    """
    tree, p, q = ops.tree, ops.p, ops.q
    node_xy, bdry = tree.gauss(q)
    kind = tree.bdry_kind(q)
    f = np.asarray(f, dtype=float)
    boxes = tree.boxes
    h = {}
    w = {}
    for tau in reversed(boxes):                      # upward pass
        o = ops.box[tau.id]
        if tau.is_leaf:
            h[tau.id] = o["H"] @ g[ops.leaf_pos[tau.id]]
            continue
        p1a, p2b, p3a, p3b = o["idx"]
        ha, hb = h[tau.alpha.id], h[tau.beta.id]
        w[tau.id] = o["X"] @ (-ha[p3a] + hb[p3b])
        hf = np.concatenate([ha[p1a], hb[p2b]]) + o["Q"] @ w[tau.id]
        h[tau.id] = tau.Pdown @ hf if tau.Pdown is not None else hf
    u = np.zeros(node_xy.shape[0])
    u[bdry[kind == "D"]] = f[kind == "D"]
    if ops.closure:
        neu_pos = {int(bdry[i]): i for i in np.where(kind == "N")[0]}
        for r in tree.roots:
            c = ops.closure.get(r.id)
            if c is None:
                continue
            ge = np.array(r.ge)
            psi = np.array([f[neu_pos[int(j)]] for j in ge[c["iN"]]])
            rhs = psi - h[r.id][c["iN"]] - c["TND"] @ u[ge[c["iD"]]]
            u[ge[c["iN"]]] = sla.lu_solve(c["lu"], rhs)
    u_c = np.zeros((len(tree.leaves), p * p))
    for tau in boxes:                                # downward pass
        o = ops.box[tau.id]
        if tau.Pup is not None:
            u[tau.ge_fine] = tau.Pup @ u[tau.ge]
        ge = tau.ge_fine if tau.ge_fine is not None else tau.ge
        if tau.is_leaf:
            i = ops.leaf_pos[tau.id]
            u_c[i] = o["S"] @ u[ge] + o["F"] @ g[i]
        else:
            u[tau.gi] = o["S"] @ u[ge] + w[tau.id]
    return u_c, u


def solve_adjoint(ops, ubar_c):
    """Transpose of (f, g) -> u_c.  ubar_c: [n_leaves, p*p].

    Returns (fbar [n_bdry], gbar [n_leaves, (p-2)^2]).  The steps of
    ``solve`` are taken in reverse order, each transposed:

    * downward pass, children before parents: u_c = S u_ge + F g at a leaf
      sends S^T ubar_c to the leaf's Gauss nodes and F^T ubar_c to gbar;
      u_gi = S u_ge + w at a parent sends the cotangent of u_gi to w (wbar)
      and S^T of it to the parent's boundary nodes; a slave node written as
      P_up times the coarse values sends its cotangent back through P_up^T;
    * Neumann closure of a root (u_N = T_NN^-1 (psi - h_N - T_ND u_D)):
      y = T_NN^-T ubar_N goes to the Neumann data psi, -y to the root's h at
      the Neumann positions, and -T_ND^T y to the Dirichlet nodes of the root;
    * the boundary data: fbar = ubar at Dirichlet entries, the closure's y at
      Neumann entries and 0 at periodic entries (the forward solve does not
      read f there);
    * upward pass, parents before children: h = [h1a; h2b] + Q w with
      w = X (h3b - h3a) sends hbar through P_down^T, then wbar += Q^T hbar and
      d = X^T wbar to h3a (minus) and h3b (plus); at a leaf, h = H g sends
      H^T hbar to gbar.
    """
    tree, p, q = ops.tree, ops.p, ops.q
    node_xy, bdry = tree.gauss(q)
    kind = tree.bdry_kind(q)
    boxes = tree.boxes
    N = node_xy.shape[0]
    mi = (p - 2) ** 2
    gbar = np.zeros((len(tree.leaves), mi))
    ubar = np.zeros(N)
    wbar = {}
    # reverse of the downward pass: children before parents
    for tau in reversed(boxes):
        o = ops.box[tau.id]
        ge = tau.ge_fine if tau.ge_fine is not None else tau.ge
        if tau.is_leaf:
            i = ops.leaf_pos[tau.id]
            np.add.at(ubar, ge, o["S"].T @ ubar_c[i])
            gbar[i] += o["F"].T @ ubar_c[i]
        else:
            ugi = ubar[tau.gi].copy()
            ubar[tau.gi] = 0.0
            wbar[tau.id] = ugi
            np.add.at(ubar, ge, o["S"].T @ ugi)
        if tau.Pup is not None:
            # u[fine] = P_up u[coarse] overwrote the slave entries
            coarse = set(tau.ge)
            slaves = [k for k, j in enumerate(tau.ge_fine) if j not in coarse]
            sl_ids = [tau.ge_fine[k] for k in slaves]
            ub_s = ubar[sl_ids].copy()
            ubar[sl_ids] = 0.0
            np.add.at(ubar, tau.ge, tau.Pup[slaves].T @ ub_s)
    # reverse of the Neumann closures
    fbar = np.zeros(len(bdry))
    hbar = {tau.id: None for tau in boxes}
    if ops.closure:
        neu_pos = {int(bdry[i]): i for i in np.where(kind == "N")[0]}
        for r in tree.roots:
            c = ops.closure.get(r.id)
            if c is None:
                continue
            ge = np.array(r.ge)
            nN, nD = ge[c["iN"]], ge[c["iD"]]
            y = sla.lu_solve(c["lu"], ubar[nN], trans=1)
            ubar[nN] = 0.0
            for a, j in enumerate(nN):
                fbar[neu_pos[int(j)]] += y[a]
            np.add.at(ubar, nD, -(c["TND"].T @ y))
            hr = np.zeros(len(r.ge))
            hr[c["iN"]] = -y
            hbar[r.id] = hr
    dm = kind == "D"
    fbar[dm] = ubar[bdry[dm]]
    # reverse of the upward pass: parents before children
    for tau in boxes:
        o = ops.box[tau.id]
        hb = hbar[tau.id]
        if tau.is_leaf:
            if hb is not None:
                gbar[ops.leaf_pos[tau.id]] += o["H"].T @ hb
            continue
        a, b = tau.alpha, tau.beta
        p1a, p2b, p3a, p3b = o["idx"]
        wb = wbar[tau.id].copy()
        ha = np.zeros(len(a.ge))
        hbb = np.zeros(len(b.ge))
        if hb is not None:
            hf = tau.Pdown.T @ hb if tau.Pdown is not None else hb
            n1 = p1a.size
            ha[p1a] += hf[:n1]
            hbb[p2b] += hf[n1:]
            wb += o["Q"].T @ hf
        d = o["X"].T @ wb
        ha[p3a] -= d
        hbb[p3b] += d
        hbar[a.id] = ha
        hbar[b.id] = hbb
    return fbar, gbar


def coeff_gradient(ops, u_c, gbar):
    """dL/dc_k at every leaf node, [n_leaves, 6, p*p] (k = c11, c12, c22,
    c1, c2, c); exterior nodes get zero."""
    tree, p = ops.tree, ops.p
    out = np.zeros((len(tree.leaves), 6, p * p))
    for tau in tree.leaves:
        i = ops.leaf_pos[tau.id]
        o = ops.box[tau.id]
        from .leaf import leaf_geometry, reference_matrices
        x0, x1, y0, y1 = tree.box_phys(tau)
        D, _, _ = reference_matrices(p, ops.q)
        Ip = np.eye(p)
        D1 = np.kron(Ip, (2.0 / (x1 - x0)) * D)
        D2 = np.kron((2.0 / (y1 - y0)) * D, Ip)
        u = u_c[i]
        Bu = [-(D1 @ (D1 @ u)), -2.0 * (D1 @ (D2 @ u)), -(D2 @ (D2 @ u)),
              D1 @ u, D2 @ u, u]
        I_ci = o["I_ci"]
        for k in range(6):
            out[i, k, I_ci] = -gbar[i] * Bu[k][I_ci]
    return out
