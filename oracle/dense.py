"""The global collocation system, assembled and solved by a library LU
(oracle; test infrastructure only).

This is the plain definition of what Algorithms 1 and 2 compute: they perform
exact block elimination (nested dissection) of one square linear system
K x = b (Sec. 3.2, Sec. 4 and the merge remark).  Unknowns: the p^2 values
u_c on every leaf and the value at every interior "master" Gauss node.  Rows:

* E1 (collocated PDE, Sec. 3.2):  A(I_ci, :) u_c = g_ci on every leaf;
* E2 (Gauss -> Chebyshev exterior, eq. alpine2p5):  u_c(I_ce) - L_ce,ge u_ge = 0,
  where u_ge holds f on the domain boundary and P_up times the coarse values
  on refined, coarsened sides (Sec. 6.3);
* E3 (flux continuity, Sec. 4): at a Gauss node shared by two leaves the two
  leaf fluxes D_ge,c u_c agree; at a coarse node of a refined interface the
  coarse leaf's flux equals P_down applied to the fine leaves' fluxes;
* side conditions (Sec. 7.6): a node on a Neumann side is an unknown whose
  row sets its leaf's flux to the data; a node of a periodic seam is shared
  by the leaves on the two sides and gets an ordinary E3 row.  Only
  Dirichlet nodes are known values.

``dense_solve`` solves this system directly; ``dense_adjoint`` solves the
transposed system for the cotangents of the data; ``residual`` evaluates
b - K x.
"""

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .leaf import leaf_operators


def _structure(tree, q):
    """Classify Gauss nodes: boundary, slave (fine node on a coarsened side)
    or master; collect the P_up rows of slaves and the P_down rows of coarse
    nodes."""
    node_xy, bdry = tree.gauss(q)
    N = node_xy.shape[0]
    kind = np.zeros(N, dtype=int)            # 0 master, 1 boundary, 2 slave
    kind[bdry[tree.bdry_kind(q) == "D"]] = 1
    slave_rows = {}                          # slave -> [(coarse node, w)]
    coarse_fine = {}                         # coarse -> [(fine node, w)]
    for b in tree.boxes:
        if not b.cblocks:
            continue
        for (on, coarse, Pup, Pdn) in b.cblocks:
            for a, j in enumerate(on):
                kind[j] = 2
                slave_rows[j] = [(c, Pup[a, k]) for k, c in enumerate(coarse)]
            for k, c in enumerate(coarse):
                coarse_fine[c] = [(j, Pdn[k, a]) for a, j in enumerate(on)]
    # nodes that no leaf carries on its boundary are unused
    used = np.zeros(N, dtype=bool)
    for b in tree.leaves:
        used[b.ge] = True
    return node_xy, bdry, kind, used, slave_rows, coarse_fine


def assemble_system(tree, coeffs, p, q=None):
    """Return (K sparse CSR, layout dict)."""
    if q is None:
        q = p - 1
    node_xy, bdry, kind, used, slave_rows, coarse_fine = _structure(tree, q)
    leaves = tree.leaves
    nl = len(leaves)
    p2 = p * p
    masters = np.where((kind == 0) & used)[0]
    mcol = {int(j): nl * p2 + k for k, j in enumerate(masters)}
    bkind = tree.bdry_kind(q)
    bpos = {int(j): k for k, j in enumerate(bdry) if bkind[k] == "D"}
    npos = {int(j): k for k, j in enumerate(bdry) if bkind[k] == "N"}
    e3_f = []                                # Neumann rows: (row, bdry index)
    nunk = nl * p2 + masters.size
    rows, cols, vals = [], [], []
    # right-hand-side maps: E1 rows take g; E2 rows take -(L f) terms
    e1_rows = np.zeros((nl, (p - 2) ** 2), dtype=int)
    e2_f = []                                # (row, bdry index, weight)
    leaf_ops = []
    r = 0
    owners = {}                              # node -> [(leaf idx, local row)]
    for i, b in enumerate(leaves):
        o = leaf_operators(tree.box_phys(b), coeffs[i], p, q)
        leaf_ops.append(o)
        A, L, I_ci, I_ce = o["A"], o["L"], o["I_ci"], o["I_ce"]
        base = i * p2
        for a, k in enumerate(I_ci):               # E1
            nz = np.nonzero(A[k])[0]
            rows += [r] * nz.size
            cols += list(base + nz)
            vals += list(A[k, nz])
            e1_rows[i, a] = r
            r += 1
        for a, k in enumerate(I_ce):               # E2
            rows.append(r)
            cols.append(base + k)
            vals.append(1.0)
            for c, j in enumerate(b.ge):
                wgt = -L[a, c]
                if wgt == 0.0:
                    continue
                if kind[j] == 1:
                    e2_f.append((r, bpos[int(j)], -wgt))
                elif kind[j] == 2:
                    for (cn, pw) in slave_rows[int(j)]:
                        rows.append(r)
                        cols.append(mcol[int(cn)])
                        vals.append(wgt * pw)
                else:
                    rows.append(r)
                    cols.append(mcol[int(j)])
                    vals.append(wgt)
            r += 1
        for c, j in enumerate(b.ge):
            owners.setdefault(int(j), []).append((i, c))
    for j in masters:                               # E3
        j = int(j)
        own = owners[j]
        if len(own) == 2:
            terms = [(own[0], 1.0), (own[1], -1.0)]
        elif j in npos:                     # Neumann: flux = data
            terms = [(own[0], 1.0)]
            e3_f.append((r, npos[j]))
        else:
            terms = [(own[0], 1.0)]
            for (fj, pw) in coarse_fine[j]:
                terms.append((owners[int(fj)][0], -pw))
        for ((i, c), s) in terms:
            row = leaf_ops[i]["Dge"][c]
            nz = np.nonzero(row)[0]
            rows += [r] * nz.size
            cols += list(i * p2 + nz)
            vals += list(s * row[nz])
        r += 1
    assert r == nunk, (r, nunk)
    K = sp.csr_matrix((vals, (rows, cols)), shape=(nunk, nunk))
    lay = dict(nl=nl, p2=p2, masters=masters, e1_rows=e1_rows, e2_f=e2_f,
               e3_f=e3_f, nunk=nunk, kind=kind, slave_rows=slave_rows, bdry=bdry,
               bkind=bkind, node_xy=node_xy)
    return K, lay


def _rhs(lay, f, g):
    b = np.zeros(lay["nunk"])
    b[lay["e1_rows"].ravel()] = np.asarray(g).ravel()
    for (r, k, wgt) in lay["e2_f"]:
        b[r] += wgt * f[k]
    for (r, k) in lay["e3_f"]:
        b[r] += f[k]
    return b


def _unpack(lay, x, f):
    nl, p2 = lay["nl"], lay["p2"]
    u_c = x[:nl * p2].reshape(nl, p2)
    N = lay["kind"].size
    u = np.zeros(N)
    u[lay["masters"]] = x[nl * p2:]
    dm = lay["bkind"] == "D"
    u[lay["bdry"][dm]] = np.asarray(f)[dm]
    for j, terms in lay["slave_rows"].items():
        u[j] = sum(w * u[c] for (c, w) in terms)
    return u_c, u


def dense_solve(tree, coeffs, p, q=None, f=None, g=None, dense=True):
    """Solve K x = b directly.  Returns (u_c [n_leaves, p^2], u [N])."""
    K, lay = assemble_system(tree, coeffs, p, q)
    b = _rhs(lay, f, g)
    # scaling each row by its largest entry leaves the solution unchanged and
    # keeps partial pivoting from being misled by the mixed row scales
    s = 1.0 / abs(K).max(axis=1).toarray().ravel()
    Ks = sp.diags(s) @ K
    if dense:
        x = sla.solve(Ks.toarray(), s * b)
    else:
        x = spla.spsolve(Ks.tocsc(), s * b)
    return _unpack(lay, x, f)


def residual(tree, coeffs, p, q, u_c, u, f, g):
    """b - K x for x = (u_c, u at master nodes); returns the residual vector
    and the layout (so callers can split E1 / E2 / E3 rows)."""
    K, lay = assemble_system(tree, coeffs, p, q)
    b = _rhs(lay, f, g)
    x = np.concatenate([np.asarray(u_c).ravel(), np.asarray(u)[lay["masters"]]])
    return b - K @ x, lay


def dense_adjoint(tree, coeffs, p, q, ubar_c):
    """Transpose of the map (f, g) -> u_c through the global system.

    u_c is the first block of x = K^-1 b(f, g), and b depends on the data
    linearly: g fills the PDE rows (E1) with coefficient +1, f enters the
    interpolation rows (E2) through -L f and the Neumann flux rows with
    coefficient +1.  So with lam = K^-T [ubar_c; 0], gbar = lam at the E1
    rows and fbar collects lam over the rows that read each entry of f.
    Periodic entries of f are read by no row, so their fbar is 0.
    Returns (fbar [n_bdry], gbar [n_leaves, (p-2)^2])."""
    K, lay = assemble_system(tree, coeffs, p, q)
    y = np.zeros(lay["nunk"])
    y[:lay["nl"] * lay["p2"]] = np.asarray(ubar_c).ravel()
    # K^T lam = y with the rows of K scaled as in dense_solve: (S K)^T mu = y,
    # lam = S mu
    s = 1.0 / abs(K).max(axis=1).toarray().ravel()
    Ks = (sp.diags(s) @ K).toarray()
    lam = s * sla.solve(Ks.T, y)
    gbar = lam[lay["e1_rows"]].copy()
    fbar = np.zeros(len(lay["bdry"]))
    for (r, k, wgt) in lay["e2_f"]:
        fbar[k] += wgt * lam[r]
    for (r, k) in lay["e3_f"]:
        fbar[k] += lam[r]
    return fbar, gbar
