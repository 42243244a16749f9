"""Leaf operators (oracle; test infrastructure only).

Paper Sec. 3: on a leaf with a p x p Chebyshev grid and q Gauss nodes per side
build

* A = -C11 (D1)^2 - 2 C12 D1 D2 - C22 (D2)^2 + C1 D1 + C2 D2 + C   (Sec. 3.2)
* F_c,ci = [0; A_ci,ci^-1]                                        (eq. alpine1)
* S_c,ge = [I; -A_ci,ci^-1 A_ci,ce] L_ce,ge                       (eq. alpine3)
* D_ge,c = [L_loc D2(I_s,:); L_loc D1(I_e,:); L_loc D2(I_n,:); L_loc D1(I_w,:)]
* H = D_ge,c F,  T = D_ge,c S                                      (eq. alpine4)

Grid index of node (ix, iy) is iy*p + ix, so D1 = I (x) Dx and D2 = Dy (x) I.
(D1)^2 is read literally as the square of the first-derivative matrix.
The boundary flux is +d/dx on vertical sides and +d/dy on horizontal sides
(the sign convention of Sec. 3.1, not the outward normal).
L_ce,ge: a non-corner exterior node takes the degree q-1 interpolant of the
Gauss data of its own side; a corner takes the mean of the two values
extrapolated from the two sides that meet there (Sec. 3.4).
"""

import functools

import numpy as np
import scipy.linalg as sla

from .spectral import cheb_nodes, diff_matrix, gauss_nodes, interp_matrix


def leaf_geometry(p):
    """Index sets of a p x p grid: I_ci, I_ce (ascending grid index) and the
    four sides I_s, I_e, I_n, I_w (increasing coordinate)."""
    idx = np.arange(p * p).reshape(p, p)       # [iy, ix]
    inner = np.zeros((p, p), dtype=bool)
    inner[1:-1, 1:-1] = True
    I_ci = idx[inner]
    I_ce = idx[~inner]
    I_s = idx[0, :]
    I_e = idx[:, p - 1]
    I_n = idx[p - 1, :]
    I_w = idx[:, 0]
    return I_ci, I_ce, (I_s, I_e, I_n, I_w)


@functools.lru_cache(maxsize=None)
def reference_matrices(p, q):
    """Reference-box matrices: 1-D D on [-1,1], L_loc (q x p), L_ce,ge."""
    xc = cheb_nodes(p)
    xg = gauss_nodes(q)
    D = diff_matrix(xc)
    L_loc = interp_matrix(xc, xg)
    I_ci, I_ce, (I_s, I_e, I_n, I_w) = leaf_geometry(p)
    # interpolation from one side's Gauss nodes to the p Chebyshev points of
    # that side (end points are extrapolations)
    G2C = interp_matrix(xg, xc)                  # p x q
    L = np.zeros((I_ce.size, 4 * q))
    row_of = {int(k): r for r, k in enumerate(I_ce)}
    S, E, N, W = 0, 1, 2, 3

    def put(r, side, t_index, weight):
        L[r, side * q:(side + 1) * q] += weight * G2C[t_index]

    for k in I_ce:
        iy, ix = divmod(int(k), p)
        r = row_of[int(k)]
        corner_x = ix in (0, p - 1)
        corner_y = iy in (0, p - 1)
        if corner_x and corner_y:
            hside = S if iy == 0 else N
            vside = W if ix == 0 else E
            put(r, hside, ix, 0.5)
            put(r, vside, iy, 0.5)
        elif iy == 0:
            put(r, S, ix, 1.0)
        elif iy == p - 1:
            put(r, N, ix, 1.0)
        elif ix == 0:
            put(r, W, iy, 1.0)
        else:
            put(r, E, iy, 1.0)
    return D, L_loc, L


def leaf_operators(box_xyxy, coeffs, p, q):
    """Operators of one leaf (Sec. 3, Algorithm 1 leaf branch).

    box_xyxy: (x0, x1, y0, y1); coeffs: [6, p*p] nodal values of
    c11, c12, c22, c1, c2, c (grid order iy*p+ix).
    Returns dict with F (p^2 x (p-2)^2), S (p^2 x 4q), H (4q x (p-2)^2),
    T (4q x 4q), the collocation matrix A (p^2 x p^2) and D_ge,c.
    """
    x0, x1, y0, y1 = box_xyxy
    D, L_loc, L = reference_matrices(p, q)
    Dx = (2.0 / (x1 - x0)) * D
    Dy = (2.0 / (y1 - y0)) * D
    Ip = np.eye(p)
    D1 = np.kron(Ip, Dx)
    D2 = np.kron(Dy, Ip)
    c11, c12, c22, c1, c2, c0 = [np.asarray(coeffs[i], dtype=np.float64)
                                 for i in range(6)]
    A = (-c11[:, None] * (D1 @ D1) - 2.0 * c12[:, None] * (D1 @ D2)
         - c22[:, None] * (D2 @ D2) + c1[:, None] * D1 + c2[:, None] * D2
         + np.diag(c0))
    I_ci, I_ce, (I_s, I_e, I_n, I_w) = leaf_geometry(p)
    Aii = A[np.ix_(I_ci, I_ci)]
    Aie = A[np.ix_(I_ci, I_ce)]
    lu = sla.lu_factor(Aii)
    if np.any(np.diag(lu[0]) == 0.0):
        raise np.linalg.LinAlgError("singular leaf interior block")
    Aii_inv = sla.lu_solve(lu, np.eye(I_ci.size))
    mi = I_ci.size
    F = np.zeros((p * p, mi))
    F[I_ci] = Aii_inv
    S = np.zeros((p * p, 4 * q))
    S[I_ce] = L
    S[I_ci] = -sla.lu_solve(lu, Aie @ L)
    Dge = np.vstack([L_loc @ D2[I_s], L_loc @ D1[I_e],
                     L_loc @ D2[I_n], L_loc @ D1[I_w]])
    H = Dge @ F
    T = Dge @ S
    return dict(F=F, S=S, H=H, T=T, A=A, Dge=Dge, L=L, I_ci=I_ci, I_ce=I_ce)
