"""Spectral primitives on [-1, 1] (oracle; test infrastructure only).

* Chebyshev grid of Sec. 3.1: p Chebyshev points per direction, including the
  two end points (the exterior set of a leaf has 4(p-1) members and the
  interior set (p-2)^2, which needs the end points).  We take the
  Chebyshev-Lobatto family x_j = -cos(pi j/(p-1)), ascending.
* Differentiation (Sec. 3.2): the matrix that maps values at the nodes to the
  values of the derivative of the interpolating polynomial; it is exact for
  polynomials of degree <= p-1.
* Gauss nodes (Sec. 2, Sec. 3.1): the q roots of the Legendre polynomial P_q.
* Interpolation (Sec. 3.4): Lagrange interpolation between node sets.

Every routine is the textbook definition written out with products; no
stabilised or recursive formula is used, so each entry can be checked by eye.
"""

import numpy as np
from numpy.polynomial import legendre as _leg


def cheb_nodes(p):
    """Chebyshev-Lobatto points on [-1, 1], ascending, p >= 2."""
    j = np.arange(p, dtype=np.float64)
    return -np.cos(np.pi * j / (p - 1))


def gauss_nodes(q):
    """Gauss-Legendre points (roots of P_q) on [-1, 1], ascending."""
    x, _ = _leg.leggauss(q)
    return np.sort(x)


def bary_weights(x):
    """w_j = 1 / prod_{k != j} (x_j - x_k)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    w = np.empty(n)
    for j in range(n):
        d = x[j] - np.delete(x, j)
        w[j] = 1.0 / np.prod(d)
    return w


def diff_matrix(x):
    """D[i, j] = l_j'(x_i) for the Lagrange basis l_j on the nodes x.

    Off-diagonal: (w_j / w_i) / (x_i - x_j); diagonal: sum_{k != i} 1/(x_i - x_k).
    """
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    w = bary_weights(x)
    D = np.empty((n, n))
    for i in range(n):
        for j in range(n):
            if i == j:
                D[i, i] = np.sum(1.0 / (x[i] - np.delete(x, i)))
            else:
                D[i, j] = (w[j] / w[i]) / (x[i] - x[j])
    return D


def interp_matrix(src, dst):
    """P[i, j] = l_j(dst_i), Lagrange basis on the nodes src (product form).

    Evaluating at points outside [min(src), max(src)] is extrapolation, which
    the corner rule of Sec. 3.4 needs.
    """
    src = np.asarray(src, dtype=np.float64)
    dst = np.asarray(dst, dtype=np.float64)
    n = src.size
    P = np.empty((dst.size, n))
    for i, t in enumerate(dst):
        for j in range(n):
            num = 1.0
            den = 1.0
            for k in range(n):
                if k != j:
                    num *= (t - src[k])
                    den *= (src[j] - src[k])
            P[i, j] = num / den
    return P
