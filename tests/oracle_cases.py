"""Oracle-side problem setup for tests: node coordinates from the oracle's own
geometry, inputs from the shared seeded generators."""

import numpy as np

import oracle
from oracle.leaf import leaf_geometry
import workloads as W


def leaf_nodes(tree, p):
    """[n_leaves, p*p, 2] Chebyshev node coordinates (grid order iy*p+ix)."""
    xc = oracle.cheb_nodes(p)
    out = []
    for b in tree.leaves:
        x0, x1, y0, y1 = tree.box_phys(b)
        X = x0 + (x1 - x0) * (xc + 1.0) / 2.0
        Y = y0 + (y1 - y0) * (xc + 1.0) / 2.0
        YY, XX = np.meshgrid(Y, X, indexing="ij")
        out.append(np.stack([XX.ravel(), YY.ravel()], -1))
    return np.array(out)


def make_inputs(tree, p, q, coeff_fn, sol):
    """coeffs [nl, 6, p^2], f [n_bdry], g [nl, (p-2)^2], exact u_c."""
    xy = leaf_nodes(tree, p)
    coeffs = np.stack([coeff_fn(xy[i, :, 0], xy[i, :, 1])
                       for i in range(len(xy))])
    I_ci, _, _ = leaf_geometry(p)
    g = np.stack([sol.g(xy[i, I_ci, 0], xy[i, I_ci, 1], coeffs[i][:, I_ci])
                  for i in range(len(xy))])
    node_xy, bdry = tree.gauss(q)
    f = sol.u(node_xy[bdry, 0], node_xy[bdry, 1])
    ex = sol.u(xy[..., 0], xy[..., 1])
    return coeffs, f, g, ex


class Poisson:
    """Workload 1: u = exp(x) cos(y) + x^2 y under -Lap."""
    coeff = staticmethod(W.poisson_coeffs)

    def u(self, x, y):
        return W.poisson_u(x, y)

    def g(self, x, y, c):
        return W.poisson_g(x, y)


def relerr(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) /
                 np.max(np.abs(np.asarray(b))))
