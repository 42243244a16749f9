"""Shared setup of GPU parity cases: the library side takes node coordinates
from the library, the oracle side from the oracle; inputs come from the shared
seeded generators in ``workloads``."""

import numpy as np

import oracle
import workloads as W
from oracle.leaf import leaf_geometry

from oracle_cases import make_inputs


def interior_index(p):
    I_ci, _, _ = leaf_geometry(p)
    return I_ci


def lib_inputs(tree, p, q, coeff_fn, sol):
    """coeffs [nl, 6, p^2], f [n_bdry], g [nl, mi] from library nodes."""
    xy = tree.leaf_cheb_nodes(p)
    coeffs = np.stack([coeff_fn(xy[i, :, 0], xy[i, :, 1]) for i in range(len(xy))])
    I_ci = interior_index(p)
    g = np.stack([sol.g(xy[i, I_ci, 0], xy[i, I_ci, 1], coeffs[i][:, I_ci])
                  for i in range(len(xy))])
    b = tree.bdry_gauss_nodes(q)
    f = sol.u(b[:, 0], b[:, 1])
    return coeffs, f, g, xy


def oracle_solution(otree, p, q, coeff_fn, sol):
    coeffs, f, g, ex = make_inputs(otree, p, q, coeff_fn, sol)
    ops = oracle.build(otree, coeffs, p, q)
    uc, u = oracle.solve(ops, f, g)
    return uc, ex


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def relerr(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


class PoissonSol:
    def u(self, x, y):
        return W.poisson_u(x, y)

    def g(self, x, y, c):
        return W.poisson_g(x, y)
