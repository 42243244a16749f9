"""Implicit time stepping with a fixed elliptic operator (oracle; test
infrastructure only).

Sec. 7.6 advances u_t = A_pde u with Crank-Nicolson: every step solves
(I/k - A_pde/2) u_new = (I/k + A_pde/2) u_old.  The left operator L is built
once (Algorithm 1); each step evaluates the right side on the leaf grids and
runs one solve (Algorithm 2).  With L = I/k - A_pde/2 the right side is
(2/k) u_old - L u_old, so ``operator_apply`` with sigma = 2/k gives it.
"""

import numpy as np

from .leaf import leaf_operators
from .hps import build, solve


def operator_apply(tree, coeffs, p, u_c, sigma):
    """sigma u - A u at the interior Chebyshev nodes of every leaf, with A the
    collocated operator of Sec. 3.2 on the leaf grid (rows I_ci).
    u_c: [n_leaves, p*p]; returns [n_leaves, (p-2)^2]."""
    out = []
    for i, b in enumerate(tree.leaves):
        o = leaf_operators(tree.box_phys(b), coeffs[i], p, 2)
        A, I_ci = o["A"], o["I_ci"]
        out.append(sigma * u_c[i][I_ci] - A[I_ci] @ u_c[i])
    return np.array(out)


def crank_nicolson(tree, coeffs, p, q, k, u0_c, n_steps, f=None):
    """n_steps Crank-Nicolson steps from u0_c [n_leaves, p*p]; coeffs are
    those of L = I/k - A_pde/2 (so c carries 1/k).  f: boundary data of every
    step (zeros if None).  Returns u_c after the last step."""
    ops = build(tree, coeffs, p, q)
    _, bdry = tree.gauss(q)
    if f is None:
        f = np.zeros(len(bdry))
    u = np.asarray(u0_c, dtype=float)
    for _ in range(n_steps):
        g = operator_apply(tree, coeffs, p, u, 2.0 / k)
        u, _ = solve(ops, f, g)
    return u
