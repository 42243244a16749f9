"""Pins of ``oracle.residual`` (b - K x of the global collocation system, the
quantity that mixed-precision refinement drives to zero):

* the exact nodal values of a polynomial solution of tensor degree <= q - 1
  have a zero residual to rounding, for the full variable-coefficient
  operator, on uniform, refined and side-condition trees (every row of the
  system -- collocated PDE, Gauss-to-Chebyshev interpolation, flux
  continuity, refined-interface P_up / P_down, Neumann data -- is exact on
  such a polynomial);
* the solution of Algorithms 1-2 (a different code path from the system's
  assembly) has a zero residual to rounding;
* changing one interior value changes exactly the PDE rows of its leaf and
  the flux rows of that leaf's Gauss nodes, and a wrong sign on g is caught.
"""

import numpy as np
import pytest

import oracle
import workloads as W
from oracle.leaf import leaf_geometry

from oracle_cases import leaf_nodes, make_inputs


def _scaled(K, r):
    """Residual rows scaled by the largest entry of their row of K (the rows
    mix derivative scales of order (2/h)^2 with unit interpolation rows)."""
    return r / abs(K).max(axis=1).toarray().ravel()


def _exact_x(t, q, sol, xy):
    node_xy, _ = t.gauss(q)
    return sol.u(xy[..., 0], xy[..., 1]), sol.u(node_xy[:, 0], node_xy[:, 1])


@pytest.mark.parametrize("bc,n,p,q,refine", [
    ("DDDD", 3, 8, 7, None), ("DDDD", 2, 8, 6, (0.3, 0.7, 2)),
    ("NDND", 3, 10, 9, None), ("NNNN", 3, 10, 8, None)])
def test_residual_vanishes_on_polynomial_solutions(bc, n, p, q, refine):
    t = oracle.Tree.uniform(0, 1, 0, 1, n, n)
    t.set_bc(bc)
    if refine:
        t.refine_point(0, *refine)
    sol = W.PolySolution(3, q - 1)
    xy = leaf_nodes(t, p)
    coeffs = np.stack([W.varcoeff(xy[i, :, 0], xy[i, :, 1]) for i in range(len(xy))])
    I_ci, _, _ = leaf_geometry(p)
    g = np.stack([sol.g(xy[i, I_ci, 0], xy[i, I_ci, 1], coeffs[i][:, I_ci])
                  for i in range(len(xy))])
    node_xy, bdry = t.gauss(q)
    kind = t.bdry_kind(q)
    f = W.side_data(sol, node_xy[bdry], kind, (0.0, 1.0, 0.0, 1.0))
    uc, u = _exact_x(t, q, sol, xy)
    r, lay = oracle.residual(t, coeffs, p, q, uc, u, f, g)
    K, _ = oracle.assemble_system(t, coeffs, p, q)
    assert np.abs(_scaled(K, r)).max() <= 1e-11 * np.abs(uc).max()
    # the same values with the load's sign flipped are far from a solution
    r2, _ = oracle.residual(t, coeffs, p, q, uc, u, f, -g)
    assert np.abs(_scaled(K, r2)).max() > 1e-3 * np.abs(uc).max()


def test_residual_of_the_hps_solution_vanishes():
    t = oracle.Tree.uniform(0, 1, 0, 1, 3, 3)
    t.refine_point(0, 0.4, 0.55, 1)
    p, q = 8, 7
    coeffs, f, g, _ = make_inputs(t, p, q, W.varcoeff, W.FourierSolution(9))
    uc, u = oracle.solve(oracle.build(t, coeffs, p, q), f, g)
    r, _ = oracle.residual(t, coeffs, p, q, uc, u, f, g)
    K, _ = oracle.assemble_system(t, coeffs, p, q)
    assert np.abs(_scaled(K, r)).max() <= 1e-11 * np.abs(uc).max()


def test_residual_rows_touched_by_one_value():
    t = oracle.Tree.uniform(0, 1, 0, 1, 3, 3)
    p, q = 8, 7
    coeffs, f, g, _ = make_inputs(t, p, q, W.varcoeff, W.FourierSolution(9))
    uc, u = oracle.solve(oracle.build(t, coeffs, p, q), f, g)
    r0, lay = oracle.residual(t, coeffs, p, q, uc, u, f, g)
    leaf, node = 4, 3 * p + 3                 # the centre leaf, an interior node
    uc2 = uc.copy()
    uc2[leaf, node] += 1.0
    r1, _ = oracle.residual(t, coeffs, p, q, uc2, u, f, g)
    changed = np.nonzero(np.abs(r1 - r0) > 1e-9)[0]
    e1 = set(lay["e1_rows"][leaf].tolist())
    nl_rows = lay["nl"] * ((p - 2) ** 2 + 4 * (p - 1))
    pde = [k for k in changed if k < nl_rows]
    flux = [k for k in changed if k >= nl_rows]
    assert set(pde) <= e1 and len(pde) > 0
    assert 0 < len(flux) <= 4 * q             # flux rows of the leaf's own Gauss nodes
