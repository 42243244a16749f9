"""Pins for the oracle's tree, merge and full solve (Sec. 4, Algorithms 1-2,
Sec. 6): brute force against the global collocation system, exactness on
harmonic and on arbitrary low-degree polynomials, the physical meaning of the
merge, split-order invariance, refinement counts and spectral convergence."""

import os

import numpy as np
import pytest

import oracle
import workloads as W

from oracle_cases import Poisson, leaf_nodes, make_inputs, relerr

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_uniform_tree_shape_and_node_count():
    for n in (1, 2, 4, 8):
        t = oracle.Tree.uniform(0, 1, 0, 1, n, n)
        q = 7
        xy, bd = t.gauss(q)
        assert len(t.leaves) == n * n
        assert len(t.boxes) == 2 * n * n - 1
        assert xy.shape[0] == 2 * n * (n + 1) * q
        assert bd.size == 4 * n * q
        for b in t.boxes:                       # parent numbered before child
            if not b.is_leaf:
                assert b.alpha.id > b.id and b.beta.id > b.id
    t = oracle.Tree.uniform(0, 1, 0, 1, 4, 4)
    assert t.boxes[0].cut == "x"               # square: x first
    assert t.boxes[0].alpha.cut == "y"         # then the longer side


def test_refinement_leaf_counts_from_paper():
    rows = np.atleast_2d(np.loadtxt(os.path.join(GOLD, "refine_counts.txt"),
                                    comments="#"))
    for n, nref, px, py, nleaves in rows:
        t = oracle.Tree.uniform(0, 1, 0, 1, int(n), int(n))
        if nref:
            t.refine_point(0, px, py, int(nref))
        assert len(t.leaves) == int(nleaves)


def test_dtn_exact_on_harmonic_polynomials_every_box():
    p, q = 10, 9
    t = oracle.Tree.uniform(0, 1, 0, 1, 4, 4)
    xy = leaf_nodes(t, p)
    coeffs = np.stack([W.poisson_coeffs(xy[i, :, 0], xy[i, :, 1])
                       for i in range(len(xy))])
    ops = oracle.build(t, coeffs, p, q)
    node_xy, _ = t.gauss(q)
    z = node_xy[:, 0] + 1j * node_xy[:, 1]
    # vertical-side nodes have x on the leaf grid lines: flux = d/dx there
    xs = set(np.round(np.linspace(0, 1, 5), 12))
    vert = np.array([round(x, 12) in xs and round(y, 12) not in xs
                     for x, y in node_xy])
    for k in range(1, q):
        for part in (np.real, np.imag):
            d = part(z ** k)
            fx = part(k * z ** (k - 1))
            fy = part(1j * k * z ** (k - 1))
            ref = np.where(vert, fx, fy)
            for b in t.boxes:
                Tb = ops.box[b.id]["T"]
                got = Tb @ d[b.ge]
                np.testing.assert_allclose(got, ref[b.ge], atol=1e-8 * max(1, np.abs(ref).max()))


@pytest.mark.parametrize("n,p", [(2, 8), (4, 8), (2, 12), (4, 12)])
def test_hps_matches_dense_collocation(n, p):
    q = p - 1
    t = oracle.Tree.uniform(0, 1, 0, 1, n, n)
    coeffs, f, g, _ = make_inputs(t, p, q, W.varcoeff, W.FourierSolution(2))
    uc, _ = oracle.solve(oracle.build(t, coeffs, p, q), f, g)
    ud, _ = oracle.dense_solve(t, coeffs, p, q, f, g)
    assert relerr(uc, ud) < 1e-11


def test_workload1_matches_dense_and_exact():
    p, q = 16, 15
    t = oracle.Tree.uniform(0, 1, 0, 1, 4, 4)
    coeffs, f, g, ex = make_inputs(t, p, q, W.poisson_coeffs, Poisson())
    uc, _ = oracle.solve(oracle.build(t, coeffs, p, q), f, g)
    ud, _ = oracle.dense_solve(t, coeffs, p, q, f, g)
    assert relerr(uc, ud) < 1e-11
    assert relerr(uc, ex) < 1e-12


@pytest.mark.parametrize("n,p,deg", [(4, 8, 6), (3, 10, 8), (8, 6, 4)])
def test_polynomial_reproduction_variable_coefficients(n, p, deg):
    """Every operator is exact on tensor degree <= q-1, and K is nonsingular,
    so such a u is reproduced to roundoff on any tree."""
    q = p - 1
    t = oracle.Tree.uniform(0, 1, 0, 1, n, n)
    coeffs, f, g, ex = make_inputs(t, p, q, W.varcoeff, W.PolySolution(5, deg))
    uc, u = oracle.solve(oracle.build(t, coeffs, p, q), f, g)
    assert relerr(uc, ex) < 1e-12
    node_xy, _ = t.gauss(q)
    assert relerr(u, W.PolySolution(5, deg).u(node_xy[:, 0], node_xy[:, 1])) < 1e-12


def test_split_order_invariance():
    p, q = 10, 9
    res = []
    for tie in ("x", "y"):
        t = oracle.Tree.uniform(0, 1, 0, 1, 4, 4, tie=tie)
        coeffs, f, g, _ = make_inputs(t, p, q, W.varcoeff, W.FourierSolution(4))
        res.append(oracle.solve(oracle.build(t, coeffs, p, q), f, g)[0])
    assert oracle.Tree.uniform(0, 1, 0, 1, 4, 4, tie="y").boxes[0].cut == "y"
    assert relerr(res[0], res[1]) < 1e-11


def test_merge_particular_solution_meaning():
    """Sec. 5.3 remark: w_gi of a parent equals the zero-Dirichlet particular
    solution of that parent box on its interior edge; computed here by the
    global collocation system posed on the parent box alone."""
    p, q = 10, 9
    t = oracle.Tree.uniform(0, 1, 0, 1, 4, 4)
    sol = W.FourierSolution(6)
    coeffs, f, g, _ = make_inputs(t, p, q, W.varcoeff, sol)
    ops = oracle.build(t, coeffs, p, q)
    node_xy, _ = t.gauss(q)
    # recompute w of every parent with the upward pass of the solve
    _, _ = oracle.solve(ops, f, g)
    tau = t.boxes[0].alpha                     # west half, 2 x 4 leaves
    x0, x1, y0, y1 = t.box_phys(tau)
    sub = oracle.Tree.uniform(x0, x1, y0, y1, 2, 4)
    cs, _, gs, _ = make_inputs(sub, p, q, W.varcoeff, sol)
    sxy, sbd = sub.gauss(q)
    _, us = oracle.dense_solve(sub, cs, p, q, np.zeros(sbd.size), gs)
    # w for tau via the upward pass only
    h, w = {}, {}
    leaves = t.leaves
    pos = {b.id: i for i, b in enumerate(leaves)}
    for b in reversed(t.boxes):
        o = ops.box[b.id]
        if b.is_leaf:
            h[b.id] = o["H"] @ g[pos[b.id]]
            continue
        p1a, p2b, p3a, p3b = o["idx"]
        ha, hb = h[b.alpha.id], h[b.beta.id]
        w[b.id] = o["X"] @ (-ha[p3a] + hb[p3b])
        h[b.id] = np.concatenate([ha[p1a], hb[p2b]]) + o["Q"] @ w[b.id]
    # match tau's interior nodes to the sub-tree's nodes by coordinates
    key = {tuple(np.round(xy, 12)): j for j, xy in enumerate(sxy)}
    idx = [key[tuple(np.round(node_xy[j], 12))] for j in tau.gi]
    np.testing.assert_allclose(w[tau.id], us[idx], atol=1e-11 * np.abs(us).max())


@pytest.mark.parametrize("base,pt,nref,p", [(2, (0.3, 0.6), 2, 8),
                                           (4, (0.37, 0.61), 3, 8),
                                           (2, (0.5, 0.5), 3, 9)])
def test_refined_tree_matches_dense_and_reproduces_polynomials(base, pt, nref, p):
    q = p - 1
    t = oracle.Tree.uniform(0, 1, 0, 1, base, base)
    t.refine_point(0, pt[0], pt[1], nref)
    coeffs, f, g, _ = make_inputs(t, p, q, W.varcoeff, W.FourierSolution(9))
    uc, _ = oracle.solve(oracle.build(t, coeffs, p, q), f, g)
    ud, _ = oracle.dense_solve(t, coeffs, p, q, f, g)
    assert relerr(uc, ud) < 1e-11
    poly = W.PolySolution(10, q - 1)
    coeffs, f, g, ex = make_inputs(t, p, q, W.varcoeff, poly)
    uc, _ = oracle.solve(oracle.build(t, coeffs, p, q), f, g)
    assert relerr(uc, ex) < 1e-12


def test_two_panel_interface_operators_are_paper_blocks():
    """Sec. 6.3: for a side with 2q fine nodes against q coarse ones, P_down
    is two q/2 x q blocks (q even) and P_up reproduces the coarse data."""
    p, q = 9, 8
    t = oracle.Tree.uniform(0, 1, 0, 1, 2, 2)
    t.refine_point(0, 0.1, 0.1, 1)             # refines the SW leaf only
    t.gauss(q)
    coarsened = [b for b in t.boxes if b.cblocks]
    assert len(coarsened) == 1
    blocks = coarsened[0].cblocks
    assert len(blocks) == 2                    # its E and N sides
    for (on, coarse, Pup, Pdn) in blocks:
        assert Pup.shape == (2 * q, q) and Pdn.shape == (q, 2 * q)
        np.testing.assert_allclose(Pdn[:q // 2, q:], 0.0)
        np.testing.assert_allclose(Pdn[q // 2:, :q], 0.0)
        np.testing.assert_allclose(Pup.sum(1), 1.0, atol=1e-12)
        np.testing.assert_allclose(Pdn.sum(1), 1.0, atol=1e-12)


def test_spectral_convergence_workload1():
    errs = []
    for p in (6, 8, 10, 12, 14):
        q = p - 1
        t = oracle.Tree.uniform(0, 1, 0, 1, 2, 2)
        coeffs, f, g, ex = make_inputs(t, p, q, W.poisson_coeffs, Poisson())
        uc, _ = oracle.solve(oracle.build(t, coeffs, p, q), f, g)
        errs.append(relerr(uc, ex))
    errs = np.array(errs)
    assert errs[-1] < 1e-12
    assert np.all(errs[1:] < errs[:-1] * 0.5) or errs[-1] < 1e-13
    assert errs[0] > 1e-9                      # not trivially exact
