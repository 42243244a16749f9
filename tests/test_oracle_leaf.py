"""Pins for the oracle's leaf operators (Sec. 3): exactness on polynomials,
harmonic polynomials, the flux sign convention and a brute-force 1-leaf solve."""

import numpy as np
import pytest

import oracle
from oracle.leaf import leaf_geometry, leaf_operators, reference_matrices
import workloads as W

from oracle_cases import leaf_nodes, make_inputs, relerr

BOX = (0.2, 0.45, -0.1, 0.3)       # a non-square leaf


def _grid(p, box=BOX):
    x0, x1, y0, y1 = box
    xc = oracle.cheb_nodes(p)
    YY, XX = np.meshgrid(y0 + (y1 - y0) * (xc + 1) / 2,
                         x0 + (x1 - x0) * (xc + 1) / 2, indexing="ij")
    return XX.ravel(), YY.ravel()


def _gauss_sides(q, box=BOX):
    """Gauss node coordinates of a leaf, sides S, E, N, W, increasing."""
    x0, x1, y0, y1 = box
    g = oracle.gauss_nodes(q)
    gx = x0 + (x1 - x0) * (g + 1) / 2
    gy = y0 + (y1 - y0) * (g + 1) / 2
    xs = np.concatenate([gx, np.full(q, x1), gx, np.full(q, x0)])
    ys = np.concatenate([np.full(q, y0), gy, np.full(q, y1), gy])
    return xs, ys


@pytest.mark.parametrize("p", [6, 10, 16])
def test_L_ce_ge_exact_and_corner_rule(p):
    q = p - 1
    _, _, L = reference_matrices(p, q)
    X, Y = _grid(p)
    I_ci, I_ce, _ = leaf_geometry(p)
    gx, gy = _gauss_sides(q)
    rng = np.random.default_rng(p)
    c = rng.standard_normal((q, q))           # total degree <= q-1 in x and y

    def u(x, y):
        return sum(c[i, j] * x ** i * y ** j for i in range(q) for j in range(q - i))
    np.testing.assert_allclose(L @ u(gx, gy), u(X[I_ce], Y[I_ce]), atol=1e-10)
    # corner rows carry weight 1/2 on each of two sides and sum to one
    corner = [k for k, idx in enumerate(I_ce)
              if idx in (0, p - 1, p * (p - 1), p * p - 1)]
    for r in corner:
        side_sum = [L[r, s * q:(s + 1) * q].sum() for s in range(4)]
        assert sorted(np.round(side_sum, 12)) == [0.0, 0.0, 0.5, 0.5]


def test_flux_sign_convention():
    # Sec. 3.1: +d/dx on both vertical sides, +d/dy on both horizontal sides
    p, q = 8, 7
    X, Y = _grid(p)
    o = leaf_operators(BOX, W.poisson_coeffs(X, Y), p, q)
    Dge = o["Dge"]
    vx = Dge @ X
    vy = Dge @ Y
    S, E, N, Wd = [slice(k * q, (k + 1) * q) for k in range(4)]
    np.testing.assert_allclose(vx[E], 1.0, atol=1e-12)
    np.testing.assert_allclose(vx[Wd], 1.0, atol=1e-12)      # not -1
    np.testing.assert_allclose(vx[S], 0.0, atol=1e-12)
    np.testing.assert_allclose(vy[S], 1.0, atol=1e-12)
    np.testing.assert_allclose(vy[N], 1.0, atol=1e-12)
    np.testing.assert_allclose(vy[E], 0.0, atol=1e-12)


@pytest.mark.parametrize("p", [8, 12, 16])
def test_dtn_exact_on_harmonic_polynomials(p):
    q = p - 1
    X, Y = _grid(p)
    o = leaf_operators(BOX, W.poisson_coeffs(X, Y), p, q)
    gx, gy = _gauss_sides(q)
    vert = np.r_[np.zeros(q), np.ones(q), np.zeros(q), np.ones(q)].astype(bool)
    for k in range(q):                         # Re/Im (x+iy)^k, degree <= q-1
        z = (gx + 1j * gy)
        dz = k * z ** (k - 1) if k else 0 * z
        for part in (np.real, np.imag):
            d = part(z ** k)
            # d/dx z^k = k z^(k-1); d/dy z^k = i k z^(k-1)
            fx = part(dz)
            fy = part(1j * dz)
            ref = np.where(vert, fx, fy)
            scale = max(1.0, np.abs(ref).max())
            np.testing.assert_allclose(o["T"] @ d, ref, atol=2e-9 * scale)
    # constants are in the kernel of the Laplace DtN map
    np.testing.assert_allclose(o["T"] @ np.ones(4 * q), 0.0, atol=1e-9)


@pytest.mark.parametrize("p", [8, 14])
def test_particular_and_full_leaf_solution_exact(p):
    """u_c = S u_ge + F g reproduces a polynomial of degree <= q-1 for the full
    variable-coefficient operator; F g alone reproduces a polynomial that
    vanishes on the leaf boundary (eqs. alpine1, alpine3)."""
    q = p - 1
    X, Y = _grid(p)
    coeffs = W.varcoeff(X, Y)
    o = leaf_operators(BOX, coeffs, p, q)
    I_ci, _, _ = leaf_geometry(p)
    sol = W.PolySolution(7, q - 1)
    gx, gy = _gauss_sides(q)
    g = sol.g(X, Y, coeffs)[I_ci]
    u = o["S"] @ sol.u(gx, gy) + o["F"] @ g
    assert relerr(u, sol.u(X, Y)) < 1e-12
    # bubble: (x-x0)(x1-x)(y-y0)(y1-y) * poly(deg p-3)
    x0, x1, y0, y1 = BOX
    inner = W.PolySolution(8, p - 3)

    class Bubble:
        def derivs(self, x, y):
            b = (x - x0) * (x1 - x) * (y - y0) * (y1 - y)
            bx = ((x1 - x) - (x - x0)) * (y - y0) * (y1 - y)
            by = (x - x0) * (x1 - x) * ((y1 - y) - (y - y0))
            bxx = -2.0 * (y - y0) * (y1 - y)
            byy = -2.0 * (x - x0) * (x1 - x)
            bxy = ((x1 - x) - (x - x0)) * ((y1 - y) - (y - y0))
            v, vx, vy, vxx, vxy, vyy = inner.derivs(x, y)
            return (b * v, bx * v + b * vx, by * v + b * vy,
                    bxx * v + 2 * bx * vx + b * vxx,
                    bxy * v + bx * vy + by * vx + b * vxy,
                    byy * v + 2 * by * vy + b * vyy)
    bub = Bubble()
    gb = W.apply_A(coeffs, *bub.derivs(X, Y))[I_ci]
    assert relerr(o["F"] @ gb, bub.derivs(X, Y)[0]) < 1e-11
    # H = D_ge,c F and T = D_ge,c S by definition (eq. alpine4)
    np.testing.assert_allclose(o["H"], o["Dge"] @ o["F"], atol=1e-12 * np.abs(o["H"]).max())


def test_single_leaf_matches_direct_collocation():
    """A 1-leaf tree: Algorithm 2 against the directly solved collocation
    system (brute force)."""
    p, q = 10, 9
    tree = oracle.Tree.uniform(0.0, 1.0, 0.0, 1.0, 1, 1)
    coeffs, f, g, _ = make_inputs(tree, p, q, W.varcoeff, W.FourierSolution(3))
    ops = oracle.build(tree, coeffs, p, q)
    uc, _ = oracle.solve(ops, f, g)
    ud, _ = oracle.dense_solve(tree, coeffs, p, q, f, g)
    assert relerr(uc, ud) < 1e-12
