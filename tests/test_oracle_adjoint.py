"""Pins for the oracle's adjoint (transposed Algorithm 2) and the coefficient
gradient: the dot-product identity, the transposed global collocation system
and central finite differences."""

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
import workloads as W

from oracle_cases import leaf_nodes, make_inputs


def _setup(n=3, p=8, refine=None, seed=2):
    q = p - 1
    t = oracle.Tree.uniform(0, 1, 0, 1, n, n)
    if refine:
        t.refine_point(0, *refine)
    coeffs, f, g, _ = make_inputs(t, p, q, W.varcoeff, W.FourierSolution(seed))
    return t, p, q, coeffs, f, g


@pytest.mark.parametrize("refine", [None, (0.4, 0.55, 2)])
def test_dot_product_identity(refine):
    t, p, q, coeffs, f, g = _setup(refine=refine)
    ops = oracle.build(t, coeffs, p, q)
    rng = np.random.default_rng(11)
    f1 = rng.standard_normal(f.shape)
    g1 = rng.standard_normal(g.shape)
    y = rng.standard_normal((len(t.leaves), p * p))
    uc, _ = oracle.solve(ops, f1, g1)
    fb, gb = oracle.solve_adjoint(ops, y)
    lhs = np.sum(uc * y)
    rhs = np.sum(f1 * fb) + np.sum(g1 * gb)
    assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + np.abs(uc * y).sum())


def test_adjoint_matches_transposed_global_system():
    t, p, q, coeffs, f, g = _setup(n=2, p=8)
    ops = oracle.build(t, coeffs, p, q)
    rng = np.random.default_rng(12)
    y = rng.standard_normal((len(t.leaves), p * p))
    fb, gb = oracle.solve_adjoint(ops, y)
    K, lay = oracle.assemble_system(t, coeffs, p, q)
    rhs = np.zeros(lay["nunk"])
    rhs[:y.size] = y.ravel()
    lam = sla.solve(K.toarray().T, rhs)
    # g enters only the PDE rows with coefficient +1
    np.testing.assert_allclose(gb.ravel(), lam[lay["e1_rows"].ravel()],
                               rtol=1e-9, atol=1e-9 * np.abs(gb).max())
    # f enters the interpolation rows through -L f
    fref = np.zeros(f.size)
    for (r, k, wgt) in lay["e2_f"]:
        fref[k] += wgt * lam[r]
    np.testing.assert_allclose(fb, fref, rtol=1e-9, atol=1e-9 * np.abs(fb).max())


def test_coefficient_gradient_finite_differences():
    """L = sum (u_c - u_obs)^2; dL/dc along 6 seeded directions vs central
    differences with h = 1e-6 (relative change of the field)."""
    t, p, q, coeffs, f, g = _setup(n=2, p=8)
    ops = oracle.build(t, coeffs, p, q)
    rng = np.random.default_rng(100)
    u_obs = oracle.solve(ops, f, g)[0] + 0.1 * rng.standard_normal((len(t.leaves), p * p))

    def loss(c):
        uc = oracle.solve(oracle.build(t, c, p, q), f, g)[0]
        return np.sum((uc - u_obs) ** 2), uc

    L0, uc = loss(coeffs)
    _, gb = oracle.solve_adjoint(ops, 2.0 * (uc - u_obs))
    cbar = oracle.coeff_gradient(ops, uc, gb)
    for s in range(6):
        d = np.random.default_rng(100 + s).standard_normal(coeffs.shape)
        d /= np.linalg.norm(d)
        h = 1e-6
        fd = (loss(coeffs + h * d)[0] - loss(coeffs - h * d)[0]) / (2 * h)
        an = np.sum(cbar * d)
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * abs(L0)), (s, fd, an)


def _bc_setup(bc, nx, ny, p, q, refine=None, seed=4):
    t = oracle.Tree.uniform(0, 1, 0, 1, nx, ny)
    t.set_bc(bc)
    if refine:
        t.refine_point(0, *refine)
    coeffs, _, _, _ = make_inputs(t, p, q, W.varcoeff, W.FourierSolution(seed))
    return t, coeffs


BC_CASES = [("NPNP", 4, 4, 8, 6, None), ("PPPP", 4, 4, 8, 6, None),
            ("NNNN", 3, 4, 8, 6, None), ("DNDN", 4, 3, 8, 7, None),
            ("NPDP", 4, 4, 8, 7, None), ("NDDD", 3, 3, 8, 7, (0.3, 0.6, 1))]


@pytest.mark.parametrize("bc,nx,ny,p,q,refine", BC_CASES)
def test_adjoint_with_side_conditions_matches_transposed_global_system(bc, nx, ny, p, q, refine):
    """The reverse sweeps (Algorithm 2 transposed, with the Neumann closure
    reversed) against the brute-force route: lam = K^-T [ubar; 0] through the
    global collocation system, whose Neumann rows read the data and whose
    periodic seams are ordinary flux-continuity rows."""
    t, coeffs = _bc_setup(bc, nx, ny, p, q, refine)
    ops = oracle.build(t, coeffs, p, q)
    rng = np.random.default_rng(31)
    y = rng.standard_normal((len(t.leaves), p * p))
    fb, gb = oracle.solve_adjoint(ops, y)
    fd, gd = oracle.dense_adjoint(t, coeffs, p, q, y)
    scale_g, scale_f = np.abs(gd).max(), np.abs(fd).max()
    assert np.abs(gb - gd).max() <= 1e-10 * scale_g, np.abs(gb - gd).max() / scale_g
    assert np.abs(fb - fd).max() <= 1e-10 * scale_f, np.abs(fb - fd).max() / scale_f
    kind = t.bdry_kind(q)
    assert np.all(fb[kind == "P"] == 0.0)
    if "N" in bc:
        assert np.abs(fb[kind == "N"]).max() > 1e-3 * scale_f   # the Neumann data matters


@pytest.mark.parametrize("bc,nx,ny,p,q,refine", BC_CASES)
def test_adjoint_with_side_conditions_dot_product_identity(bc, nx, ny, p, q, refine):
    """<u_c(f, g), y> = <f, fbar> + <g, gbar> for the oracle's forward solve
    (Algorithm 2 with the closure), including random data on periodic
    entries, which the forward solve ignores and fbar zeroes."""
    t, coeffs = _bc_setup(bc, nx, ny, p, q, refine)
    ops = oracle.build(t, coeffs, p, q)
    rng = np.random.default_rng(32)
    _, bdry = t.gauss(q)
    f1 = rng.standard_normal(len(bdry))
    g1 = rng.standard_normal((len(t.leaves), (p - 2) ** 2))
    y = rng.standard_normal((len(t.leaves), p * p))
    uc, _ = oracle.solve(ops, f1, g1)
    fb, gb = oracle.solve_adjoint(ops, y)
    lhs = np.sum(uc * y)
    rhs = np.sum(f1 * fb) + np.sum(g1 * gb)
    assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + np.abs(uc * y).sum()), (lhs, rhs)


def test_adjoint_closure_sign_is_pinned():
    """A planted mistake in the reversed Neumann closure (the cotangent sent
    to the root's h with the wrong sign) breaks the dense-route agreement."""
    import oracle.hps as OH
    t, coeffs = _bc_setup("NNNN", 3, 3, 8, 6)
    ops = oracle.build(t, coeffs, p=8, q=6)
    y = np.random.default_rng(33).standard_normal((len(t.leaves), 64))
    _, gd = oracle.dense_adjoint(t, coeffs, 8, 6, y)
    orig = OH.sla.lu_solve

    def wrong(lu, b, trans=0):
        return -orig(lu, b, trans=trans) if trans == 1 else orig(lu, b, trans=trans)

    OH.sla.lu_solve = wrong
    try:
        _, gw = oracle.solve_adjoint(ops, y)
    finally:
        OH.sla.lu_solve = orig
    assert np.abs(gw - gd).max() > 1e-3 * np.abs(gd).max()
