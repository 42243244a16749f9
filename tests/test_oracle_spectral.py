"""Pins for the oracle's spectral primitives (closed forms, exactness)."""

import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    return np.loadtxt(os.path.join(GOLD, name), comments="#")


def legendre_eval(n, x):
    """P_n(x) by the three-term recurrence (n+1)P_{n+1} = (2n+1)xP_n - nP_{n-1}."""
    p0, p1 = np.ones_like(x), x.copy()
    if n == 0:
        return p0
    for k in range(1, n):
        p0, p1 = p1, ((2 * k + 1) * x * p1 - k * p0) / (k + 1)
    return p1


def test_cheb_diff_golden_p3():
    D = oracle.diff_matrix(oracle.cheb_nodes(3))
    np.testing.assert_allclose(D, _load("cheb_diff_p3.txt"), atol=1e-15)


def test_gauss_golden_q3():
    np.testing.assert_allclose(oracle.gauss_nodes(3), _load("gauss_q3.txt"),
                               atol=1e-15)


@pytest.mark.parametrize("p", [4, 9, 12, 16, 20])
def test_cheb_nodes_are_extrema_of_T(p):
    x = oracle.cheb_nodes(p)
    assert np.all(np.diff(x) > 0) and x[0] == -1.0 and x[-1] == 1.0
    # T_{p-1}(x_j) = cos((p-1) arccos x_j) = +-1 alternately
    T = np.cos((p - 1) * np.arccos(np.clip(x, -1, 1)))
    np.testing.assert_allclose(np.abs(T), 1.0, atol=1e-13)
    np.testing.assert_allclose(x, -x[::-1], atol=1e-15)


@pytest.mark.parametrize("p", [5, 12, 16])
def test_diff_exact_on_monomials(p):
    # Sec. 3.2: exact for polynomials of degree <= p-1
    x = oracle.cheb_nodes(p)
    D = oracle.diff_matrix(x)
    for k in range(p):
        d = D @ x ** k
        ref = k * x ** (k - 1) if k else np.zeros_like(x)
        np.testing.assert_allclose(d, ref, atol=1e-11 * max(1, k * k))


@pytest.mark.parametrize("q", [3, 8, 11, 14, 15, 16])
def test_gauss_nodes_are_legendre_roots(q):
    x = oracle.gauss_nodes(q)
    assert x.size == q and np.all(np.diff(x) > 0)
    assert np.all(np.abs(x) < 1.0)
    np.testing.assert_allclose(legendre_eval(q, x), 0.0, atol=1e-13)
    np.testing.assert_allclose(x, -x[::-1], atol=1e-15)


@pytest.mark.parametrize("n", [3, 8, 15])
def test_interp_exact_on_polynomials(n):
    rng = np.random.default_rng(0)
    src = oracle.gauss_nodes(n)
    dst = np.linspace(-1.2, 1.2, 17)          # includes extrapolation
    P = oracle.interp_matrix(src, dst)
    for deg in range(n):
        c = rng.standard_normal(deg + 1)
        np.testing.assert_allclose(P @ np.polyval(c, src), np.polyval(c, dst),
                                   atol=1e-11)
    # partition of unity and the identity on the nodes themselves
    np.testing.assert_allclose(P.sum(1), 1.0, atol=1e-12)
    np.testing.assert_allclose(oracle.interp_matrix(src, src), np.eye(n),
                               atol=1e-15)
