"""GPU parity: the HIP build + solve (through the C ABI) against the oracle.

Tolerance: relative max-norm error <= 1e-11 for FP64 paths (the stated target;
both sides are FP64 with different but backward-stable elimination orders).
"""

import sys

import numpy as np
import pytest

import oracle
import workloads as W

from gpu_cases import (PoissonSol, lib_inputs, oracle_solution, relerr, to_dev)

pytestmark = pytest.mark.gpu

TOL = 1e-11


def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1612_02736_amd as H
    H.lib()
    return H


def _case(nx, ny, p, coeff_fn, sol, q=None, refine=None, nprob=1):
    H = _lib()
    q = q or p - 1
    print(f"case nx={nx} ny={ny} p={p} q={q} refine={refine}", flush=True)
    t = H.Tree(0.0, 1.0, 0.0, 1.0, nx, ny, nprob)
    ot = oracle.Tree.uniform(0.0, 1.0, 0.0, 1.0, nx, ny, nprob)
    if refine:
        for (prob, px, py, n) in refine:
            t.refine_point(prob, px, py, n)
            ot.refine_point(prob, px, py, n)
    coeffs, f, g, xy = lib_inputs(t, p, q, coeff_fn, sol)
    s = H.Solver(t, to_dev(coeffs), p, q)
    u = s.solve(to_dev(f[None]), to_dev(g[None]))[0].cpu().numpy()
    uo, ex = oracle_solution(ot, p, q, coeff_fn, sol)
    return u, uo, ex


def test_workload1_poisson_4x4_p16():
    u, uo, ex = _case(4, 4, 16, W.poisson_coeffs, PoissonSol())
    assert relerr(u, uo) <= TOL
    assert relerr(u, ex) <= 1e-12


@pytest.mark.parametrize("nx,ny,p", [(1, 1, 8), (2, 1, 8), (3, 5, 8), (4, 4, 12),
                                     (2, 4, 16), (4, 4, 16)])
def test_variable_coefficients_small(nx, ny, p):
    u, uo, _ = _case(nx, ny, p, W.varcoeff, W.FourierSolution(2))
    assert relerr(u, uo) <= TOL


def test_heat_coefficients_p12():
    class Bump:
        def u(self, x, y):
            return np.zeros_like(x)

        def g(self, x, y, c):
            return W.gaussian_bumps(x, y, seed=1)
    u, uo, _ = _case(8, 8, 12, W.heat_coeffs, Bump())
    assert relerr(u, uo) <= TOL


def test_blocked_interface_inverse_16x16():
    # the top merge has 16 * 15 = 240 interface nodes: blocked Gauss-Jordan
    u, uo, _ = _case(16, 16, 16, W.varcoeff, W.FourierSolution(3))
    assert relerr(u, uo) <= TOL


@pytest.mark.parametrize("refine,q", [([(0, 0.37, 0.61, 3)], 14), ([(0, 0.5, 0.5, 2)], 15)])
def test_refined_tree(refine, q):
    u, uo, _ = _case(4, 4, 16, W.varcoeff, W.FourierSolution(4), q=q, refine=refine)
    assert relerr(u, uo) <= TOL


def test_several_problems_refined_differently():
    refine = [(0, 0.3, 0.3, 2), (2, 0.8, 0.2, 1)]
    u, uo, _ = _case(2, 2, 12, W.varcoeff, W.FourierSolution(5), q=10, refine=refine, nprob=3)
    assert relerr(u, uo) <= TOL


@pytest.mark.parametrize("nrhs", [3, 8, 11])
def test_multiple_rhs(nrhs):
    H = _lib()
    p, q = 12, 11
    t = H.Tree(0, 1, 0, 1, 4, 4)
    ot = oracle.Tree.uniform(0, 1, 0, 1, 4, 4)
    sols = [W.FourierSolution(10 + r) for r in range(nrhs)]
    fs, gs = [], []
    for sol in sols:
        coeffs, f, g, _ = lib_inputs(t, p, q, W.varcoeff, sol)
        fs.append(f)
        gs.append(g)
    s = H.Solver(t, to_dev(coeffs), p, q)
    u = s.solve(to_dev(np.stack(fs)), to_dev(np.stack(gs))).cpu().numpy()
    for r, sol in enumerate(sols):
        uo, _ = oracle_solution(ot, p, q, W.varcoeff, sol)
        assert relerr(u[r], uo) <= TOL, r


@pytest.mark.parametrize("nrhs,p,q", [(16, 12, 11), (20, 12, 11), (32, 12, 11), (16, 16, 15),
                                      (40, 16, 15), (20, 16, 14)])
def test_many_rhs_matrix_core_path(nrhs, p, q):
    """16 or more right-hand sides take the MFMA apply path (32 per
    workgroup: 20 and 40 leave a partial block): every column agrees with
    the single-right-hand-side solve (the vector path) and two of them with
    the oracle; p = 16 with q = 14 pads the leaf level's K = 4q + 196."""
    H = _lib()
    print(f"many rhs: nrhs={nrhs} p={p} q={q}", flush=True)
    t = H.Tree(0, 1, 0, 1, 4, 4)
    ot = oracle.Tree.uniform(0, 1, 0, 1, 4, 4)
    sols = [W.FourierSolution(40 + r) for r in range(nrhs)]
    fs, gs = [], []
    for sol in sols:
        coeffs, f, g, _ = lib_inputs(t, p, q, W.varcoeff, sol)
        fs.append(f)
        gs.append(g)
    s = H.Solver(t, to_dev(coeffs), p, q)
    F, G = np.stack(fs), np.stack(gs)
    u = s.solve(to_dev(F), to_dev(G)).cpu().numpy()
    for r in range(nrhs):
        u1 = s.solve(to_dev(F[r:r + 1]), to_dev(G[r:r + 1]))[0].cpu().numpy()
        assert relerr(u[r], u1) <= 1e-13, r
    for r in (0, nrhs - 1):
        uo, _ = oracle_solution(ot, p, q, W.varcoeff, sols[r])
        assert relerr(u[r], uo) <= TOL, r


def test_polynomial_reproduction_full_size_64x64():
    """A solution of tensor degree <= q-1 is reproduced to roundoff on any
    tree for the full variable-coefficient operator.  The FP64 floor at this
    size is measured, not extrapolated: the oracle's own error on the same
    polynomial is stored by tests/golden/make_oracle_refs.py for both split
    orders (5.1e-12).  The library's elimination order differs again
    (Gauss-Jordan inverses with threshold pivoting, FMA contraction, its own
    summation orders); the bound allows 4x the oracle's measured floor."""
    import os
    H = _lib()
    ref = np.load(os.path.join(os.path.dirname(__file__), "golden",
                               "oracle_varcoeff_64x64_p16_seed2.npz"), allow_pickle=False)
    floor = max(float(ref["poly_err_xfirst"]), float(ref["poly_err_yfirst"]))
    p, q = 16, 15
    t = H.Tree(0, 1, 0, 1, 64, 64)
    sol = W.PolySolution(21, 6)
    coeffs, f, g, xy = lib_inputs(t, p, q, W.varcoeff, sol)
    s = H.Solver(t, to_dev(coeffs), p, q)
    u = s.solve(to_dev(f[None]), to_dev(g[None]))[0].cpu().numpy()
    ex = sol.u(xy[..., 0], xy[..., 1])
    err = relerr(u, ex)
    print(f"64x64 polynomial: library {err:.3e}, oracle floor {floor:.3e}", flush=True)
    assert err <= 4.0 * floor


def test_singular_and_nonfinite_inputs_are_reported():
    H = _lib()
    p = 8
    t = H.Tree(0, 1, 0, 1, 2, 2)
    z = np.zeros((4, 6, p * p))
    with pytest.raises(H.HPSError) as e:
        H.Solver(t, to_dev(z), p)
    assert e.value.code == -3
    c = np.stack([W.varcoeff(*t.leaf_cheb_nodes(p)[i].T) for i in range(4)])
    c[2, 5, 20] = np.nan
    with pytest.raises(H.HPSError) as e:
        H.Solver(t, to_dev(c), p)
    assert e.value.code == -4


def test_full_size_workload2_against_stored_oracle():
    """64 x 64 leaves, p = 16, seeded Fourier solution (seed 2): FP64 and
    mixed-precision solves against oracle values written by
    tests/golden/make_oracle_refs.py, element by element on 436 leaves: both
    diagonals (every leaf row and column), the leaves bordering the two top
    interfaces x = 1/2 and y = 1/2, and the west column."""
    import os
    H = _lib()
    ref = np.load(os.path.join(os.path.dirname(__file__), "golden",
                               "oracle_varcoeff_64x64_p16_seed2.npz"), allow_pickle=False)
    p, q = 16, 15
    t = H.Tree(0, 1, 0, 1, 64, 64)
    coeffs, f, g, _ = lib_inputs(t, p, q, W.varcoeff, W.FourierSolution(2))
    s = H.Solver(t, to_dev(coeffs), p, q, keep_fp32=True)
    u = s.solve(to_dev(f[None]), to_dev(g[None]))[0].cpu().numpy()
    assert len(ref["leaves"]) >= 400
    err = relerr(u[ref["leaves"]], ref["u"])
    um = s.solve(to_dev(f[None]), to_dev(g[None]), precision=H.HPS_PREC_MIXED)[0].cpu().numpy()
    err_m = relerr(um[ref["leaves"]], ref["u"])
    print(f"64x64 vs stored oracle: FP64 {err:.3e}, mixed {err_m:.3e}", flush=True)
    assert err <= TOL
    assert err_m <= 1e-10


def test_refactor_graph_replays_match_fresh_builds():
    """Refactorization replays the build program as a captured HIP graph.
    Alternate two coefficient sets over several replays, with eager solves
    and synchronizations in between: every replay must give bit for bit the
    operators of a fresh (eager) build with the same coefficients."""
    import torch
    H = _lib()
    p, q = 12, 11
    t = H.Tree(0, 1, 0, 1, 8, 8)
    sol = W.FourierSolution(6)
    c1, f, g, _ = lib_inputs(t, p, q, W.varcoeff, sol)
    c2, _, _, _ = lib_inputs(t, p, q, W.heat_coeffs, sol)
    fd, gd = to_dev(np.stack([f, 2 * f])), to_dev(np.stack([g, -g]))
    refs = {}
    for name, c in (("c1", c1), ("c2", c2)):
        refs[name] = H.Solver(t, to_dev(c), p, q).solve(fd, gd).cpu().numpy()
    s = H.Solver(t, to_dev(c1), p, q)
    for i, name in enumerate(["c2", "c1", "c2", "c2", "c1"]):
        s.refactor(to_dev(c2 if name == "c2" else c1))
        u = s.solve(fd, gd).cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(u, refs[name]), (i, name)
