"""GPU checks of the storage-economic version (the remark on a storage
efficient version, Sec. 5.4): the leaf operators F are not stored, and every
solve redoes the leaf Gauss-Jordan eliminations (in chunks of 1024 leaves)
to form u_ci = S_ci u_ge + F g.  The result is the same map as the stored
build's: against the oracle on small trees (to the FP64 parity tolerance)
and against the stored build at full size (to rounding, since the same
kernels form the same F and only the order of the two products in u_ci
changes).
"""

import numpy as np
import pytest

import workloads as W

from gpu_cases import lib_inputs, oracle_solution, relerr, to_dev

import oracle

pytestmark = pytest.mark.gpu

TOL = 1e-11


def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1612_02736_amd as H
    H.lib()
    return H


@pytest.mark.parametrize("nx,ny,p,refine", [(4, 4, 16, None), (3, 5, 12, None),
                                            (2, 2, 8, (0.3, 0.6, 2))])
def test_economic_matches_oracle(nx, ny, p, refine):
    H = _lib()
    q = p - 1
    print(f"economic nx={nx} ny={ny} p={p} refine={refine}", flush=True)
    t = H.Tree(0, 1, 0, 1, nx, ny)
    ot = oracle.Tree.uniform(0, 1, 0, 1, nx, ny)
    if refine:
        t.refine_point(0, *refine)
        ot.refine_point(0, *refine)
    sol = W.FourierSolution(2)
    coeffs, f, g, _ = lib_inputs(t, p, q, W.varcoeff, sol)
    s = H.Solver(t, to_dev(coeffs), p, q, economic=True)
    u = s.solve(to_dev(f[None]), to_dev(g[None]))[0].cpu().numpy()
    uo, _ = oracle_solution(ot, p, q, W.varcoeff, sol)
    print(f"  rel err {relerr(u, uo):.2e}", flush=True)
    assert relerr(u, uo) <= TOL


@pytest.mark.parametrize("n,p,nrhs", [(64, 16, 32), (64, 16, 1), (40, 12, 20)])
def test_economic_equals_stored_full_size(n, p, nrhs):
    """64 x 64 leaves (4 chunks of 1024) and 40 x 40 (a ragged second chunk
    of 576), against the stored build on the same inputs; then a refactor of
    the economic handle (graph replay of the chunked build) and the same
    check again."""
    import torch
    H = _lib()
    q = p - 1
    print(f"economic vs stored {n}x{n} p={p} nrhs={nrhs}", flush=True)
    t = H.Tree(0, 1, 0, 1, n, n)
    xy = t.leaf_cheb_nodes(p)
    ph = W.problem_phases(11)
    coeffs = np.stack([W.varcoeff(xy[i, :, 0], xy[i, :, 1], ph) for i in range(t.n_leaves)])
    rng = np.random.default_rng(n + nrhs)
    ng, nb = t.counts(q)
    F = rng.standard_normal((nrhs, nb))
    G = rng.standard_normal((nrhs, t.n_leaves, (p - 2) ** 2))
    cd = to_dev(coeffs)
    fd, gd = to_dev(F), to_dev(G)
    us = H.Solver(t, cd, p, q).solve(fd, gd).cpu().numpy()
    se = H.Solver(t, cd, p, q, economic=True)
    ue = se.solve(fd, gd).cpu().numpy()
    torch.cuda.synchronize()
    err = relerr(ue, us)
    print(f"  rel diff {err:.2e}", flush=True)
    assert err <= 1e-13
    se.refactor(cd)
    ue2 = se.solve(fd, gd).cpu().numpy()
    assert relerr(ue2, us) <= 1e-13


def test_economic_rejects_adjoint_and_mixed():
    H = _lib()
    import torch
    p, q = 8, 7
    t = H.Tree(0, 1, 0, 1, 2, 2)
    coeffs, f, g, _ = lib_inputs(t, p, q, W.varcoeff, W.FourierSolution(2))
    s = H.Solver(t, to_dev(coeffs), p, q, economic=True)
    fd, gd = to_dev(f[None]), to_dev(g[None])
    with pytest.raises(H.HPSError):
        s.solve(fd, gd, precision=H.HPS_PREC_MIXED)
    with pytest.raises(H.HPSError):
        s.solve_adjoint(torch.zeros((1, t.n_leaves, p * p), dtype=torch.float64, device=fd.device))
