"""GPU checks of translation-invariant builds (constant coefficients, the
remark after the timings of Sec. 7.1): boxes with the same shape and
position in their parent share one copy of their operators, built once.
Shared operators come from the same kernels on the same inputs, so the
solution equals the full build's to rounding; the small case is also
checked against the oracle.
"""

import numpy as np
import pytest

import oracle
import workloads as W

from gpu_cases import PoissonSol, lib_inputs, oracle_solution, relerr, to_dev

pytestmark = pytest.mark.gpu


def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1612_02736_amd as H
    H.lib()
    return H


def test_dedup_poisson_4x4_p16_matches_oracle_and_full_build():
    H = _lib()
    p, q = 16, 15
    t = H.Tree(0, 1, 0, 1, 4, 4)
    ot = oracle.Tree.uniform(0, 1, 0, 1, 4, 4)
    sol = PoissonSol()
    coeffs, f, g, _ = lib_inputs(t, p, q, W.poisson_coeffs, sol)
    cd, fd, gd = to_dev(coeffs), to_dev(f[None]), to_dev(g[None])
    ud = H.Solver(t, cd, p, q, translation_invariant=True).solve(fd, gd)[0].cpu().numpy()
    uf = H.Solver(t, cd, p, q).solve(fd, gd)[0].cpu().numpy()
    uo, _ = oracle_solution(ot, p, q, W.poisson_coeffs, sol)
    print(f"dedup vs oracle {relerr(ud, uo):.2e}, vs full {relerr(ud, uf):.2e}", flush=True)
    assert relerr(ud, uo) <= 1e-11
    assert relerr(ud, uf) <= 1e-14


def test_dedup_heat_128x128_p12_full_size():
    """(I - dt Lap) u = g on 128 x 128 leaves, p = 12, 32 right-hand sides:
    the shared build against the full one (FP64), then a mixed-precision
    solve and a refactor with a new time step on the shared handle."""
    import torch
    H = _lib()
    n, p, q, nrhs = 128, 12, 11, 32
    print(f"dedup heat {n}x{n} p={p} nrhs={nrhs}", flush=True)
    t = H.Tree(0, 1, 0, 1, n, n)
    xy = t.leaf_cheb_nodes(p)
    coeffs = np.stack([W.heat_coeffs(xy[i, :, 0], xy[i, :, 1]) for i in range(t.n_leaves)])
    rng = np.random.default_rng(5)
    ng, nb = t.counts(q)
    fd = to_dev(rng.standard_normal((nrhs, nb)))
    gd = to_dev(rng.standard_normal((nrhs, t.n_leaves, (p - 2) ** 2)))
    cd = to_dev(coeffs)
    uf = H.Solver(t, cd, p, q).solve(fd, gd).cpu().numpy()
    sd = H.Solver(t, cd, p, q, keep_fp32=True, translation_invariant=True)
    ud = sd.solve(fd, gd).cpu().numpy()
    err = relerr(ud, uf)
    print(f"  dedup vs full {err:.2e}", flush=True)
    assert err <= 1e-14
    um = sd.solve(fd, gd, precision=H.HPS_PREC_MIXED).cpu().numpy()
    print(f"  mixed vs full {relerr(um, uf):.2e}", flush=True)
    assert relerr(um, uf) <= 1e-10
    c2 = np.stack([W.heat_coeffs(xy[i, :, 0], xy[i, :, 1], dt=2e-3) for i in range(t.n_leaves)])
    c2d = to_dev(c2)
    sd.refactor(c2d)
    ur = sd.solve(fd, gd).cpu().numpy()
    u2 = H.Solver(t, c2d, p, q).solve(fd, gd).cpu().numpy()
    torch.cuda.synchronize()
    assert relerr(ur, u2) <= 1e-14


def test_dedup_rejects_varying_coefficients_and_refined_trees():
    H = _lib()
    p, q = 8, 7
    t = H.Tree(0, 1, 0, 1, 2, 2)
    coeffs, _, _, _ = lib_inputs(t, p, q, W.varcoeff, W.FourierSolution(2))
    with pytest.raises(H.HPSError):
        H.Solver(t, to_dev(coeffs), p, q, translation_invariant=True)
    tr = H.Tree(0, 1, 0, 1, 4, 4).refine_point(0, 0.3, 0.6, 2)   # refined interfaces
    cr, _, _, _ = lib_inputs(tr, p, q, W.poisson_coeffs, PoissonSol())
    with pytest.raises(H.HPSError):
        H.Solver(tr, to_dev(cr), p, q, translation_invariant=True)
    s = H.Solver(t, to_dev(lib_inputs(t, p, q, W.poisson_coeffs, PoissonSol())[0]), p, q,
                 translation_invariant=True)
    with pytest.raises(H.HPSError):
        s.refactor(to_dev(coeffs))
