"""GPU: the allocation-free solve (hps_solve_noalloc, work memory in the
library's fixed device array) against hps_solve on the same handle, through
the C ABI.  Both run the same kernels on the same descriptors, so the results
must agree bitwise; two calls in a row, the second with a smaller input (a
smaller tree and fewer right-hand sides), check that the array's leftover
contents never leak into a later solve.  The parity bar of the FP64 path
(<= 1e-11 against the oracle) is checked on the smaller case as well.  The
file is collected last, so that a failure here cannot hide other tests.
"""

import numpy as np
import pytest

import oracle
import workloads as W

from gpu_cases import lib_inputs, oracle_solution, relerr, to_dev

pytestmark = pytest.mark.gpu


def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1612_02736_amd as H
    H.lib()
    return H


def _problem(H, n, p, nrhs, keep_fp32=False):
    q = p - 1
    t = H.Tree(0.0, 1.0, 0.0, 1.0, n, n)
    fs, gs = [], []
    coeffs = None
    for r in range(nrhs):
        coeffs, f, g, _ = lib_inputs(t, p, q, W.varcoeff, W.FourierSolution(2 + r))
        fs.append(f)
        gs.append(g)
    s = H.Solver(t, to_dev(coeffs), p, q, keep_fp32=keep_fp32)
    return t, s, to_dev(np.stack(fs)), to_dev(np.stack(gs))


def _both(H, s, f, g, precision):
    import torch
    ref = s.solve(f, g, precision=precision)
    u = torch.full_like(ref, float("nan"))
    s.solve_noalloc(f, g, u, precision=precision)
    torch.cuda.synchronize()
    return ref, u


def test_noalloc_matches_solve_two_calls_second_smaller():
    import torch
    H = _lib()
    print("noalloc: 8x8 leaves p=16, 12 RHS, then 4x4 leaves p=12, 3 RHS", flush=True)
    _, s1, f1, g1 = _problem(H, 8, 16, 12)
    assert H.hps.debug_solve_work_bytes(s1, 12) <= H.HPS_SOLVE_NOALLOC_MAX_BYTES
    ref1, u1 = _both(H, s1, f1, g1, H.HPS_PREC_FP64)
    assert torch.equal(ref1, u1)
    t2, s2, f2, g2 = _problem(H, 4, 12, 3)
    ref2, u2 = _both(H, s2, f2, g2, H.HPS_PREC_FP64)
    assert torch.equal(ref2, u2)
    # the smaller case also against the oracle, right-hand side 0
    ot = oracle.Tree.uniform(0.0, 1.0, 0.0, 1.0, 4, 4)
    uo, _ = oracle_solution(ot, 12, 11, W.varcoeff, W.FourierSolution(2))
    assert relerr(u2[0].cpu().numpy(), uo) <= 1e-11
    # and the larger handle again after the smaller call
    u1b = torch.full_like(ref1, float("nan"))
    s1.solve_noalloc(f1, g1, u1b)
    torch.cuda.synchronize()
    assert torch.equal(ref1, u1b)


def test_noalloc_fp32_sweep_matches_solve():
    import torch
    H = _lib()
    print("noalloc FP32: 8x8 leaves p=16, 16 RHS (matrix-core apply), then 2 RHS", flush=True)
    _, s, f, g = _problem(H, 8, 16, 16, keep_fp32=True)
    ref, u = _both(H, s, f, g, H.HPS_PREC_FP32)
    assert torch.equal(ref, u)
    ref2, u2 = _both(H, s, f[:2].contiguous(), g[:2].contiguous(), H.HPS_PREC_FP32)
    assert torch.equal(ref2, u2)


def test_noalloc_refuses_what_it_cannot_do():
    import torch
    H = _lib()
    print("noalloc refusals: oversize nrhs, mixed precision, economic build", flush=True)
    t, s, f, g = _problem(H, 4, 12, 1, keep_fp32=True)
    per = H.hps.debug_solve_work_bytes(s, 1)
    big = H.HPS_SOLVE_NOALLOC_MAX_BYTES // per + 1
    while H.hps.debug_solve_work_bytes(s, big) <= H.HPS_SOLVE_NOALLOC_MAX_BYTES:
        big += 1
    fb = f.expand(big, -1).contiguous()
    gb = g.expand(big, -1, -1).contiguous()
    ub = torch.empty((big, s.n_leaves, s.p * s.p), dtype=torch.float64, device=f.device)
    with pytest.raises(H.HPSError, match="bytes of work memory"):
        s.solve_noalloc(fb, gb, ub)
    u = torch.empty((1, s.n_leaves, s.p * s.p), dtype=torch.float64, device=f.device)
    with pytest.raises(H.HPSError, match="FP64 or FP32"):
        s.solve_noalloc(f, g, u, precision=H.HPS_PREC_MIXED)
    coeffs, _, _, _ = lib_inputs(t, 12, 11, W.varcoeff, W.FourierSolution(2))
    se = H.Solver(t, to_dev(coeffs), 12, 11, economic=True)
    with pytest.raises(H.HPSError, match="economic"):
        se.solve_noalloc(f, g, u)
    # a refused call leaves the entry point usable
    ref, u1 = _both(H, s, f, g, H.HPS_PREC_FP64)
    assert torch.equal(ref, u1)
