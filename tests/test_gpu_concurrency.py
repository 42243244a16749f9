"""Factorizations and solves in flight on several streams at once.

The interface inversions of the upper merge levels run as one launch per
level whose workgroups wait for each other's panels; a workgroup whose next
panel's owner cannot be scheduled (the device is shared with the other
streams' kernels) retires and leaves its later panels to a remainder kernel.
The results must not depend on which path a strip took: every strip applies
the same panel halves in the same order either way, so the solutions are
bitwise those of the same factorization run alone.
"""

import threading

import numpy as np
import pytest

import workloads as W
from gpu_cases import PoissonSol, lib_inputs, to_dev

pytestmark = pytest.mark.gpu


def test_concurrent_factorizations_match_sequential():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1612_02736_amd as H
    n, p, q, nstreams, steps = 64, 16, 15, 4, 3
    print(f"concurrent factorizations: {n}x{n} leaves, p={p}, {nstreams} streams x {steps}",
          flush=True)
    t = H.Tree(0.0, 1.0, 0.0, 1.0, n, n)
    coeffs, f, g, _ = lib_inputs(t, p, q, W.varcoeff, PoissonSol())
    cd, fd, gd = to_dev(coeffs), to_dev(f[None]), to_dev(g[None])
    ref = H.Solver(t, cd, p, q).solve(fd, gd)
    torch.cuda.synchronize()
    sols = [H.Solver(t, cd, p, q) for _ in range(nstreams)]
    streams = [torch.cuda.Stream() for _ in range(nstreams)]
    outs = [[] for _ in range(nstreams)]
    errors = []

    def worker(i):
        try:
            for _ in range(steps):
                sols[i].refactor(cd, stream=streams[i])
                outs[i].append(sols[i].solve(fd, gd, stream=streams[i]))
        except Exception as e:            # reported after the join
            errors.append(e)

    th = [threading.Thread(target=worker, args=(i,)) for i in range(nstreams)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    torch.cuda.synchronize()
    if errors:
        raise errors[0]
    for i in range(nstreams):
        assert len(outs[i]) == steps
        for u in outs[i]:
            assert torch.equal(u, ref)
