"""GPU: operators built into caller-owned device memory (hps_build_opts
.workspace, here a torch tensor) equal those of a library-allocated build
bitwise, survive a refactor, and a workspace that is too small or misaligned
is refused before any device work.  The workspace also holds the reference
matrices the build uploads once, so a caller must leave it untouched while
the handle lives."""

import numpy as np
import pytest

import workloads as W

from gpu_cases import lib_inputs, to_dev

pytestmark = pytest.mark.gpu


def _H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1612_02736_amd as H
    H.lib()
    return H


@pytest.mark.parametrize("nx,ny,p,economic", [(8, 8, 16, False), (6, 4, 12, True)])
def test_build_into_torch_workspace_matches_library_allocation(nx, ny, p, economic):
    import torch
    H = _H()
    print(f"workspace {nx}x{ny} p={p} economic={economic}", flush=True)
    t = H.Tree(0, 1, 0, 1, nx, ny)
    coeffs, f, g, _ = lib_inputs(t, p, p - 1, W.varcoeff, W.FourierSolution(4))
    need = t.workspace_bytes(p, p - 1, economic=economic)
    ws = torch.full((need // 8,), float("nan"), dtype=torch.float64, device="cuda")
    s_own = H.Solver(t, to_dev(coeffs), p, economic=economic)
    s_ws = H.Solver(t, to_dev(coeffs), p, economic=economic, workspace=ws)
    assert s_ws.workspace is ws
    fd, gd = to_dev(f[None]), to_dev(g[None])
    u0 = s_own.solve(fd, gd)
    assert torch.equal(u0, s_ws.solve(fd, gd))
    # the handle reads its operators (and reference matrices) from the
    # tensor: clearing it changes the solution, restoring it restores it
    saved = ws.clone()
    ws.zero_()
    assert not torch.equal(u0, s_ws.solve(fd, gd))
    ws.copy_(saved)
    assert torch.equal(u0, s_ws.solve(fd, gd))
    c2 = coeffs.copy()
    c2[:, 5] += 0.5
    s_own.refactor(to_dev(c2))
    s_ws.refactor(to_dev(c2))
    assert torch.equal(s_own.solve(fd, gd), s_ws.solve(fd, gd))


def test_workspace_too_small_or_misaligned_is_refused():
    import torch
    H = _H()
    t = H.Tree(0, 1, 0, 1, 4, 4)
    coeffs, _, _, _ = lib_inputs(t, 12, 11, W.varcoeff, W.FourierSolution(4))
    need = t.workspace_bytes(12)
    small = torch.empty(need - 8, dtype=torch.uint8, device="cuda")
    with pytest.raises(H.HPSError, match="workspace holds"):
        H.Solver(t, to_dev(coeffs), 12, workspace=small)
    big = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(H.HPSError, match="aligned"):
        H.Solver(t, to_dev(coeffs), 12, workspace=big[8:])
    s = H.Solver(t, to_dev(coeffs), 12, workspace=True)
    assert s.workspace.numel() == need
