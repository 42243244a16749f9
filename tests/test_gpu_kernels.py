"""Per-kernel GPU parity through the test hooks: the MFMA GEMM, the
Gauss-Jordan inversions and the stored leaf / merge operators of a build
against the oracle's operators (unit parity <= 1e-12 relative)."""

import numpy as np
import pytest

import oracle
import workloads as W

from gpu_cases import lib_inputs, relerr, to_dev
from oracle_cases import make_inputs

pytestmark = pytest.mark.gpu


def _H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1612_02736_amd as H
    H.lib()
    return H


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (17, 33, 5), (64, 64, 16), (196, 60, 196),
                                   (100, 300, 37), (130, 70, 1),
                                   (128, 128, 256), (300, 260, 301), (960, 128, 961),
                                   (129, 1000, 3)])
def test_gemm_matches_numpy(M, N, K):
    """The grouped GEMM against numpy: partial MFMA tiles, wavefronts whose
    part of a tile lies outside the matrix, and K tails that are not a
    multiple of the chunk or of the MFMA depth."""
    import torch
    from paper_1612_02736_amd.hps import debug_gemm
    rng = np.random.default_rng(M * 1000 + N + K)
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((K, N))
    print(f"gemm {M}x{N}x{K}", flush=True)
    C = debug_gemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), alpha=-0.5)
    ref = -0.5 * A @ B
    np.testing.assert_allclose(C.cpu().numpy(), ref, atol=1e-13 * max(1, np.abs(ref).max()))


@pytest.mark.parametrize("M,N,K", [(17, 33, 5), (196, 60, 196), (60, 196, 196),
                                   (300, 260, 301), (960, 130, 961), (2880, 129, 480)])
def test_gemm_tile_variants_agree_bitwise(M, N, K):
    """Every tile variant of the grouped GEMM (64 x 64, 128 x 64, 64 x 128,
    128 x 128, 32 x 32, 64 x 32, 32 x 64 with K chunks of 16, 64 x 64 with K
    chunks of 8) accumulates each output over k in the same order, so all
    give bitwise the same product; variant 0 also against numpy."""
    import torch
    from paper_1612_02736_amd.hps import debug_gemm
    rng = np.random.default_rng(M + 7 * N + 11 * K)
    A = torch.from_numpy(rng.standard_normal((M, K))).cuda()
    B = torch.from_numpy(rng.standard_normal((K, N))).cuda()
    print(f"gemm variants {M}x{N}x{K}", flush=True)
    outs = [debug_gemm(A, B, alpha=0.75, variant=v) for v in range(8)]
    for v in range(1, 8):
        assert torch.equal(outs[0], outs[v]), v
    ref = 0.75 * A.cpu().numpy() @ B.cpu().numpy()
    np.testing.assert_allclose(outs[0].cpu().numpy(), ref, atol=1e-13 * max(1, np.abs(ref).max()))


def test_gemm_tuner_choices_and_cache():
    """The first build of a handle times the tile variants on every GEMM
    step and keeps one per step; a second build of the same shapes takes the
    cached choices and solves bitwise like the first."""
    import torch
    from paper_1612_02736_amd.hps import debug_gemm_choices
    H = _H()
    t = H.Tree(0, 1, 0, 1, 8, 8)
    coeffs, f, g, _ = lib_inputs(t, 16, 15, W.varcoeff, W.FourierSolution(3))
    s1 = H.Solver(t, to_dev(coeffs), 16)
    c1 = debug_gemm_choices(s1)
    print(f"tuner choices {c1}", flush=True)
    assert len(c1) > 0 and all(0 <= v < 8 for v in c1)
    s2 = H.Solver(t, to_dev(coeffs), 16)
    assert debug_gemm_choices(s2) == c1
    u1 = s1.solve(to_dev(f[None]), to_dev(g[None]))
    u2 = s2.solve(to_dev(f[None]), to_dev(g[None]))
    assert torch.equal(u1, u2)


@pytest.mark.parametrize("n", [1, 5, 32, 33, 64, 100, 128, 196, 197, 240, 500])
def test_inverse_matches_numpy(n):
    import torch
    from paper_1612_02736_amd.hps import debug_invert
    rng = np.random.default_rng(n)
    A = rng.standard_normal((3, n, n)) + 2.0 * np.sqrt(n) * np.eye(n) * (rng.random((3, 1, 1)) > 0.5)
    print(f"invert n={n}", flush=True)
    X = debug_invert(torch.from_numpy(A).cuda()).cpu().numpy()
    for b in range(3):
        ref = np.linalg.inv(A[b])
        assert relerr(X[b], ref) < 1e-10 * np.linalg.cond(A[b]) / n


@pytest.mark.parametrize("n", [40, 196, 300, 700, 960, 1408, 1920])
def test_inverse_needs_pivoting(n):
    """One large entry per row and column at random places, the diagonal 0:
    any pivot choice other than the largest candidate meets a zero or tiny
    pivot, so this checks the pivot search of both Gauss-Jordan paths."""
    import torch
    from paper_1612_02736_amd.hps import debug_invert
    rng = np.random.default_rng(1000 + n)
    A = np.zeros((2, n, n))
    for b in range(2):
        perm = rng.permutation(n)
        while np.any(perm == np.arange(n)):
            perm = rng.permutation(n)
        A[b] = 1e-3 * rng.standard_normal((n, n))
        A[b][np.arange(n), np.arange(n)] = 0.0
        A[b][np.arange(n), perm] = 1.0 + rng.random(n)
    print(f"invert (pivoting) n={n}", flush=True)
    X = debug_invert(torch.from_numpy(A).cuda()).cpu().numpy()
    for b in range(2):
        ref = np.linalg.inv(A[b])
        assert relerr(X[b], ref) < 1e-12


# ragged last panels: 5 (197), 10 (250, the first half's counter never
# raised mid-sweep), 13 (253) and 4 (500) columns
@pytest.mark.parametrize("n", [197, 240, 250, 253, 500, 960])
def test_inverse_level_form_matches_panel_form(n, monkeypatch):
    """The blocked inversion in one launch per level (strips resident in
    registers, panels passed through memory as two rank-8 halves), the same
    with every strip retiring after its own sweep (the remainder kernel
    applies the later halves in the same order: bitwise the same), and one
    launch per panel (one rank-16 update per panel: the same inverse up to
    rounding)."""
    import torch
    from paper_1612_02736_amd.hps import debug_invert
    rng = np.random.default_rng(2000 + n)
    A = rng.standard_normal((2, n, n)) + 2.0 * np.sqrt(n) * np.eye(n)
    Ad = torch.from_numpy(A).cuda()
    out = {}
    for form in ("1", "2", "0"):
        monkeypatch.setenv("HPS_GJ_LEVEL", form)
        print(f"invert n={n} form {form}", flush=True)
        out[form] = debug_invert(Ad)
    assert torch.equal(out["1"], out["2"])
    X, X0 = out["1"].cpu().numpy(), out["0"].cpu().numpy()
    for b in range(2):
        assert relerr(X[b], X0[b]) < 1e-13
        assert relerr(X[b], np.linalg.inv(A[b])) < 1e-12


def _build_pair(nx, ny, p, q=None, refine=None, coef=W.varcoeff):
    H = _H()
    q = q or p - 1
    t = H.Tree(0, 1, 0, 1, nx, ny)
    ot = oracle.Tree.uniform(0, 1, 0, 1, nx, ny)
    if refine:
        t.refine_point(0, *refine)
        ot.refine_point(0, *refine)
    sol = W.FourierSolution(1)
    coeffs, _, _, _ = lib_inputs(t, p, q, coef, sol)
    s = H.Solver(t, to_dev(coeffs), p, q)
    oc, _, _, _ = make_inputs(ot, p, q, coef, sol)
    ops = oracle.build(ot, oc, p, q)
    return H, s, ot, ops, p, q


def _helmholtz80(x, y):
    return W.helmholtz_coeffs(x, y, kappa=80.0)


@pytest.mark.parametrize("nx,ny,p,coef", [(2, 2, 8, W.varcoeff), (2, 2, 16, W.varcoeff),
                                          (4, 4, 12, W.varcoeff), (2, 2, 16, _helmholtz80)])
def test_leaf_operators(nx, ny, p, coef):
    """Leaf operators F, S_ci, H and T against the oracle's (Sec. 3); the
    Helmholtz case (kappa = 80 on leaves of side 1/2) makes A_ci,ci strongly
    indefinite, so the pivot search leaves the diagonal."""
    print(f"leaf operators {nx}x{ny} p={p} {coef.__name__}", flush=True)
    H, s, ot, ops, p, q = _build_pair(nx, ny, p, coef=coef)
    from paper_1612_02736_amd.hps import debug_boxes, debug_box_nodes, debug_box_op
    boxes = debug_boxes(s)
    mi, g4 = (p - 2) ** 2, 4 * q
    leaves = ot.leaves
    for b, info in enumerate(boxes):
        if not info[0]:
            continue
        li = info[1]
        ob = leaves[li]
        o = ops.box[ob.id]
        fin = debug_box_nodes(s, b, 0)
        pos = {j: i for i, j in enumerate(ob.ge)}
        perm = np.array([pos[j] for j in fin])
        I_ci = o["I_ci"]
        F = debug_box_op(s, b, 3, (mi, mi))
        assert relerr(F, o["F"][I_ci]) < 1e-12, ("F", li)
        Sci = debug_box_op(s, b, 2, (mi, g4))
        assert relerr(Sci, o["S"][I_ci][:, perm]) < 1e-12, ("S", li)
        Hm = debug_box_op(s, b, 4, (g4, mi))
        assert relerr(Hm, o["H"][perm]) < 1e-12, ("H", li)
        if info[2] >= 0 or len(boxes) == 1:
            T = debug_box_op(s, b, 0, (g4, g4))
            assert relerr(T, o["T"][np.ix_(perm, perm)]) < 1e-12, ("T", li)


@pytest.mark.parametrize("nx,ny,p,refine", [(2, 2, 8, None), (4, 4, 8, None),
                                            (4, 4, 12, None), (2, 2, 8, (0.1, 0.1, 1)),
                                            (16, 16, 8, None)])
def test_merge_operators(nx, ny, p, refine):
    H, s, ot, ops, p, q = _build_pair(nx, ny, p, refine=refine)
    from paper_1612_02736_amd.hps import debug_boxes, debug_box_nodes, debug_box_op
    boxes = debug_boxes(s)
    obox = ot.boxes
    assert len(obox) == len(boxes)
    for b, info in enumerate(boxes):
        if info[0]:
            continue
        ob = obox[b]                 # both number boxes in the same pre-order
        o = ops.box[ob.id]
        ef, en, m = info[5], info[6], info[7]
        gi = debug_box_nodes(s, b, 2)
        nat = debug_box_nodes(s, b, 1)
        fin = debug_box_nodes(s, b, 0)
        assert set(gi) == set(ob.gi)
        pg = {j: i for i, j in enumerate(ob.gi)}
        ig = np.array([pg[j] for j in gi])
        X = debug_box_op(s, b, 1, (m, m))
        assert relerr(X, o["X"][np.ix_(ig, ig)]) < 1e-11, ("X", b)
        ge_f = ob.ge_fine if ob.ge_fine is not None else ob.ge
        pn = {j: i for i, j in enumerate(ge_f)}
        inat = np.array([pn[j] for j in nat])
        S = debug_box_op(s, b, 2, (m, en))
        assert relerr(S, o["S"][np.ix_(ig, inat)]) < 1e-11, ("S", b)
        if info[2] >= 0:
            pf = {j: i for i, j in enumerate(ob.ge)}
            ifin = np.array([pf[j] for j in fin])
            T = debug_box_op(s, b, 0, (ef, ef))
            assert relerr(T, o["T"][np.ix_(ifin, ifin)]) < 1e-11, ("T", b)
