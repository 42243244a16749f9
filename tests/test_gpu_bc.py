"""GPU parity of Neumann and periodic sides (Sec. 7.6) and of the implicit
time step built on them: the library against the oracle on the same seeded
inputs, at sizes that span several levels, plus the Crank-Nicolson workload
of Sec. 7.6 (16 x 16 leaves) against a closed form that holds at any size.
"""

import numpy as np
import pytest

import oracle
import workloads as W
from oracle.leaf import leaf_geometry

from gpu_cases import relerr, to_dev

pytestmark = pytest.mark.gpu


def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1612_02736_amd as H
    H.lib()
    return H


def _kinds(xy, bc, rect=(0.0, 1.0, 0.0, 1.0)):
    """Side condition of each boundary entry from its coordinates (a periodic
    side's entries sit on its partner, which is periodic too)."""
    X0, X1, Y0, Y1 = rect
    tol = 1e-12
    out = []
    for x, y in xy:
        s = 0 if abs(y - Y0) <= tol else 2 if abs(y - Y1) <= tol else 1 if abs(x - X1) <= tol else 3
        out.append(bc[s])
    return np.array(out)


def _lib_case(t, p, q, sol, bc, coeff_fn=W.varcoeff):
    """Library-side inputs of one problem on the unit square."""
    xy = t.leaf_cheb_nodes(p)
    coeffs = np.stack([coeff_fn(xy[i, :, 0], xy[i, :, 1]) for i in range(len(xy))])
    I_ci, _, _ = leaf_geometry(p)
    g = np.stack([sol.g(xy[i, I_ci, 0], xy[i, I_ci, 1], coeffs[i][:, I_ci])
                  for i in range(len(xy))])
    b = t.bdry_gauss_nodes(q)
    f = W.side_data(sol, b, _kinds(b, bc), (0, 1, 0, 1))
    return coeffs, f, g, xy


def _oracle_g(ot, coeffs, p, sol):
    from oracle_cases import leaf_nodes
    xy = leaf_nodes(ot, p)
    I_ci, _, _ = leaf_geometry(p)
    return np.stack([sol.g(xy[i, I_ci, 0], xy[i, I_ci, 1], coeffs[i][:, I_ci])
                     for i in range(len(xy))])


@pytest.mark.parametrize("bc,nx,ny,p,q,nrhs", [
    ("NPNP", 4, 4, 12, 10, 1),
    ("PPPP", 4, 4, 12, 10, 2),
    ("NNNN", 4, 6, 10, 8, 1),
    ("DNDN", 4, 4, 16, 15, 3),
    ("PDPD", 4, 8, 12, 11, 1),
    ("NPNP", 8, 8, 16, 14, 20),
])
def test_side_conditions_match_oracle(bc, nx, ny, p, q, nrhs):
    import torch
    H = _lib()
    print(f"bc {bc} {nx}x{ny} p={p} q={q} nrhs={nrhs}", flush=True)
    t = H.Tree(0, 1, 0, 1, nx, ny).set_bc(bc)
    ot = oracle.Tree.uniform(0, 1, 0, 1, nx, ny)
    ot.set_bc(bc)
    sols = [W.FourierSolution(40 + r) for r in range(nrhs)]
    coeffs, _, _, _ = _lib_case(t, p, q, sols[0], bc)
    F, G = [], []
    for sol in sols:
        _, f, g, _ = _lib_case(t, p, q, sol, bc)
        F.append(f)
        G.append(g)
    s = H.Solver(t, to_dev(coeffs), p, q)
    u = s.solve(to_dev(np.stack(F)), to_dev(np.stack(G))).cpu().numpy()
    torch.cuda.synchronize()
    ops = oracle.build(ot, coeffs, p, q)
    nxy, bdry = ot.gauss(q)
    for r in (0, nrhs - 1):
        fo = W.side_data(sols[r], nxy[bdry], ot.bdry_kind(q), (0, 1, 0, 1))
        uo, _ = oracle.solve(ops, fo, _oracle_g(ot, coeffs, p, sols[r]))
        err = relerr(u[r], uo)
        print(f"  rhs {r}: rel err vs oracle {err:.2e}", flush=True)
        assert err <= 1e-11


def test_periodic_neumann_polynomials_full_size():
    """The Sec. 7.6 geometry (16 x 16 leaves, periodic in x, Neumann in y) at
    p = 16, q = 14: solutions constant in x and polynomial of degree q - 1 in
    y are reproduced exactly (to the FP64 floor)."""
    import torch
    H = _lib()
    n, p, q = 16, 16, 14
    t = H.Tree(0, 1, 0, 1, n, n).set_bc("NPNP")
    sol = W.PolyYSolution(3, q - 1)
    coeffs, f, g, xy = _lib_case(t, p, q, sol, "NPNP")
    s = H.Solver(t, to_dev(coeffs), p, q)
    u = s.solve(to_dev(f[None]), to_dev(g[None]))[0].cpu().numpy()
    torch.cuda.synchronize()
    err = relerr(u, sol.u(xy[..., 0], xy[..., 1]))
    print(f"polynomial in y, NPNP 16x16 p=16: {err:.2e}", flush=True)
    assert err <= 1e-10


def test_forest_with_side_conditions_and_refinement():
    """Three problems in one build: periodic/Neumann, Dirichlet refined at a
    point, all-Neumann refined at a point; each against the oracle."""
    import torch
    H = _lib()
    p, q = 12, 10
    bcs = ["NPNP", "DDDD", "NNNN"]
    t = H.Tree(0, 1, 0, 1, 4, 4, 3)
    ot = oracle.Tree.uniform(0, 1, 0, 1, 4, 4, 3)
    for k, bc in enumerate(bcs):
        t.set_bc(bc, k)
        ot.set_bc(bc, k)
    for tt in (t, ot):
        tt.refine_point(1, 0.3, 0.6, 3)
        tt.refine_point(2, 0.55, 0.45, 2)
    sol = W.FourierSolution(11)
    xy = t.leaf_cheb_nodes(p)
    coeffs = np.stack([W.varcoeff(xy[i, :, 0], xy[i, :, 1]) for i in range(len(xy))])
    nxy, bdry = ot.gauss(q)
    fo = W.side_data(sol, nxy[bdry], ot.bdry_kind(q), (0, 1, 0, 1))
    # the library's boundary list is the oracle's (same canonical order)
    assert np.abs(t.bdry_gauss_nodes(q) - nxy[bdry]).max() <= 1e-14
    go = _oracle_g(ot, coeffs, p, sol)
    s = H.Solver(t, to_dev(coeffs), p, q)
    u = s.solve(to_dev(fo[None]), to_dev(go[None]))[0].cpu().numpy()
    torch.cuda.synchronize()
    uo, _ = oracle.solve(oracle.build(ot, coeffs, p, q), fo, go)
    err = relerr(u, uo)
    print(f"forest NPNP / DDDD refined / NNNN refined: {err:.2e}", flush=True)
    assert err <= 1e-11


def test_economic_and_fp32_with_side_conditions():
    import torch
    H = _lib()
    n, p, q = 8, 16, 14
    t = H.Tree(0, 1, 0, 1, n, n).set_bc("NPNP")
    sols = [W.FourierSolution(60 + r) for r in range(4)]
    coeffs, _, _, _ = _lib_case(t, p, q, sols[0], "NPNP")
    F = np.stack([_lib_case(t, p, q, s_, "NPNP")[1] for s_ in sols])
    G = np.stack([_lib_case(t, p, q, s_, "NPNP")[2] for s_ in sols])
    cd, fd, gd = to_dev(coeffs), to_dev(F), to_dev(G)
    full = H.Solver(t, cd, p, q, keep_fp32=True)
    u = full.solve(fd, gd)
    u32 = full.solve(fd, gd, precision=H.HPS_PREC_FP32)
    econ = H.Solver(t, cd, p, q, economic=True)
    ue = econ.solve(fd, gd)
    torch.cuda.synchronize()
    u, u32, ue = u.cpu().numpy(), u32.cpu().numpy(), ue.cpu().numpy()
    print(f"economic vs stored {relerr(ue, u):.2e}, fp32 vs fp64 {relerr(u32, u):.2e}", flush=True)
    assert relerr(ue, u) <= 1e-13
    assert relerr(u32, u) <= 1e-4


def test_side_condition_refusals():
    H = _lib()
    p = 12
    t = H.Tree(0, 1, 0, 1, 4, 4).set_bc("NPNP")
    xy = t.leaf_cheb_nodes(p)
    coeffs = to_dev(np.stack([W.varcoeff(xy[i, :, 0], xy[i, :, 1]) for i in range(len(xy))]))
    with pytest.raises(H.HPSError, match="q <= p - 2"):
        H.Solver(t, coeffs, p, p - 1)
    with pytest.raises(H.HPSError, match="opposite pairs"):
        H.Tree(0, 1, 0, 1, 4, 4).set_bc("PDDD")
    # a Dirichlet side allows q = p - 1
    H.Solver(H.Tree(0, 1, 0, 1, 4, 4).set_bc("NPDP"), coeffs, p, p - 1)


@pytest.mark.parametrize("bc,nx,ny,p,q,nrhs", [
    ("NPNP", 8, 8, 16, 14, 4),
    ("PPPP", 4, 4, 12, 10, 2),
    ("NNNN", 4, 6, 12, 10, 1),
    ("DNDN", 4, 4, 16, 15, 16),
])
def test_mixed_precision_with_side_conditions(bc, nx, ny, p, q, nrhs):
    """FP32 sweeps refined against the FP64 residual, whose flux rows include
    the periodic seams (oriented by the merge that eliminates them) and the
    Neumann rows (data minus leaf flux): within 1e-10 of the oracle, while
    one FP32 sweep alone is not."""
    import torch
    H = _lib()
    print(f"mixed {bc} {nx}x{ny} p={p} q={q} nrhs={nrhs}", flush=True)
    t = H.Tree(0, 1, 0, 1, nx, ny).set_bc(bc)
    ot = oracle.Tree.uniform(0, 1, 0, 1, nx, ny)
    ot.set_bc(bc)
    sols = [W.FourierSolution(80 + r) for r in range(nrhs)]
    coeffs, _, _, _ = _lib_case(t, p, q, sols[0], bc)
    F = np.stack([_lib_case(t, p, q, s_, bc)[1] for s_ in sols])
    G = np.stack([_lib_case(t, p, q, s_, bc)[2] for s_ in sols])
    s = H.Solver(t, to_dev(coeffs), p, q, keep_fp32=True)
    stats = {}
    um = s.solve(to_dev(F), to_dev(G), precision=H.HPS_PREC_MIXED, stats=stats).cpu().numpy()
    u32 = s.solve(to_dev(F), to_dev(G), precision=H.HPS_PREC_FP32).cpu().numpy()
    torch.cuda.synchronize()
    ops = oracle.build(ot, coeffs, p, q)
    nxy, bdry = ot.gauss(q)
    for r in (0, nrhs - 1):
        fo = W.side_data(sols[r], nxy[bdry], ot.bdry_kind(q), (0, 1, 0, 1))
        uo, _ = oracle.solve(ops, fo, _oracle_g(ot, coeffs, p, sols[r]))
        em, e32 = relerr(um[r], uo), relerr(u32[r], uo)
        print(f"  rhs {r}: mixed {em:.2e} ({stats}), one FP32 sweep {e32:.2e}", flush=True)
        assert em <= 1e-10
        assert e32 > 1e-9


def test_crank_nicolson_mixed_precision():
    """The Sec. 7.6 workload (16 x 16 leaves, p = 16, q = 14) stepped with
    mixed-precision solves agrees with the FP64 stepping to 1e-10 after 8
    steps."""
    import torch
    H = _lib()
    k, steps = 0.05, 8
    t = H.Tree(0, 1, 0, 1, 16, 16).set_bc("NPNP")
    xy = t.leaf_cheb_nodes(16)
    X, Y = xy[..., 0], xy[..., 1]
    coeffs = np.stack([W.convdiff_coeffs(X[i], Y[i], k) for i in range(len(xy))])
    s = H.Solver(t, to_dev(coeffs), 16, 14, keep_fp32=True)
    f = to_dev(np.zeros((1, s.n_bdry)))
    u0 = to_dev(W.convdiff_initial(X, Y)[None])
    u64, umx = u0, u0
    for _ in range(steps):
        u64 = s.solve(f, s.apply_operator(u64, 2.0 / k))
        umx = s.solve(f, s.apply_operator(umx, 2.0 / k), precision=H.HPS_PREC_MIXED)
    torch.cuda.synchronize()
    err = relerr(umx.cpu().numpy(), u64.cpu().numpy())
    print(f"CN mixed vs FP64 after {steps} steps: {err:.2e}", flush=True)
    assert err <= 1e-10


@pytest.mark.parametrize("bc,nx,ny,p,q,refine", [
    ("NPNP", 4, 4, 12, 10, None), ("PPPP", 4, 4, 12, 10, None),
    ("NNNN", 4, 6, 10, 8, (0, 0.4, 0.55, 2)), ("DNDN", 4, 4, 16, 15, None),
    ("NPDP", 4, 4, 12, 11, None)])
def test_adjoint_with_side_conditions(bc, nx, ny, p, q, refine):
    """The transposed sweeps against the oracle's adjoint (fbar and gbar
    element by element, <= 1e-11 relative, on the first and last of 3
    right-hand sides) and against the forward solve: the dot-product
    identity <u(f, g), ubar> = <f, fbar> + <g, gbar> on seeded random
    vectors (f only on Dirichlet and Neumann entries, since periodic entries
    are not read); fbar is zero on periodic entries."""
    import torch
    H = _lib()
    print(f"adjoint {bc} {nx}x{ny} p={p} q={q} refine={refine}", flush=True)
    t = H.Tree(0, 1, 0, 1, nx, ny).set_bc(bc)
    if refine:
        t.refine_point(*refine)
    xy = t.leaf_cheb_nodes(p)
    coeffs = np.stack([W.varcoeff(xy[i, :, 0], xy[i, :, 1]) for i in range(len(xy))])
    s = H.Solver(t, to_dev(coeffs), p, q)
    rng = np.random.default_rng(17)
    nrhs, nl, mi = 3, t.n_leaves, (p - 2) ** 2
    b = t.bdry_gauss_nodes(q)
    per = _kinds(b, bc) == "P"
    f = rng.standard_normal((nrhs, s.n_bdry))
    f[:, per] = 0.0
    g = rng.standard_normal((nrhs, nl, mi))
    ub = rng.standard_normal((nrhs, nl, p * p))
    u = s.solve(to_dev(f), to_dev(g)).cpu().numpy()
    fb, gb = s.solve_adjoint(to_dev(ub))
    torch.cuda.synchronize()
    fb, gb = fb.cpu().numpy(), gb.cpu().numpy()
    for r in range(nrhs):
        lhs = float(np.sum(u[r] * ub[r]))
        rhs = float(np.sum(f[r] * fb[r]) + np.sum(g[r] * gb[r]))
        scale = float(np.abs(u[r] * ub[r]).sum())
        print(f"  rhs {r}: <u, ubar> {lhs:.12e}  <f, fbar> + <g, gbar> {rhs:.12e}", flush=True)
        assert abs(lhs - rhs) <= 1e-12 * scale
    assert np.all(fb[:, per] == 0.0)
    if (~per).any():
        assert np.abs(fb[:, ~per]).max() > 0.0
    ot = oracle.Tree.uniform(0, 1, 0, 1, nx, ny)
    ot.set_bc(bc)
    if refine:
        ot.refine_point(*refine)
    ops = oracle.build(ot, coeffs, p, q)
    for r in (0, nrhs - 1):
        fo, go = oracle.solve_adjoint(ops, ub[r])
        assert np.all(fo[per] == 0.0)
        # on a torus every entry is periodic and both fbar vectors are zero
        ef = relerr(fb[r][~per], fo[~per]) if (~per).any() else 0.0
        eg = relerr(gb[r], go)
        print(f"  rhs {r}: fbar vs oracle {ef:.2e}, gbar vs oracle {eg:.2e}", flush=True)
        assert ef <= 1e-11 and eg <= 1e-11


@pytest.mark.parametrize("bc,n", [("NPNP", 16), ("PPPP", 8), ("NNNN", 8), ("PDPD", 8)])
def test_translation_invariant_with_side_conditions(bc, n):
    """Constant coefficients (the Crank-Nicolson operator of Sec. 7.6): the
    build that stores one operator copy per distinct box solves exactly like
    the full build (FP64 and mixed), with far less operator memory."""
    import torch
    H = _lib()
    p, q, k = 16, 14, 0.01
    t = H.Tree(0, 1, 0, 1, n, n).set_bc(bc)
    xy = t.leaf_cheb_nodes(p)
    X, Y = xy[..., 0], xy[..., 1]
    cd = to_dev(np.stack([W.convdiff_coeffs(X[i], Y[i], k) for i in range(len(xy))]))
    full = H.Solver(t, cd, p, q, keep_fp32=True)
    shared = H.Solver(t, cd, p, q, keep_fp32=True, translation_invariant=True)
    rng = np.random.default_rng(23)
    f = to_dev(rng.standard_normal((4, full.n_bdry)))
    g = to_dev(rng.standard_normal((4, t.n_leaves, (p - 2) ** 2)))
    u1, u2 = full.solve(f, g), shared.solve(f, g)
    m1 = full.solve(f, g, precision=H.HPS_PREC_MIXED)
    m2 = shared.solve(f, g, precision=H.HPS_PREC_MIXED)
    torch.cuda.synchronize()
    d64 = relerr(u2.cpu().numpy(), u1.cpu().numpy())
    dmx = relerr(m2.cpu().numpy(), u1.cpu().numpy())
    wf = t.workspace_bytes(p, q)
    ws = t.workspace_bytes(p, q, translation_invariant=True)
    print(f"{bc} {n}x{n}: shared vs full {d64:.2e} (mixed {dmx:.2e}), operators {ws / wf:.3f} of full",
          flush=True)
    assert d64 <= 1e-13
    assert dmx <= 1e-10
    assert ws < 0.5 * wf


def test_refactor_with_side_conditions_matches_fresh_build():
    """hps_refactor (the build replayed as a HIP graph) on a periodic /
    Neumann tree, three times with alternating coefficients, each against a
    fresh build of the same coefficients (bitwise)."""
    import torch
    H = _lib()
    p, q = 12, 10
    t = H.Tree(0, 1, 0, 1, 8, 8).set_bc("NPNP")
    xy = t.leaf_cheb_nodes(p)
    X, Y = xy[..., 0], xy[..., 1]
    cs = [to_dev(np.stack([W.convdiff_coeffs(X[i], Y[i], k) for i in range(len(xy))]))
          for k in (0.01, 0.002)]
    rng = np.random.default_rng(29)
    s = H.Solver(t, cs[0], p, q)
    f = to_dev(rng.standard_normal((2, s.n_bdry)))
    g = to_dev(rng.standard_normal((2, t.n_leaves, (p - 2) ** 2)))
    for rep in range(3):
        c = cs[(rep + 1) % 2]
        s.refactor(c)
        u = s.solve(f, g)
        ref = H.Solver(t, c, p, q).solve(f, g)
        torch.cuda.synchronize()
        d = float((u - ref).abs().max())
        print(f"  refactor {rep}: max diff vs fresh build {d:.1e}", flush=True)
        assert d == 0.0


def test_autograd_gradient_with_side_conditions():
    """Loss sum(u^2) on a periodic / Neumann tree: the autograd gradient with
    respect to c (adjoint sweeps) against central differences along three
    seeded directions (h = 1e-4; the loss is smooth in c, so the O(h^2)
    truncation is far below the 1e-6 relative bound)."""
    import torch
    from paper_1612_02736_amd.autograd import hps_solve
    H = _lib()
    p, q = 12, 10
    t = H.Tree(0, 1, 0, 1, 4, 4).set_bc("NPNP")
    xy = t.leaf_cheb_nodes(p)
    coeffs = np.stack([W.varcoeff(xy[i, :, 0], xy[i, :, 1]) for i in range(len(xy))])
    cd = to_dev(coeffs)
    s = H.Solver(t, cd, p, q)
    rng = np.random.default_rng(31)
    f = to_dev(rng.standard_normal((1, s.n_bdry)))
    g = to_dev(rng.standard_normal((1, t.n_leaves, (p - 2) ** 2)))
    c = to_dev(coeffs[:, 5]).requires_grad_(True)
    u = hps_solve(s, cd, c, g, f)
    (u ** 2).sum().backward()
    grad = c.grad.cpu().numpy()
    for k in range(3):
        d = np.random.default_rng(700 + k).standard_normal(grad.shape)
        h = 1e-4
        with torch.no_grad():
            lp = float((hps_solve(s, cd, c.detach() + h * to_dev(d), g, f) ** 2).sum())
            lm = float((hps_solve(s, cd, c.detach() - h * to_dev(d), g, f) ** 2).sum())
        fd, an = (lp - lm) / (2 * h), float(np.sum(grad * d))
        print(f"  direction {k}: fd {fd:.10e} adjoint {an:.10e}", flush=True)
        assert abs(fd - an) <= 1e-6 * abs(an)


def test_apply_operator_matches_oracle():
    """sigma u - A u at interior nodes on random leaf values, 3 right-hand
    sides, variable coefficients on a refined tree."""
    import torch
    H = _lib()
    p, sigma = 12, 3.75
    t = H.Tree(0, 1, 0, 1, 3, 4).refine_point(0, 0.4, 0.5, 2)
    ot = oracle.Tree.uniform(0, 1, 0, 1, 3, 4)
    ot.refine_point(0, 0.4, 0.5, 2)
    xy = t.leaf_cheb_nodes(p)
    coeffs = np.stack([W.varcoeff(xy[i, :, 0], xy[i, :, 1]) for i in range(len(xy))])
    u = np.random.default_rng(5).standard_normal((3, len(xy), p * p))
    s = H.Solver(t, to_dev(coeffs), p)
    out = s.apply_operator(to_dev(u), sigma).cpu().numpy()
    torch.cuda.synchronize()
    for r in range(3):
        want = oracle.operator_apply(ot, coeffs, p, u[r], sigma)
        err = relerr(out[r], want)
        print(f"  rhs {r}: {err:.2e}", flush=True)
        assert err <= 1e-12


def _cn_setup(H, n, p, q, k):
    t = H.Tree(0, 1, 0, 1, n, n).set_bc("NPNP")
    xy = t.leaf_cheb_nodes(p)
    X, Y = xy[..., 0], xy[..., 1]
    coeffs = np.stack([W.convdiff_coeffs(X[i], Y[i], k) for i in range(len(xy))])
    s = H.Solver(t, to_dev(coeffs), p, q)
    return t, s, X, Y


def _cn_run(H, s, u0, k, steps):
    f = to_dev(np.zeros((u0.shape[0], s.n_bdry)))
    u = u0
    for _ in range(steps):
        u = s.solve(f, s.apply_operator(u, 2.0 / k))
    return u


def test_crank_nicolson_eigenmode_full_size_and_oracle():
    """Sec. 7.6 workload (16 x 16 leaves, eps = 1/200, periodic in x, zero
    Neumann data in y) at p = 16, q = 14: 8 steps of k = 0.05 on the mode
    e^{2 pi i x} cos(pi y) give Re(R^8 e^{2 pi i x}) cos(pi y),
    R = (1 - k lam/2)/(1 + k lam/2), lam = 5 eps pi^2 + 2 pi i; and two steps
    on 4 x 4 leaves match the oracle's Crank-Nicolson loop."""
    import torch
    H = _lib()
    k, steps = 0.05, 8
    t, s, X, Y = _cn_setup(H, 16, 16, 14, k)
    u0 = np.cos(2 * np.pi * X) * np.cos(np.pi * Y)
    u = _cn_run(H, s, to_dev(u0[None]), k, steps)[0].cpu().numpy()
    torch.cuda.synchronize()
    lam = 5 * W.CD_EPS * np.pi ** 2 + 2j * np.pi
    R = (1 - k * lam / 2) / (1 + k * lam / 2)
    closed = np.real(R ** steps * np.exp(2j * np.pi * X)) * np.cos(np.pi * Y)
    err = relerr(u, closed)
    print(f"CN 16x16 p=16, 8 steps: vs closed form {err:.2e}", flush=True)
    assert err <= 1e-10
    # oracle parity of two steps from the Gaussian initial value
    n, p, q = 4, 12, 10
    t, s, X, Y = _cn_setup(H, n, p, q, k)
    u0 = W.convdiff_initial(X, Y)
    u = _cn_run(H, s, to_dev(u0[None]), k, 2)[0].cpu().numpy()
    ot = oracle.Tree.uniform(0, 1, 0, 1, n, n)
    ot.set_bc("NPNP")
    uo = oracle.crank_nicolson(ot, np.stack([W.convdiff_coeffs(X[i], Y[i], k)
                                             for i in range(len(X))]), p, q, k, u0, 2)
    err = relerr(u, uo)
    print(f"CN 4x4 p=12, 2 steps: vs oracle {err:.2e}", flush=True)
    assert err <= 1e-11


def test_crank_nicolson_second_order_in_time():
    """A smooth bump that fits the side conditions (periodic in x, even about
    y = 0 and y = 1) advanced to t = 0.1 with k = 0.02, 0.01, 0.005, 0.0025
    (one build per k): successive differences shrink by about 4 (second
    order).  The Gaussian of Sec. 7.6 itself is neither periodic nor of zero
    normal derivative on the boundary, and Crank-Nicolson, which does not
    damp the stiff part of that mismatch, converges at about first order on
    it (differences shrink by about 2)."""
    import torch
    H = _lib()
    n, p, q, T = 16, 16, 14, 0.1
    outs = []
    for k in (0.02, 0.01, 0.005, 0.0025):
        t, s, X, Y = _cn_setup(H, n, p, q, k)
        u0 = to_dev(W.convdiff_smooth_initial(X, Y)[None])
        outs.append(_cn_run(H, s, u0, k, int(round(T / k)))[0].cpu().numpy())
        torch.cuda.synchronize()
    d = [np.abs(outs[i] - outs[i + 1]).max() for i in range(3)]
    rates = [d[i] / d[i + 1] for i in range(2)]
    print(f"CN differences {d}, ratios {rates}", flush=True)
    assert all(3.5 <= r <= 4.5 for r in rates), rates
