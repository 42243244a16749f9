"""GPU checks of the solve-stage extensions: mixed precision (FP32 sweeps +
FP64 residual iterative refinement) against the FP64 oracle at <= 1e-10, and
the adjoint (transposed sweeps) against the oracle's adjoint, the dot-product
identity and central finite differences."""

import numpy as np
import pytest

import oracle
import workloads as W

from gpu_cases import lib_inputs, oracle_solution, relerr, to_dev
from oracle_cases import make_inputs

pytestmark = pytest.mark.gpu


def _H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1612_02736_amd as H
    H.lib()
    return H


@pytest.mark.parametrize("n,p,coeff", [(4, 16, "var"), (16, 16, "var"), (8, 12, "heat")])
def test_mixed_precision_refines_to_fp64(n, p, coeff):
    H = _H()
    q = p - 1
    fn = W.varcoeff if coeff == "var" else W.heat_coeffs
    sol = W.FourierSolution(6)
    print(f"mixed n={n} p={p} {coeff}", flush=True)
    t = H.Tree(0, 1, 0, 1, n, n)
    coeffs, f, g, _ = lib_inputs(t, p, q, fn, sol)
    s = H.Solver(t, to_dev(coeffs), p, q, keep_fp32=True)
    stats = {}
    u = s.solve(to_dev(f[None]), to_dev(g[None]), precision=H.HPS_PREC_MIXED,
                stats=stats)[0].cpu().numpy()
    u32 = s.solve(to_dev(f[None]), to_dev(g[None]), precision=H.HPS_PREC_FP32)[0].cpu().numpy()
    uo, _ = oracle_solution(oracle.Tree.uniform(0, 1, 0, 1, n, n), p, q, fn, sol)
    e_mixed, e_32 = relerr(u, uo), relerr(u32, uo)
    print(f"  fp32 {e_32:.2e}  mixed {e_mixed:.2e}  iters {stats}", flush=True)
    assert e_32 > 1e-9            # the FP32 sweeps alone are not FP64-accurate
    assert e_mixed <= 1e-10
    assert 1 <= stats["iters"] <= 6


@pytest.mark.parametrize("nrhs", [5, 20])
def test_mixed_precision_many_rhs(nrhs):
    """5 right-hand sides run the FP32 sweeps on the vector path, 20 on the
    FP32 matrix cores; every column refines to the oracle's FP64 answer."""
    H = _H()
    p, q, n = 12, 11, 8
    t = H.Tree(0, 1, 0, 1, n, n)
    sols = [W.FourierSolution(30 + r) for r in range(nrhs)]
    fs, gs = [], []
    for sol in sols:
        coeffs, f, g, _ = lib_inputs(t, p, q, W.varcoeff, sol)
        fs.append(f)
        gs.append(g)
    s = H.Solver(t, to_dev(coeffs), p, q, keep_fp32=True)
    u = s.solve(to_dev(np.stack(fs)), to_dev(np.stack(gs)),
                precision=H.HPS_PREC_MIXED).cpu().numpy()
    u32 = s.solve(to_dev(np.stack(fs)), to_dev(np.stack(gs)),
                  precision=H.HPS_PREC_FP32).cpu().numpy()
    ot = oracle.Tree.uniform(0, 1, 0, 1, n, n)
    for r, sol in enumerate(sols):
        if nrhs > 16 and 0 < r < nrhs - 1:
            continue
        uo, _ = oracle_solution(ot, p, q, W.varcoeff, sol)
        assert relerr(u[r], uo) <= 1e-10, r
        assert 1e-13 < relerr(u32[r], uo) < 1e-4, r     # one FP32 sweep: FP32-accurate only
    if nrhs > 16:
        u64 = s.solve(to_dev(np.stack(fs)), to_dev(np.stack(gs))).cpu().numpy()
        for r in range(nrhs):
            assert relerr(u[r], u64[r]) <= 1e-10, r


def _adjoint_pair(n, p, refine=None, nprob=1):
    H = _H()
    q = p - 1
    t = H.Tree(0, 1, 0, 1, n, n, nprob)
    ot = oracle.Tree.uniform(0, 1, 0, 1, n, n, nprob)
    if refine:
        t.refine_point(*refine)
        ot.refine_point(*refine)
    sol = W.FourierSolution(7)
    coeffs, f, g, _ = lib_inputs(t, p, q, W.varcoeff, sol)
    s = H.Solver(t, to_dev(coeffs), p, q)
    oc, _, _, _ = make_inputs(ot, p, q, W.varcoeff, sol)
    ops = oracle.build(ot, oc, p, q)
    return H, s, ops, t, p, q, f, g


@pytest.mark.parametrize("n,p,refine,nprob", [(4, 12, None, 1), (2, 8, (0, 0.4, 0.55, 2), 1),
                                              (2, 8, None, 3), (16, 16, None, 1)])
def test_adjoint_matches_oracle(n, p, refine, nprob):
    H, s, ops, t, p, q, f, g = _adjoint_pair(n, p, refine, nprob)
    rng = np.random.default_rng(5)
    nl = t.n_leaves
    ub = rng.standard_normal((2, nl, p * p))
    fb, gb = s.solve_adjoint(to_dev(ub))
    fb, gb = fb.cpu().numpy(), gb.cpu().numpy()
    for r in range(2):
        fo, go = oracle.solve_adjoint(ops, ub[r])
        assert relerr(fb[r], fo) <= 1e-11, ("fbar", r)
        assert relerr(gb[r], go) <= 1e-11, ("gbar", r)


@pytest.mark.parametrize("nrhs", [3, 18])
def test_adjoint_dot_product_identity(nrhs):
    """<u, y> = <f, fbar> + <g, gbar> for u = solve(f, g) and (fbar, gbar) =
    adjoint(y); 18 right-hand sides take the MFMA apply path both ways."""
    H, s, ops, t, p, q, f, g = _adjoint_pair(4, 12)
    rng = np.random.default_rng(8)
    nl, nb = t.n_leaves, t.counts(q)[1]
    f1 = rng.standard_normal((nrhs, nb))
    g1 = rng.standard_normal((nrhs, nl, (p - 2) ** 2))
    y = rng.standard_normal((nrhs, nl, p * p))
    u = s.solve(to_dev(f1), to_dev(g1)).cpu().numpy()
    fb, gb = s.solve_adjoint(to_dev(y))
    fb, gb = fb.cpu().numpy(), gb.cpu().numpy()
    for r in range(nrhs):
        lhs = np.sum(u[r] * y[r])
        rhs = np.sum(f1[r] * fb[r]) + np.sum(g1[r] * gb[r])
        assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(u[r] * y[r])), r
    if nrhs > 16:
        for r in (0, nrhs - 1):
            fo, go = oracle.solve_adjoint(ops, y[r])
            assert relerr(fb[r], fo) <= 1e-11, ("fbar", r)
            assert relerr(gb[r], go) <= 1e-11, ("gbar", r)


def test_coefficient_gradient_finite_differences():
    """L = sum (u - u_obs)^2 over problems and nodes; dL/dc by the autograd
    wrapper against central differences on seeded unit directions.

    Step h = 1e-3: the FP64 solve's rounding contributes ~1e-9 relative and
    truncation (h |d| / |c|)^2 ~ 1e-10, so the bound is 1e-6 relative.
    Step h = 1e-6 (the workload's step): each u carries rounding of about
    1e-13 max|u|, so each L carries noise up to 2e-13 max|u| sum|u - u_obs|
    and the central difference up to twice that over 2h; the bound is that
    noise estimate (measured disagreement 1e-5 .. 2e-4 relative)."""
    import torch
    from paper_1612_02736_amd.autograd import hps_solve
    H = _H()
    n, p, q, nprob = 4, 12, 11, 2
    t = H.Tree(0, 1, 0, 1, n, n, nprob)
    xy = t.leaf_cheb_nodes(p)
    coeffs = np.stack([W.varcoeff(xy[i, :, 0], xy[i, :, 1]) for i in range(len(xy))])
    _, f, g, _ = lib_inputs(t, p, q, W.varcoeff, W.FourierSolution(2))
    cd = to_dev(coeffs)
    s = H.Solver(t, cd, p, q)
    pert = W.Perturbation(3)
    c_obs = coeffs[:, 5] * (1 + 0.1 * pert(xy[..., 0], xy[..., 1]))
    fd_, gd_ = to_dev(f[None]), to_dev(g[None])
    u_obs = hps_solve(s, cd, to_dev(c_obs), gd_, fd_).detach()
    c = to_dev(coeffs[:, 5]).requires_grad_(True)
    u = hps_solve(s, cd, c, gd_, fd_)
    L = ((u - u_obs) ** 2).sum()
    L.backward()
    grad = c.grad.cpu().numpy()
    for k in range(4):
        d = np.random.default_rng(100 + k).standard_normal(grad.shape)
        d /= np.linalg.norm(d)
        an = float(np.sum(grad * d))
        umax = float(u.detach().abs().max())
        dsum = float((u.detach() - u_obs).abs().sum())
        for hh in (1e-3, 1e-6):
            with torch.no_grad():
                lp = ((hps_solve(s, cd, c + hh * to_dev(d), gd_, fd_) - u_obs) ** 2).sum().item()
                lm = ((hps_solve(s, cd, c - hh * to_dev(d), gd_, fd_) - u_obs) ** 2).sum().item()
            fdv = (lp - lm) / (2 * hh)
            noise = 2.0 * (2e-13 * umax * dsum) / (2 * hh)
            tol = 1e-6 * abs(an) if hh == 1e-3 else max(1e-6 * abs(an), noise)
            print(f"direction {k} h={hh:g}: fd {fdv:.10e} adjoint {an:.10e} "
                  f"(bound {tol:.1e})", flush=True)
            assert abs(fdv - an) <= tol, (k, hh, fdv, an)


def test_coefficient_gradient_matches_oracle():
    H, s, ops, t, p, q, f, g = _adjoint_pair(4, 12)
    u = s.solve(to_dev(f[None]), to_dev(g[None]))
    rng = np.random.default_rng(9)
    ub = rng.standard_normal(u.shape)
    _, gb = s.solve_adjoint(to_dev(ub))
    cb = s.coeff_grad_c(u, gb).cpu().numpy()[0]
    uo = oracle.solve(ops, *make_inputs(oracle.Tree.uniform(0, 1, 0, 1, 4, 4), p, q,
                                        W.varcoeff, W.FourierSolution(7))[1:3])[0]
    _, go = oracle.solve_adjoint(ops, ub[0])
    co = oracle.coeff_gradient(ops, uo, go)[:, 5]
    assert relerr(cb, co) <= 1e-10


def test_mixed_precision_error_codes():
    """A mixed solve fed a NaN in its boundary data returns HPS_ENONFINITE;
    one that stops above its tolerance (one refinement step against an
    unreachable ir_tol) returns HPS_ENOCONV."""
    H = _H()
    p, q, n = 12, 11, 4
    print("mixed precision error codes", flush=True)
    t = H.Tree(0, 1, 0, 1, n, n)
    coeffs, f, g, _ = lib_inputs(t, p, q, W.varcoeff, W.FourierSolution(6))
    s = H.Solver(t, to_dev(coeffs), p, q, keep_fp32=True)
    fbad = f.copy()
    fbad[3] = np.nan
    with pytest.raises(H.HPSError) as e:
        s.solve(to_dev(fbad[None]), to_dev(g[None]), precision=H.HPS_PREC_MIXED)
    assert e.value.code == -4
    gbad = g.copy()
    gbad[1, 7] = np.inf
    with pytest.raises(H.HPSError) as e:
        s.solve(to_dev(f[None]), to_dev(gbad[None]), precision=H.HPS_PREC_MIXED)
    assert e.value.code == -4
    with pytest.raises(H.HPSError) as e:
        s.solve(to_dev(f[None]), to_dev(g[None]), precision=H.HPS_PREC_MIXED, ir_tol=1e-300,
                max_iter=1)
    assert e.value.code == -5
    # and the same handle still solves normally afterwards
    u = s.solve(to_dev(f[None]), to_dev(g[None]), precision=H.HPS_PREC_MIXED)
    assert np.isfinite(u.cpu().numpy()).all()


def test_autograd_two_forwards_before_backward():
    """Two forwards on one solver with different coefficient fields, then one
    backward through both: the gradients equal those of two separate
    forward/backward passes (the first term's backward must not use the
    second forward's operators)."""
    import torch
    from paper_1612_02736_amd.autograd import hps_solve
    H = _H()
    p, q, n = 12, 11, 4
    print("autograd two forwards", flush=True)
    t = H.Tree(0, 1, 0, 1, n, n)
    coeffs, f, g, _ = lib_inputs(t, p, q, W.varcoeff, W.FourierSolution(8))
    cd = to_dev(coeffs)
    s = H.Solver(t, cd, p, q)
    rng = np.random.default_rng(21)
    c1 = to_dev(coeffs[:, 5, :] * (1 + 0.2 * rng.standard_normal(coeffs[:, 5, :].shape)))
    c2 = to_dev(coeffs[:, 5, :] * (1 + 0.2 * rng.standard_normal(coeffs[:, 5, :].shape)))
    gd, fd = to_dev(g[None]), to_dev(f[None])

    def grads(terms):
        cs = [c.clone().requires_grad_(True) for c in (c1, c2)]
        loss = 0.0
        for k in terms:
            loss = loss + (hps_solve(s, cd, cs[k], gd, fd) ** 2).sum()
        loss.backward()
        return [None if c.grad is None else c.grad.cpu().numpy() for c in cs]

    both = grads([0, 1])
    one = grads([0])[0]
    two = grads([1])[1]
    assert relerr(both[0], one) <= 1e-12
    assert relerr(both[1], two) <= 1e-12
    assert relerr(one, two) > 1e-3          # the two fields give different gradients


@pytest.mark.parametrize("bc,n,p,q", [("DDDD", 4, 12, 11), ("NPNP", 4, 12, 10)])
def test_operator_residual_rows_match_oracle_residual(bc, n, p, q):
    """The PDE rows of the global system's residual, b - K x, for arbitrary
    (non-solution) leaf values: g - A u_c on every leaf's interior nodes.  The
    library evaluates -A u_c with hps_apply_operator (sigma = 0), the kernel
    the mixed-precision refinement uses for these rows; the oracle takes them
    from its assembled system (oracle.residual)."""
    H = _H()
    print(f"residual rows {bc} {n}x{n} p={p} q={q}", flush=True)
    t = H.Tree(0, 1, 0, 1, n, n).set_bc(bc)
    ot = oracle.Tree.uniform(0, 1, 0, 1, n, n)
    ot.set_bc(bc)
    xy = t.leaf_cheb_nodes(p)
    coeffs = np.stack([W.varcoeff(xy[i, :, 0], xy[i, :, 1]) for i in range(len(xy))])
    rng = np.random.default_rng(41)
    uc = rng.standard_normal((t.n_leaves, p * p))
    g = rng.standard_normal((t.n_leaves, (p - 2) ** 2))
    s = H.Solver(t, to_dev(coeffs), p, q)
    neg_au = s.apply_operator(to_dev(uc[None]), 0.0)[0].cpu().numpy()
    nxy, bdry = ot.gauss(q)
    u = rng.standard_normal(len(nxy))
    f = rng.standard_normal(len(bdry))
    r, lay = oracle.residual(ot, coeffs, p, q, uc, u, f, g)
    want = r[lay["e1_rows"]]
    err = relerr(g + neg_au, want)
    print(f"  g - A u vs oracle residual rows: {err:.2e}", flush=True)
    assert err <= 1e-12
