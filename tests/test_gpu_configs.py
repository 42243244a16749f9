"""GPU checks at the full sizes of the heat, refined-forest and gradient
workloads (the factor + solve workload has its own full-size tests in
test_gpu_parity.py).  Each compares with the oracle where the oracle can run
in seconds (sampled problems of a forest), and otherwise with properties
that hold at any size (exact reproduction of polynomial solutions, FP32
refinement against the FP64 path, finite differences of the gradient).
"""

import numpy as np
import pytest

import oracle
import workloads as W

from gpu_cases import lib_inputs, relerr, to_dev

pytestmark = pytest.mark.gpu


def _lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1612_02736_amd as H
    H.lib()
    return H


def test_heat_128x128_p12_polynomials_fp64_and_mixed():
    """(I - dt Lap) u = g on 128 x 128 leaves, p = 12: a batch of 32
    right-hand sides from polynomial solutions of degree q - 1 = 10, which
    the discretization reproduces exactly.  FP64 solve and FP32 matrix-core
    sweeps refined in FP64 both reproduce them (the operator is close to the
    identity, so the FP64 floor is ~1e-13)."""
    import torch
    H = _lib()
    n, p, q, nrhs = 128, 12, 11, 32
    print(f"heat {n}x{n} p={p} nrhs={nrhs}", flush=True)
    t = H.Tree(0, 1, 0, 1, n, n)
    xy = t.leaf_cheb_nodes(p)
    coeffs = np.stack([W.heat_coeffs(xy[i, :, 0], xy[i, :, 1]) for i in range(len(xy))])
    # 4 polynomial solutions, combined with seeded weights into 32 (the
    # problem is linear, so the combinations are exact solutions too)
    basis = [W.PolySolution(200 + j, q - 1) for j in range(4)]
    bf, bg, bu = [], [], []
    for sol in basis:
        _, f, g, _ = lib_inputs(t, p, q, W.heat_coeffs, sol)
        bf.append(f)
        bg.append(g)
        bu.append(sol.u(xy[..., 0], xy[..., 1]))
    wts = np.random.default_rng(7).standard_normal((nrhs, 4))
    F = np.einsum("rj,jk->rk", wts, np.stack(bf))
    G = np.einsum("rj,j...->r...", wts, np.stack(bg))
    ex = np.einsum("rj,j...->r...", wts, np.stack(bu))
    s = H.Solver(t, to_dev(coeffs), p, q, keep_fp32=True)
    fd, gd = to_dev(F), to_dev(G)
    u64 = s.solve(fd, gd).cpu().numpy()
    stats = {}
    umx = s.solve(fd, gd, precision=H.HPS_PREC_MIXED, stats=stats).cpu().numpy()
    torch.cuda.synchronize()
    worst64 = max(relerr(u64[r], ex[r]) for r in range(nrhs))
    worstmx = max(relerr(umx[r], ex[r]) for r in range(nrhs))
    print(f"  fp64 {worst64:.2e}  mixed {worstmx:.2e}  refinement {stats}", flush=True)
    assert worst64 <= 1e-11
    assert worstmx <= 1e-10


def test_refined_forest_64_problems_full_size():
    """64 independent problems in one build, each refined 8 levels toward a
    seeded point (coefficients of the variable-coefficient family with seeded
    phases, Gaussian load of width 1e-3, zero boundary data), p = 16, q = 14.
    Two of the problems are recomputed by the oracle on their own trees."""
    H = _lib()
    nprob, p, q = 64, 16, 14
    print(f"refined forest {nprob} problems p={p} q={q}", flush=True)
    draws = [W.refined_problem(100 + k) for k in range(nprob)]
    t = H.Tree(0, 1, 0, 1, 4, 4, nprob)
    ot = oracle.Tree.uniform(0, 1, 0, 1, 4, 4, nprob)
    for k, (_, xh) in enumerate(draws):
        t.refine_point(k, xh[0], xh[1], 8)
        ot.refine_point(k, xh[0], xh[1], 8)
    prob = np.array([b.problem for b in ot.leaves])
    assert len(prob) == t.n_leaves
    xy = t.leaf_cheb_nodes(p)
    coeffs = np.stack([W.varcoeff(xy[i, :, 0], xy[i, :, 1], draws[prob[i]][0])
                       for i in range(len(xy))])
    pi = p - 2
    inner = np.array([(iy + 1) * p + ix + 1 for iy in range(pi) for ix in range(pi)])
    g = np.stack([W.gaussian_load(xy[i, inner, 0], xy[i, inner, 1], draws[prob[i]][1])
                  for i in range(len(xy))])
    f = np.zeros(t.counts(q)[1])
    s = H.Solver(t, to_dev(coeffs), p, q)
    u = s.solve(to_dev(f[None]), to_dev(g[None]))[0].cpu().numpy()

    class Load:
        def __init__(self, xh):
            self.xh = xh

        def u(self, x, y):
            return np.zeros_like(x)

        def g(self, x, y, c):
            return W.gaussian_load(x, y, self.xh)

    for k in (0, 37):
        ph, xh = draws[k]
        tk = oracle.Tree.uniform(0, 1, 0, 1, 4, 4, 1)
        tk.refine_point(0, xh[0], xh[1], 8)
        from oracle_cases import make_inputs
        oc, of, og, _ = make_inputs(tk, p, q, lambda x, y: W.varcoeff(x, y, ph), Load(xh))
        uo, _ = oracle.solve(oracle.build(tk, oc, p, q), of, og)
        mine = u[prob == k]
        print(f"  problem {k}: {mine.shape[0]} leaves, rel err {relerr(mine, uo):.2e}",
              flush=True)
        assert relerr(mine, uo) <= 1e-11


def test_gradient_32_problems_32x32_full_size():
    """Loss sum (u - u_obs)^2 over a forest of 32 problems of 32 x 32 leaves,
    p = 16, coefficients of the variable-coefficient family with seeded
    phases per problem, u_obs from a perturbed zeroth-order coefficient.
    Gradients with respect to c, g and f from the transposed sweeps are
    checked against central differences along seeded directions with N(0, 1)
    entries (a perturbation of h per node): 20 directions of c at h = 1e-6,
    to the FP64 noise bound of the difference (each loss carries rounding of
    about 2e-13 max|u| sum|u - u_obs|); 3 directions of c at h = 1e-3, to
    1e-5 relative (the O(h^2) truncation); 3 directions each of g and f at
    h = 1e-3 (the loss is quadratic in (g, f), so the difference is exact up
    to rounding)."""
    import torch
    from paper_1612_02736_amd.autograd import hps_solve
    H = _lib()
    n, p, q, nprob = 32, 16, 15, 32
    print(f"gradient {nprob} problems {n}x{n} p={p}", flush=True)
    t = H.Tree(0, 1, 0, 1, n, n, nprob)
    nl = t.n_leaves
    per = nl // nprob
    xy = t.leaf_cheb_nodes(p)
    phases = [W.problem_phases(300 + k) for k in range(nprob)]
    coeffs = np.stack([W.varcoeff(xy[i, :, 0], xy[i, :, 1], phases[i // per])
                       for i in range(nl)])
    _, f, g, _ = lib_inputs(t, p, q, W.varcoeff, W.FourierSolution(2))
    cd = to_dev(coeffs)
    s = H.Solver(t, cd, p, q)
    pert = W.Perturbation(3)
    c_obs = coeffs[:, 5] * (1 + 0.1 * pert(xy[..., 0], xy[..., 1]))
    fd_, gd_ = to_dev(f[None]), to_dev(g[None])
    u_obs = hps_solve(s, cd, to_dev(c_obs), gd_, fd_).detach()
    c = to_dev(coeffs[:, 5]).requires_grad_(True)
    gv = gd_.clone().requires_grad_(True)
    fv = fd_.clone().requires_grad_(True)
    u = hps_solve(s, cd, c, gv, fv)
    L = ((u - u_obs) ** 2).sum()
    L.backward()
    grads = {"c": c.grad.cpu().numpy(), "g": gv.grad.cpu().numpy(),
             "f": fv.grad.cpu().numpy()}
    umax = float(u.detach().abs().max())
    dsum = float((u.detach() - u_obs).abs().sum())
    base = {"c": c.detach(), "g": gv.detach(), "f": fv.detach()}

    def loss(which, delta):
        args = dict(base)
        args[which] = base[which] + delta
        with torch.no_grad():
            return ((hps_solve(s, cd, args["c"], args["g"], args["f"]) - u_obs) ** 2).sum().item()

    for which, ndir, hh in (("c", 20, 1e-6), ("c", 3, 1e-3), ("g", 3, 1e-3), ("f", 3, 1e-3)):
        grad = grads[which]
        err_sum = an_sum = 0.0
        for k in range(ndir):
            d = np.random.default_rng(500 + k).standard_normal(grad.shape)
            an = float(np.sum(grad * d))
            dd = to_dev(d)
            fdv = (loss(which, hh * dd) - loss(which, -hh * dd)) / (2 * hh)
            noise = 2.0 * (2e-13 * umax * dsum) / (2 * hh)
            tol = max(1e-5 * abs(an), noise)
            print(f"  {which} h={hh:g} direction {k}: fd {fdv:.10e} adjoint {an:.10e} "
                  f"(bound {tol:.1e})", flush=True)
            assert abs(fdv - an) <= tol, (which, k, fdv, an)
            err_sum += abs(fdv - an)
            an_sum += abs(an)
        # the check is not vacuous: over all directions the differences agree
        # with the adjoint to a few percent even at h = 1e-6
        assert err_sum <= 0.05 * an_sum, (which, hh, err_sum, an_sum)
