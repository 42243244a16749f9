#!/usr/bin/env python
"""Benchmark: HPS factor + solve on one MI355X.

Workload: the full variable-coefficient operator
  c11 = 1 + .5 sin(2 pi x) cos(2 pi y), c22 = 1 + .3 cos(2 pi x),
  c12 = .1 sin(pi x) sin(pi y), c1 = c2 = .5 sin(2 pi y), c = 1 + x^2
on [0,1]^2 with 64 x 64 leaves, p = 16, q = 15 (N = p^2 n^2 = 1,048,576
collocation nodes), body loads and boundary data of 32 seeded manufactured
solutions (sums of 8 Fourier modes, seeds 2..33).  Synthetic data, inputs
resident in device memory before timing.

One step = Algorithm 1 (hps_refactor on the resident coefficients) followed by
Algorithm 2 for the batch of 32 right-hand sides in FP64.  value = right-hand
sides solved per second of whole steps (factor included).  Separately
reported: factor time, solve-only throughput at nrhs 32 and 1, achieved
TFLOP/s, relative error against stored oracle values, the roofline of the
dominant kernel (from HIP events around its launches in eager, profiled
steps of the same work that follow the timed steps: the timed steps replay
the factorization as a HIP graph, which admits no per-kernel events),
the CPU oracle (the full problem on one host thread, and a sample with the
BLAS thread pool at its default), and side workloads reported apart from
the headline: mixed-precision and adjoint solves, the storage-economic
build, the translation-invariant heat build, Crank-Nicolson steps of the
periodic / Neumann convection-diffusion problem, build / solve time and
operator memory against N, and the throughput of three independent steps in
flight on three streams (a serving configuration; the headline is one step
at a time).
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_LEAF_SIDE, P, Q, NRHS = 64, 16, 15, 32
# HBM bytes per launch of each kernel class from rocprofv3 FETCH_SIZE /
# WRITE_SIZE runs (bench.py --traffic-probe), scaled by what the counters read
# for a 1 GiB copy, keyed by the kernel class, with the SHA-256 prefix of the
# source files of that kernel when the counters were taken: a figure is
# reported only while those sources are unchanged.
KERNEL_SOURCES = {"gemm": ["kernels_gemm.hip", "kernel_util.hpp"],
                  "gj_leaf": ["kernels_gj_leaf.hip", "kernels_gjb_leaf.hip", "gj_core.hpp",
                              "kernel_util.hpp"],
                  "gj_panel": ["kernels_gj_blocked.hip", "gj_core.hpp", "kernel_util.hpp"],
                  "apply": ["kernels_mfma.hip", "kernels_apply.hip", "kernel_util.hpp"]}
MEASURED_TRAFFIC = {
    # gjb_leaf_kernel: FETCH_SIZE 73,281 KiB x 2.000 + WRITE_SIZE 1,736,417 KiB
    # x 1.000 per launch (64 x 64 leaves, p = 16)
    "gj_leaf[0]": ("bc2b0ff3a2829fce", 1928.2e6),
    # gj_level_kernel + gj_level_rest_kernel (the five level launches of a
    # 64 x 64-leaf factorization): FETCH_SIZE 26,371 KiB x 2.000 + WRITE_SIZE
    # 11,559 KiB x 1.000 per level
    "gj_panel[0]": ("e597f98f58b33be5", 65.84e6),
}
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6       # MI355X FP64 vector = FP64 matrix


def kernel_source_sha(kind):
    """SHA-256 prefix of the source files of one kernel class."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kind, []):
        with open(os.path.join(ROOT, "paper_1612_02736_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def make_inputs(tree, nrhs, p=P, q=Q):
    import workloads as W
    xy = tree.leaf_cheb_nodes(p)
    X, Y = xy[..., 0], xy[..., 1]
    coeffs = np.transpose(W.varcoeff(X, Y), (1, 0, 2)).copy()     # [nl, 6, p^2]
    pi = p - 2
    ii = np.array([(iy + 1) * p + ix + 1 for iy in range(pi) for ix in range(pi)])
    Xi, Yi = X[:, ii], Y[:, ii]
    ci = coeffs[:, :, ii].transpose(1, 0, 2)
    b = tree.bdry_gauss_nodes(q)
    fs, gs = [], []
    for r in range(nrhs):
        sol = W.FourierSolution(2 + r)
        gs.append(sol.g(Xi, Yi, ci))
        fs.append(sol.u(b[:, 0], b[:, 1]))
    return (np.ascontiguousarray(coeffs), np.ascontiguousarray(np.stack(fs)),
            np.ascontiguousarray(np.stack(gs)))


def flop_model(H, solver):
    """Algorithmic flops of Algorithm 1 as implemented (explicit inverses by
    Gauss-Jordan = 2 n^3) and operator bytes read by one solve."""
    from paper_1612_02736_amd.hps import debug_boxes
    boxes = debug_boxes(solver)
    mi, me, g4 = (P - 2) ** 2, 4 * (P - 1), 4 * Q
    leaf_inv = 2.0 * mi ** 3
    leaf_gemm = 2.0 * mi * me * g4 + 4.0 * mi * mi * g4 + 2.0 * g4 * g4 * mi
    nleaf = int(np.sum(boxes[:, 0] == 1))
    merge_inv = merge_gemm = 0.0
    merge_words = 0.0
    for info in boxes:
        if info[0]:
            continue
        m, en = float(info[7]), float(info[6])
        merge_inv += 2.0 * m ** 3
        merge_gemm += 2.0 * m * m * en + (2.0 * en * en * m if info[2] >= 0 else 0.0)
        merge_words += m * m + m * en + (en * m if info[2] >= 0 else 0.0)
    leaf_words = nleaf * (mi * (g4 + mi) + g4 * mi + me * g4 / nleaf)
    return dict(leaf_inv=nleaf * leaf_inv, leaf_gemm=nleaf * leaf_gemm,
                merge_inv=merge_inv, merge_gemm=merge_gemm,
                build=nleaf * (leaf_inv + leaf_gemm) + merge_inv + merge_gemm,
                solve_bytes=8.0 * (leaf_words + merge_words), nleaf=nleaf)


def cpu_baseline(nrhs):
    """The oracle as it stands on the host, two ways: on one thread on the
    full 64 x 64-leaf problem (factor + one solve; the step's 32 solves are
    32 times the one), and with the BLAS thread pool at its default on a
    16 x 16-leaf sample (scaled by 16).  The oracle's blocks (196 x 196 and
    smaller) are too small for threaded BLAS, which makes the threaded run
    ~10-20x slower; the reported value is the faster, one-thread run."""
    from threadpoolctl import threadpool_info, threadpool_limits
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import oracle
    import workloads as W
    from oracle_cases import make_inputs as oracle_inputs

    def run(n, limit):
        t = oracle.Tree.uniform(0.0, 1.0, 0.0, 1.0, n, n)
        coeffs, f, g, _ = oracle_inputs(t, P, Q, W.varcoeff, W.FourierSolution(2))
        with threadpool_limits(limits=limit):
            threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
            t0 = time.perf_counter()
            ops = oracle.build(t, coeffs, P, Q)
            t1 = time.perf_counter()
            oracle.solve(ops, f, g)
            t2 = time.perf_counter()
        scale = (N_LEAF_SIDE * N_LEAF_SIDE) / (n * n)
        b, sv = (t1 - t0) * scale, (t2 - t1) * scale
        return {"value": nrhs / (b + nrhs * sv), "cores": int(threads),
                "sample": (f"oracle build + 1 solve on {n}x{n} leaves of the same p=16 problem "
                           f"({t1 - t0:.1f} s + {t2 - t1:.2f} s)"
                           + (f", scaled x{scale:.0f} to 64x64" if scale != 1 else "")
                           + f"; step = factor + {nrhs} solves"),
                "factor_s_scaled": b, "solve_s_scaled": sv}

    one = run(N_LEAF_SIDE, 1)
    many = run(16, None)
    out = {"value": one["value"], "unit": "solves/s", "cores": 1, "kind": "oracle",
           "host_cpu_count": os.cpu_count(),
           "sample": one["sample"], "factor_s_scaled": one["factor_s_scaled"],
           "solve_s_scaled": one["solve_s_scaled"], "default_threads": many}
    return out


def translation_invariant_case(H, torch, dev, nrhs, reps=3):
    """(I - dt Lap) u = g on 128 x 128 leaves, p = 12: factor and 32-RHS
    solve times of the full build and of the translation-invariant one."""
    import workloads as W
    n, p, q = 128, 12, 11
    t = H.Tree(0.0, 1.0, 0.0, 1.0, n, n)
    xy = t.leaf_cheb_nodes(p)
    coeffs = np.stack([W.heat_coeffs(xy[i, :, 0], xy[i, :, 1]) for i in range(t.n_leaves)])
    rng = np.random.default_rng(3)
    ng, nb = t.counts(q)
    cd = torch.from_numpy(coeffs).to(dev)
    fd = torch.from_numpy(rng.standard_normal((nrhs, nb))).to(dev)
    gd = torch.from_numpy(rng.standard_normal((nrhs, t.n_leaves, (p - 2) ** 2))).to(dev)
    out = {}
    for name, ti in (("full", False), ("shared", True)):
        s = H.Solver(t, cd, p, q, translation_invariant=ti)
        s.refactor(cd)
        u = s.solve(fd, gd)
        torch.cuda.synchronize()
        f0 = time.perf_counter()
        for _ in range(reps):
            s.refactor(cd)
        torch.cuda.synchronize()
        f1 = time.perf_counter()
        for _ in range(reps):
            u = s.solve(fd, gd)
        torch.cuda.synchronize()
        f2 = time.perf_counter()
        out[name] = {"factor_ms": (f1 - f0) * 1e3 / reps, "solve_ms_nrhs32": (f2 - f1) * 1e3 / reps,
                     "operator_gb": t.workspace_bytes(p, q, translation_invariant=ti) / 1e9}
        out[name + "_u"] = u
        del s
    us, uf = out.pop("shared_u"), out.pop("full_u")
    out["rel_diff_shared_vs_full"] = float((us - uf).abs().max() / uf.abs().max())
    return out


def scaling_sweep(H, torch, dev, sizes=(16, 32, 64, 128), reps=3):
    """Build and solve time and operator memory against the number of
    unknowns N = (p n)^2 (the speed and memory experiments of Sec. 7.1):
    the variable-coefficient problem on n x n leaves, p = 16, q = 15, random
    right-hand sides (timing only)."""
    out = []
    rng = np.random.default_rng(5)
    for n in sizes:
        t = H.Tree(0.0, 1.0, 0.0, 1.0, n, n)
        coeffs, _, _ = make_inputs(t, 1)
        cd = torch.from_numpy(coeffs).to(dev)
        s = H.Solver(t, cd, P, Q)
        s.refactor(cd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            s.refactor(cd)
        torch.cuda.synchronize()
        fac = (time.perf_counter() - t0) / reps
        row = {"n": n, "N": (P * n) ** 2, "factor_ms": fac * 1e3,
               "operator_bytes_per_unknown": t.workspace_bytes(P, Q) / (P * n) ** 2}
        for nrhs in (1, 32):
            f = torch.from_numpy(rng.standard_normal((nrhs, s.n_bdry))).to(dev)
            g = torch.from_numpy(rng.standard_normal((nrhs, t.n_leaves, (P - 2) ** 2))).to(dev)
            s.solve(f, g)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                s.solve(f, g)
            torch.cuda.synchronize()
            row[f"solve_ms_nrhs{nrhs}"] = (time.perf_counter() - t0) * 1e3 / reps
        out.append(row)
        del s, cd
        torch.cuda.empty_cache()
    return out


def crank_nicolson_case(H, torch, dev, k=0.01, steps=50):
    """The parabolic problem of Sec. 7.6: u_t = eps Lap u - u_x on 16 x 16
    leaves, periodic in x, zero Neumann data in y, Crank-Nicolson with time
    step k (p = 16, q = 14).  One step = the right side sigma u - L u on the
    leaf grids plus one solve.  The initial value is the eigenmode
    e^{2 pi i x} cos(pi y), whose Crank-Nicolson iterates are known in closed
    form, so the error of the run is reported too."""
    import workloads as W
    n, p, q = 16, 16, 14
    t = H.Tree(0.0, 1.0, 0.0, 1.0, n, n).set_bc("NPNP")
    xy = t.leaf_cheb_nodes(p)
    X, Y = xy[..., 0], xy[..., 1]
    coeffs = np.stack([W.convdiff_coeffs(X[i], Y[i], k) for i in range(t.n_leaves)])
    cd = torch.from_numpy(coeffs).to(dev)
    s = H.Solver(t, cd, p, q)
    torch.cuda.synchronize()
    b0 = time.perf_counter()
    s.refactor(cd)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - b0) * 1e3
    f = torch.zeros((1, s.n_bdry), dtype=torch.float64, device=dev)
    u0 = torch.from_numpy((np.cos(2 * np.pi * X) * np.cos(np.pi * Y))[None]).to(dev)
    u = s.solve(f, s.apply_operator(u0, 2.0 / k))     # warm-up step
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u = u0
    for _ in range(steps):
        u = s.solve(f, s.apply_operator(u, 2.0 / k))
    torch.cuda.synchronize()
    step_ms = (time.perf_counter() - t0) * 1e3 / steps
    lam = 5 * W.CD_EPS * np.pi ** 2 + 2j * np.pi
    R = (1 - k * lam / 2) / (1 + k * lam / 2)
    closed = np.real(R ** steps * np.exp(2j * np.pi * X)) * np.cos(np.pi * Y)
    err = float(np.abs(u[0].cpu().numpy() - closed).max() / np.abs(closed).max())
    out = {"leaves": n * n, "p": p, "q": q, "k": k, "steps": steps, "build_ms": build_ms,
           "step_ms": step_ms, "steps_per_s": 1e3 / step_ms,
           "rel_err_vs_cn_closed_form": err,
           "operator_gb": t.workspace_bytes(p, q) / 1e9}
    # the operator has constant coefficients: one operator copy per distinct box
    del s
    s2 = H.Solver(t, cd, p, q, translation_invariant=True)
    torch.cuda.synchronize()
    b0 = time.perf_counter()
    s2.refactor(cd)
    torch.cuda.synchronize()
    b1 = time.perf_counter()
    v = u0
    for _ in range(steps):
        v = s2.solve(f, s2.apply_operator(v, 2.0 / k))
    torch.cuda.synchronize()
    b2 = time.perf_counter()
    out["translation_invariant"] = {
        "build_ms": (b1 - b0) * 1e3, "step_ms": (b2 - b1) * 1e3 / steps,
        "operator_gb": t.workspace_bytes(p, q, translation_invariant=True) / 1e9,
        "rel_diff_vs_full": float((v - u).abs().max() / u.abs().max())}
    return out


def heat_stepping_case(H, torch, dev, ntraj=32, nsteps=8):
    """Backward-Euler heat stepping (I - dt Lap) u_{n+1} = u_n, dt = 1e-3, on
    128 x 128 leaves, p = 12, q = 11, f = 0: one factorization, then 32
    trajectories (seeded Gaussian-bump initial values, seeds 0..31) advanced
    8 steps each, every step one solve of the batch of 32 right-hand sides
    (256 solves), in FP64 and in mixed precision (FP32 sweeps refined in
    FP64 to 1e-10).  The next right-hand side is the interior of the last
    solution (a device gather between the solves, inside the timing)."""
    import workloads as W
    n, p, q = 128, 12, 11
    t = H.Tree(0.0, 1.0, 0.0, 1.0, n, n)
    xy = t.leaf_cheb_nodes(p)
    X, Y = xy[..., 0], xy[..., 1]
    coeffs = np.stack([W.heat_coeffs(X[i], Y[i]) for i in range(t.n_leaves)])
    cd = torch.from_numpy(coeffs).to(dev)
    s = H.Solver(t, cd, p, q, keep_fp32=True)
    torch.cuda.synchronize()
    b0 = time.perf_counter()
    s.refactor(cd)
    torch.cuda.synchronize()
    factor_ms = (time.perf_counter() - b0) * 1e3
    pi = p - 2
    inner = torch.tensor([(iy + 1) * p + ix + 1 for iy in range(pi) for ix in range(pi)],
                         device=dev)
    u0 = torch.from_numpy(np.stack([W.gaussian_bumps(X, Y, k) for k in range(ntraj)])).to(dev)
    f = torch.zeros((ntraj, s.n_bdry), dtype=torch.float64, device=dev)
    out = {"workload": f"heat, backward Euler dt=1e-3, {n}x{n} leaves, p={p}, q={q}, "
                       f"{ntraj} trajectories x {nsteps} steps",
           "factor_ms": factor_ms}
    finals = {}
    for name, prec in (("fp64", H.HPS_PREC_FP64), ("mixed", H.HPS_PREC_MIXED)):
        u = u0
        s.solve(f, u.index_select(2, inner).contiguous(), precision=prec)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = {}
        for _ in range(nsteps):
            u = s.solve(f, u.index_select(2, inner).contiguous(), precision=prec, stats=stats)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[f"solves_per_s_{name}"] = ntraj * nsteps / dt
        out[f"ms_per_step_{name}"] = dt * 1e3 / nsteps
        if name == "mixed":
            out["mixed_refinement_steps"] = stats.get("iters")
        finals[name] = u
    out["rel_diff_mixed_vs_fp64_after_8_steps"] = float(
        (finals["mixed"] - finals["fp64"]).abs().max() / finals["fp64"].abs().max())
    del s
    torch.cuda.empty_cache()
    return out


def refined_forest_case(H, torch, dev, reps=3):
    """64 independent problems in one build: 4 x 4 base leaves refined 8
    levels toward a seeded point (seed 100 + k), coefficients of the
    variable-coefficient family with seeded phases, Gaussian load of width
    1e-3, zero boundary data, p = 16, q = 14.  Build time, solve time for the
    64 loads (one right-hand side covers every problem), and the error
    against stored oracle values of problems 0 and 37."""
    import workloads as W
    nprob, p, q = 64, 16, 14
    draws = [W.refined_problem(100 + k) for k in range(nprob)]
    t = H.Tree(0, 1, 0, 1, 4, 4, nprob)
    for k, (_, xh) in enumerate(draws):
        t.refine_point(k, xh[0], xh[1], 8)
    xy = t.leaf_cheb_nodes(p)
    # leaves are in canonical (problem, y0, x0) order: problem k's leaves are
    # the k-th contiguous run; its length follows from the per-problem counts
    boxes = t.leaf_boxes()
    starts = [0]
    for i in range(1, t.n_leaves):
        if boxes[i, 2] < boxes[i - 1, 2] - 1e-12 or (
                boxes[i, 2] == boxes[i - 1, 2] and boxes[i, 0] < boxes[i - 1, 0]):
            starts.append(i)
    prob = np.zeros(t.n_leaves, dtype=int)
    for k, st in enumerate(starts):
        prob[st:] = k
    coeffs = np.stack([W.varcoeff(xy[i, :, 0], xy[i, :, 1], draws[prob[i]][0])
                       for i in range(len(xy))])
    pi = p - 2
    inner = np.array([(iy + 1) * p + ix + 1 for iy in range(pi) for ix in range(pi)])
    g = np.stack([W.gaussian_load(xy[i, inner, 0], xy[i, inner, 1], draws[prob[i]][1])
                  for i in range(len(xy))])
    cd = torch.from_numpy(coeffs).to(dev)
    fd = torch.zeros((1, t.counts(q)[1]), dtype=torch.float64, device=dev)
    gd = torch.from_numpy(g[None]).to(dev)
    s = H.Solver(t, cd, p, q)
    s.refactor(cd)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        s.refactor(cd)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    u = s.solve(fd, gd)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(reps):
        u = s.solve(fd, gd)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    out = {"workload": f"{nprob} problems, 4x4 base leaves refined 8 levels, p={p}, q={q}",
           "leaves": t.n_leaves, "leaves_per_problem_min": int(np.bincount(prob).min()),
           "leaves_per_problem_max": int(np.bincount(prob).max()),
           "build_s": (t1 - t0) / reps, "solve_ms": (t3 - t2) * 1e3 / reps,
           "solves_per_s": reps / (t3 - t2), "problems_per_s": nprob * reps / (t3 - t2)}
    ref = os.path.join(ROOT, "tests", "golden", "oracle_refined_forest_p16_q14.npz")
    if os.path.exists(ref):
        z = np.load(ref, allow_pickle=False)
        uu = u[0].cpu().numpy()
        errs = {}
        for k in z["problems"]:
            uo = z[f"u_problem{k}"]
            mine = uu[prob == k]
            errs[int(k)] = (float(np.max(np.abs(mine - uo)) / np.max(np.abs(uo)))
                            if mine.shape == uo.shape else None)
        out["rel_err_vs_oracle_sampled_problems"] = errs
    del s
    torch.cuda.empty_cache()
    return out


def gradient_case(H, torch, dev, reps=3):
    """Loss sum (u - u_obs)^2 over 32 problems of 32 x 32 leaves, p = 16
    (variable-coefficient family with seeded phases, u_obs from a perturbed
    zeroth-order coefficient): forward (refactor with c, then solve) and
    backward (transposed sweeps and the coefficient gradient) through the
    torch.autograd.Function; the adjoint's cost over the forward cost."""
    import workloads as W
    from paper_1612_02736_amd.autograd import hps_solve
    n, p, q, nprob = 32, 16, 15, 32
    t = H.Tree(0, 1, 0, 1, n, n, nprob)
    nl = t.n_leaves
    per = nl // nprob
    xy = t.leaf_cheb_nodes(p)
    phases = [W.problem_phases(300 + k) for k in range(nprob)]
    coeffs = np.stack([W.varcoeff(xy[i, :, 0], xy[i, :, 1], phases[i // per])
                       for i in range(nl)])
    pi = p - 2
    inner = np.array([(iy + 1) * p + ix + 1 for iy in range(pi) for ix in range(pi)])
    sol = W.FourierSolution(2)
    g = np.stack([sol.g(xy[i, inner, 0], xy[i, inner, 1], coeffs[i][:, inner])
                  for i in range(nl)])
    b = t.bdry_gauss_nodes(q)
    f = sol.u(b[:, 0], b[:, 1])
    cd = torch.from_numpy(coeffs).to(dev)
    s = H.Solver(t, cd, p, q)
    pert = W.Perturbation(3)
    c_obs = torch.from_numpy(coeffs[:, 5] * (1 + 0.1 * pert(xy[..., 0], xy[..., 1]))).to(dev)
    fd = torch.from_numpy(f[None]).to(dev)
    gd = torch.from_numpy(g[None]).to(dev)
    with torch.no_grad():
        u_obs = hps_solve(s, cd, c_obs, gd, fd)
    fw = bw = 0.0
    sol_ms = adj_ms = 0.0
    for r in range(reps + 1):
        c = cd[:, 5].clone().requires_grad_(True)
        gv = gd.clone().requires_grad_(True)
        fv = fd.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u = hps_solve(s, cd, c, gv, fv)
        L = ((u - u_obs) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        # the solve alone and the transposed sweeps alone, on the same handle
        us = s.solve(fd, gd)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        s.solve_adjoint(2.0 * (us - u_obs))
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        if r:
            fw += t1 - t0
            bw += t2 - t1
            sol_ms += (t3 - t2) * 1e3
            adj_ms += (t4 - t3) * 1e3
    out = {"workload": f"{nprob} problems x {n}x{n} leaves, p={p}, loss ||u - u_obs||^2",
           "forward_ms": fw * 1e3 / reps, "backward_ms": bw * 1e3 / reps,
           "backward_over_forward": bw / fw,
           "solve_ms": sol_ms / reps, "adjoint_sweeps_ms": adj_ms / reps,
           "adjoint_over_solve": adj_ms / sol_ms}
    del s
    torch.cuda.empty_cache()
    return out


def concurrent_steps(H, tree, cd, fd, gd, nstreams=3, steps=8):
    """Throughput with nstreams independent steps in flight: one handle and
    one HIP stream per host thread (the library's calls release the GIL
    while they wait), each thread running `steps` full steps (factor + 32-RHS
    FP64 solve) of the same workload.  While one step's upper merge levels
    run their latency-bound interface inversions, another step's leaf and
    GEMM work fills the chip.  Reported beside the one-stream headline."""
    import threading
    import torch
    sols = [H.Solver(tree, cd, P, Q) for _ in range(nstreams)]
    streams = [torch.cuda.Stream() for _ in range(nstreams)]
    for s, st in zip(sols, streams):
        s.refactor(cd, stream=st)
        s.solve(fd, gd, stream=st)
    torch.cuda.synchronize()
    errors = []

    def worker(i):
        try:
            for _ in range(steps):
                sols[i].refactor(cd, stream=streams[i])
                sols[i].solve(fd, gd, stream=streams[i])
        except Exception as e:           # reported after the join
            errors.append(e)

    t0 = time.perf_counter()
    th = [threading.Thread(target=worker, args=(i,)) for i in range(nstreams)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if errors:
        raise errors[0]
    n = nstreams * steps
    return {"streams": nstreams, "steps": n, "ms_per_step": dt * 1e3 / n,
            "solves_per_s": 32 * n / dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nrhs", type=int, default=NRHS)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweep", action="store_true",
                    help="also time build and solve against N (16x16 to 128x128 leaves)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="one eager factor + solve and a 1 GiB device copy (for HBM "
                         "counter runs: the copy calibrates FETCH_SIZE / WRITE_SIZE); "
                         "prints no benchmark line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU; this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1612_02736_amd as H
    from paper_1612_02736_amd.hps import debug_profile, debug_profile_read
    H.lib()
    dev = torch.device("cuda:0")
    tree = H.Tree(0.0, 1.0, 0.0, 1.0, N_LEAF_SIDE, N_LEAF_SIDE)
    coeffs, f, g = make_inputs(tree, args.nrhs)
    cd = torch.from_numpy(coeffs).to(dev)
    fd = torch.from_numpy(f).to(dev)
    gd = torch.from_numpy(g).to(dev)
    solver = H.Solver(tree, cd, P, Q)
    if args.traffic_probe:
        debug_profile(solver, True)        # eager launches, one dispatch per step
        solver.refactor(cd)
        solver.solve(fd, gd)
        debug_profile(solver, False)
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print("traffic probe done", flush=True)
        return
    fm = flop_model(H, solver)
    for _ in range(args.warmup):
        solver.refactor(cd)
        u = solver.solve(fd, gd)
    torch.cuda.synchronize()
    ev = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e2 = torch.cuda.Event(enable_timing=True)
        e0.record()
        solver.refactor(cd)
        e1.record()
        u = solver.solve(fd, gd)
        e2.record()
        ev.append((e0, e1, e2))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    # per-launch HIP events on separate (eager, untimed) steps of the same work
    debug_profile(solver, True)
    for _ in range(args.steps):
        solver.refactor(cd)
        solver.solve(fd, gd)
    prof = debug_profile_read(solver, with_work=True)
    debug_profile(solver, False)
    factor_ms = float(np.median([a.elapsed_time(b) for a, b, _ in ev]))
    solve32_ms = float(np.median([b.elapsed_time(c) for _, b, c in ev]))
    # solve-only throughput at nrhs = 1 (outside the timed steps)
    f1, g1 = fd[:1].contiguous(), gd[:1].contiguous()
    solver.solve(f1, g1)
    torch.cuda.synchronize()
    s0 = time.perf_counter()
    for _ in range(10):
        solver.solve(f1, g1)
    torch.cuda.synchronize()
    solve1_ms = (time.perf_counter() - s0) * 1e2
    conc = concurrent_steps(H, tree, cd, fd, gd) if args.nrhs == 32 else None
    # mixed precision (FP32 sweeps + FP64 residual refinement) at nrhs = 32,
    # on a handle that also keeps FP32 copies of the solve operators (their
    # cast is timed on its own, outside the FP64 factorization)
    sm = H.Solver(tree, cd, P, Q, keep_fp32=True)
    sm.refactor(cd)
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    for _ in range(3):
        sm.refactor(cd)
    torch.cuda.synchronize()
    factor_fp32_copies_ms = (time.perf_counter() - c0) * 1e3 / 3
    stats = {}
    um = sm.solve(fd, gd, precision=H.HPS_PREC_MIXED, stats=stats)
    torch.cuda.synchronize()
    m0 = time.perf_counter()
    for _ in range(3):
        um = sm.solve(fd, gd, precision=H.HPS_PREC_MIXED, stats=stats)
    torch.cuda.synchronize()
    mixed_ms = (time.perf_counter() - m0) * 1e3 / 3
    u32 = sm.solve(fd, gd, precision=H.HPS_PREC_FP32)
    torch.cuda.synchronize()
    m1 = time.perf_counter()
    for _ in range(3):
        u32 = sm.solve(fd, gd, precision=H.HPS_PREC_FP32)
    torch.cuda.synchronize()
    fp32_sweep_ms = (time.perf_counter() - m1) * 1e3 / 3
    del sm, u32
    # adjoint (transposed sweeps) at nrhs = 32
    ub = torch.ones_like(u)
    solver.solve_adjoint(ub)
    torch.cuda.synchronize()
    a0 = time.perf_counter()
    for _ in range(3):
        solver.solve_adjoint(ub)
    torch.cuda.synchronize()
    adj_ms = (time.perf_counter() - a0) * 1e3 / 3
    # storage-economic version (leaf F not stored, recomputed by every solve)
    se = H.Solver(tree, cd, P, Q, economic=True)
    ue = se.solve(fd, gd)
    torch.cuda.synchronize()
    e0 = time.perf_counter()
    for _ in range(3):
        ue = se.solve(fd, gd)
    torch.cuda.synchronize()
    econ_ms = (time.perf_counter() - e0) * 1e3 / 3
    econ_diff = float((ue - u).abs().max() / u.abs().max())
    del se, ue
    ws_full, ws_econ = tree.workspace_bytes(P, Q), tree.workspace_bytes(P, Q, economic=True)
    # translation-invariant builds, reported apart from the general path: the
    # constant-coefficient heat operator on 128 x 128 leaves, p = 12, 32 RHS,
    # full build vs one operator copy per distinct box
    ti = translation_invariant_case(H, torch, dev, args.nrhs)
    cn = crank_nicolson_case(H, torch, dev)
    sweep = scaling_sweep(H, torch, dev) if args.sweep else None
    heat = heat_stepping_case(H, torch, dev)
    forest = refined_forest_case(H, torch, dev)
    grad = gradient_case(H, torch, dev)
    # accuracy against stored oracle values (seed 2 = right-hand side 0)
    rel_err = rel_err_mixed = None
    ref = os.path.join(ROOT, "tests", "golden", "oracle_varcoeff_64x64_p16_seed2.npz")
    if os.path.exists(ref):
        z = np.load(ref, allow_pickle=False)
        scale = np.max(np.abs(z["u"]))
        rel_err = float(np.max(np.abs(u[0].cpu().numpy()[z["leaves"]] - z["u"])) / scale)
        rel_err_mixed = float(np.max(np.abs(um[0].cpu().numpy()[z["leaves"]] - z["u"])) / scale)
    # dominant kernel from the per-launch events of the timed steps; each
    # launch carries its algorithmic work (flops, or operator elements applied
    # to each right-hand side)
    agg, work = {}, {}
    for kind, var, ms, w in prof:
        agg.setdefault((kind, var), []).append(ms)
        work[(kind, var)] = work.get((kind, var), 0.0) + w
    per_step = {k: sum(v) / args.steps for k, v in agg.items()}
    rates = {}
    for k, v in agg.items():
        t = sum(v) * 1e-3
        if k[0] == "apply":
            rates[f"{k[0]}[{k[1]}]"] = {"GB/s": 8.0 * work[k] / t / 1e9,
                                       "TFLOP/s": 2.0 * args.nrhs * work[k] / t / 1e12}
        elif work[k] > 0:
            rates[f"{k[0]}[{k[1]}]"] = {"TFLOP/s": work[k] / t / 1e12}
    dom = max(per_step, key=per_step.get)
    avg_ms = sum(agg[dom]) / len(agg[dom])
    w_launch = work[dom] / len(agg[dom])
    if dom[0] == "apply":
        # operator bytes vs FMA flops of one launch: the larger time decides
        by = 8.0 * w_launch
        fl = 2.0 * args.nrhs * w_launch
        if by / (HBM_PEAK_GBS * 1e9) >= fl / (FP64_PEAK_TFLOPS * 1e12):
            roof = {"bound": "hbm", "achieved": by / (avg_ms * 1e-3) / 1e9,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s"}
        else:
            roof = {"bound": "alu", "achieved": fl / (avg_ms * 1e-3) / 1e12,
                    "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s"}
    else:
        # the GEMMs and the blocked leaf Gauss-Jordan (its panel updates,
        # 94% of its flops per the SQ_INSTS_VALU_MFMA_MOPS_F64 counter) run on
        # the matrix cores; the interface inversions on the vector ALU (same
        # FP64 peak on MI355X)
        roof = {"bound": "mfma" if dom[0] in ("gemm", "gj_leaf") else "alu",
                "achieved": w_launch / (avg_ms * 1e-3) / 1e12,
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    meas = MEASURED_TRAFFIC.get(f"{dom[0]}[{dom[1]}]")
    if meas and meas[0] == kernel_source_sha(dom[0]):
        roof["traffic"] = meas[1]
    roof["kernel"] = f"{dom[0]}[{dom[1]}]"
    roof["avg_launch_ms"] = avg_ms
    out = {
        "metric": "factor s + solves/s at N≈1M p=16 (FP64 vs mixed); TFLOP/s, rel err vs FP64",
        "value": args.nrhs * 1e3 / ms_step,
        "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "variable-coefficient A on [0,1]^2, 64x64 leaves, p=16, q=15, "
                               "N=1,048,576, 32 RHS per step (factor + FP64 solve)",
                   "leaves": fm["nleaf"], "p": P, "q": Q, "nrhs": args.nrhs,
                   "parallelism": "single GPU"},
        "factor_s": factor_ms * 1e-3,
        "concurrent_independent_steps": conc,
        "build_tflops": fm["build"] / (factor_ms * 1e-3) / 1e12,
        "build_gflop": fm["build"] / 1e9,
        "solve_ms_fp64_nrhs32": solve32_ms,
        "solves_per_s_fp64_nrhs32": args.nrhs * 1e3 / solve32_ms,
        "solve_ms_fp64_nrhs1": solve1_ms,
        "solves_per_s_fp64_nrhs1": 1e3 / solve1_ms,
        "solve_ms_mixed_nrhs32": mixed_ms,
        "solves_per_s_mixed_nrhs32": args.nrhs * 1e3 / mixed_ms,
        "solve_ms_fp32_sweep_nrhs32": fp32_sweep_ms,
        "factor_ms_with_fp32_copies": factor_fp32_copies_ms,
        "mixed_refinement_steps": stats.get("iters"),
        "mixed_last_correction": stats.get("resid"),
        "adjoint_ms_nrhs32": adj_ms,
        "adjoint_over_forward": adj_ms / solve32_ms,
        "solve_operator_gb": fm["solve_bytes"] / 1e9,
        "economic_solve_ms_nrhs32": econ_ms,
        "economic_over_stored_solve": econ_ms / solve32_ms,
        "economic_rel_diff_vs_stored": econ_diff,
        "operator_gb_stored": ws_full / 1e9,
        "operator_gb_economic": ws_econ / 1e9,
        "translation_invariant_heat_128x128_p12": ti,
        "crank_nicolson_periodic_neumann_16x16_p16": cn,
        "heat_backward_euler_128x128_p12": heat,
        "refined_forest_64_problems_p16": forest,
        "gradient_32_problems_32x32_p16": grad,
        "rel_err_vs_oracle": rel_err,
        "rel_err_mixed_vs_oracle": rel_err_mixed,
        "kernel_ms_per_step": {f"{k[0]}[{k[1]}]": v for k, v in sorted(per_step.items(), key=lambda kv: -kv[1])},
        "kernel_rates": rates,
        "roofline": roof,
    }
    if sweep is not None:
        out["scaling_varcoeff_p16"] = sweep
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.nrhs)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
