"""Write oracle reference values for full-size GPU parity tests.

Runs only the oracle (no library code) on the 64 x 64-leaf, p = 16, q = 15
variable-coefficient workload:

* the seeded Fourier solution (seed 2): u on a sample of leaves that meets
  every leaf row and every leaf column (both diagonals), every leaf that
  borders the interfaces x = 1/2 and y = 1/2 eliminated by the two top merges
  (leaf columns 31, 32 and rows 31, 32), and the leaves along the west side;
  leaves are numbered in canonical order, iy * 64 + ix;
* the oracle's own error on the seeded polynomial of tensor degree 6
  (PolySolution(21, 6), reproduced exactly up to rounding) with both split
  orders (x first and y first): the FP64 floor that a second, equally valid
  elimination order reaches at this size.

Usage: python tests/golden/make_oracle_refs.py   (about a minute per oracle
solve on one host core).
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
import workloads as W  # noqa: E402
from oracle_cases import make_inputs  # noqa: E402

N = 64


def sample_leaves(n=N):
    ix, iy = np.meshgrid(np.arange(n), np.arange(n))
    ix, iy = ix.ravel(), iy.ravel()
    keep = ((ix == iy) | (ix == n - 1 - iy) | np.isin(ix, [n // 2 - 1, n // 2]) |
            np.isin(iy, [n // 2 - 1, n // 2]) | (ix == 0))
    return np.sort(iy[keep] * n + ix[keep])


def main():
    p, q, seed = 16, 15, 2
    t0 = time.time()
    tree = oracle.Tree.uniform(0.0, 1.0, 0.0, 1.0, N, N)
    sol = W.FourierSolution(seed)
    coeffs, f, g, ex = make_inputs(tree, p, q, W.varcoeff, sol)
    uc, _ = oracle.solve(oracle.build(tree, coeffs, p, q), f, g)
    leaves = sample_leaves()
    err_fourier = np.max(np.abs(uc - ex)) / np.max(np.abs(ex))
    print(f"Fourier solution: {len(leaves)} leaves stored, oracle error vs manufactured "
          f"u {err_fourier:.3e} ({time.time() - t0:.0f} s)", flush=True)
    poly = {}
    for tie in ("x", "y"):
        tp = oracle.Tree.uniform(0.0, 1.0, 0.0, 1.0, N, N, tie=tie)
        c2, f2, g2, ex2 = make_inputs(tp, p, q, W.varcoeff, W.PolySolution(21, 6))
        u2, _ = oracle.solve(oracle.build(tp, c2, p, q), f2, g2)
        poly[tie] = np.max(np.abs(u2 - ex2)) / np.max(np.abs(ex2))
        print(f"polynomial, split {tie} first: oracle error {poly[tie]:.3e} "
              f"({time.time() - t0:.0f} s)", flush=True)
    np.savez_compressed(os.path.join(HERE, "oracle_varcoeff_64x64_p16_seed2.npz"),
                        leaves=leaves, u=uc[leaves], err_vs_exact=err_fourier,
                        poly_err_xfirst=poly["x"], poly_err_yfirst=poly["y"])


if __name__ == "__main__":
    main()
