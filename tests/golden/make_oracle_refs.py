"""Write oracle reference values for full-size GPU parity tests.

Runs only the oracle (no library code): the 64 x 64-leaf, p = 16 variable-
coefficient workload with the seeded Fourier solution (seed 2), and stores u
on every 64th leaf in canonical order.  Usage:
python tests/golden/make_oracle_refs.py
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


def main():
    n, p, q, seed = 64, 16, 15, 2
    t0 = time.time()
    tree = oracle.Tree.uniform(0.0, 1.0, 0.0, 1.0, n, n)
    sol = W.FourierSolution(seed)
    coeffs, f, g, ex = make_inputs(tree, p, q, W.varcoeff, sol)
    ops = oracle.build(tree, coeffs, p, q)
    uc, u = oracle.solve(ops, f, g)
    leaves = np.arange(0, n * n, 64)
    np.savez_compressed(os.path.join(HERE, "oracle_varcoeff_64x64_p16_seed2.npz"),
                        leaves=leaves, u=uc[leaves], err_vs_exact=np.max(np.abs(uc - ex)) / np.max(np.abs(ex)))
    print("done in", time.time() - t0, "s; oracle error vs manufactured u:",
          np.max(np.abs(uc - ex)) / np.max(np.abs(ex)))


if __name__ == "__main__":
    main()
