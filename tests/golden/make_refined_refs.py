"""Write oracle reference values for the refined-forest workload.

Runs only the oracle (no library code): problems 0 and 37 of the forest of
64 problems (4 x 4 base leaves refined 8 levels toward a seeded point,
coefficients of the variable-coefficient family with seeded phases, Gaussian
load of width 1e-3, zero boundary data; p = 16, q = 14), each on its own
tree.  Stores u on every leaf of each problem, in canonical leaf order
(y0, x0) within the problem, which is the order of the problem's leaves in
the forest.

Usage: python tests/golden/make_refined_refs.py   (seconds on one host core).
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

P, Q, N_REF, SEED0 = 16, 14, 8, 100
SAMPLED = (0, 37)


class _Load:
    """Zero boundary data and the Gaussian load at x_hat."""

    def __init__(self, xh):
        self.xh = xh

    def u(self, x, y):
        return np.zeros_like(x)

    def g(self, x, y, c):
        return W.gaussian_load(x, y, self.xh)


def main():
    out = {}
    for k in SAMPLED:
        t0 = time.time()
        ph, xh = W.refined_problem(SEED0 + k)
        tk = oracle.Tree.uniform(0, 1, 0, 1, 4, 4, 1)
        tk.refine_point(0, xh[0], xh[1], N_REF)
        c, f, g, _ = make_inputs(tk, P, Q, lambda x, y: W.varcoeff(x, y, ph), _Load(xh))
        uo, _ = oracle.solve(oracle.build(tk, c, P, Q), f, g)
        out[f"u_problem{k}"] = uo
        print(f"problem {k}: {uo.shape[0]} leaves ({time.time() - t0:.1f} s)", flush=True)
    np.savez_compressed(os.path.join(HERE, "oracle_refined_forest_p16_q14.npz"),
                        problems=np.array(SAMPLED), **out)


if __name__ == "__main__":
    main()
