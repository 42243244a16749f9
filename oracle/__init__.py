"""Plain CPU FP64 oracle for the HPS build and solve stages.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The library under
``paper_1612_02736_amd`` never imports, links or runs anything from here, and
this package imports nothing from the library: the two share no code.

The oracle follows Babb, Gillman, Hao, Martinsson, "An accelerated Poisson
solver based on multidomain spectral discretization" (arXiv:1612.02736):

* ``spectral``  -- Chebyshev/Gauss nodes, differentiation, interpolation
                   (Sec. 3.1, 3.2, 3.4).
* ``tree``      -- the hierarchical box tree, global Gauss node numbering,
                   local refinement towards a point (Sec. 2, 4, 5.1, 5.2).
* ``leaf``      -- leaf operators F, S, H, T (Sec. 3, eqs. alpine1-alpine4).
* ``hps``       -- Algorithm 1 (build) and Algorithm 2 (solve) with explicit
                   per-box loops, plus the interface interpolation of Sec. 6.3
                   and 5.4 and the transposed (adjoint) sweeps.
* ``dense``     -- an independent route: the global collocation system
                   assembled densely/sparsely and solved by a library LU.
* ``timestep``  -- Crank-Nicolson steps with a fixed operator (Sec. 7.6).

Everything is float64 with NumPy/SciPy (LAPACK getrf/getrs) primitives.
"""

from .spectral import (cheb_nodes, diff_matrix, gauss_nodes, interp_matrix,
                       bary_weights)
from .tree import Tree
from .leaf import leaf_operators, leaf_geometry
from .hps import build, solve, solve_adjoint, coeff_gradient
from .dense import dense_solve, dense_adjoint, assemble_system, residual
from .timestep import operator_apply, crank_nicolson

__all__ = [
    "cheb_nodes", "diff_matrix", "gauss_nodes", "interp_matrix", "bary_weights",
    "Tree", "leaf_operators", "leaf_geometry", "build", "solve",
    "solve_adjoint", "coeff_gradient", "dense_solve", "dense_adjoint", "assemble_system",
    "residual", "operator_apply", "crank_nicolson",
]
