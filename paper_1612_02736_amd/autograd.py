"""torch.autograd wrapper: u = solve(c; g, f) with gradients for the nodal
zeroth-order coefficient c, the body load g and the boundary data f.

Forward: Algorithm 1 on the coefficients (the handle's operators are
recomputed in place) and Algorithm 2.  Backward: the library's transposed
sweeps (hps_solve_adjoint) give gbar and fbar; only the collocated PDE rows
depend on c, so cbar = -sum_r gbar_r * u_r on interior nodes and 0 on
exterior nodes (hps_coeff_grad_c).  The stored operators are reused, nothing
is refactored in the backward pass -- unless the solver was refactored after
this forward (another forward on the same solver, for example a loss with
two coefficient fields): then its operators belong to other coefficients,
and the backward refactors with the coefficients this forward used first.
"""

import torch


class HPSSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, solver, coeffs, c, g, f):
        """solver: a built Solver; coeffs [nl, 6, p^2] (slot 5 is replaced by
        c); c [nl, p^2]; g [nrhs, nl, (p-2)^2]; f [nrhs, n_bdry]."""
        full = coeffs.detach().clone()
        full[:, 5, :] = c.detach()
        full = full.contiguous()
        solver.refactor(full)
        u = solver.solve(f.detach().contiguous(), g.detach().contiguous())
        ctx.solver = solver
        ctx.version = solver.version
        ctx.save_for_backward(u, full)
        return u

    @staticmethod
    def backward(ctx, ubar):
        solver = ctx.solver
        u, full = ctx.saved_tensors
        if solver.version != ctx.version:
            # the operators were rebuilt for other coefficients since forward
            solver.refactor(full)
            ctx.version = solver.version
        fbar, gbar = solver.solve_adjoint(ubar.contiguous())
        cbar = None
        if ctx.needs_input_grad[2]:
            cbar = solver.coeff_grad_c(u, gbar).sum(0)
        return None, None, cbar, gbar, fbar


def hps_solve(solver, coeffs, c, g, f):
    return HPSSolve.apply(solver, coeffs, c, g, f)
