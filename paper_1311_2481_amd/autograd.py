"""Gradient of the final perturbation energy through the library's adjoint.

``TCSteps.apply(u0_pert, solver, u_base, nsteps, every)`` runs ``nsteps``
projection steps from u0 = u_base + u0_pert (history u^{-1} = u^0,
N^{-1} = N(u^0)) and returns J = E_pert(u^T).  Its backward pass is the
discrete adjoint of the steps (tc_step_adjoint): the forward keeps the
state (u^i, u^{i-1}, N^{i-1}) every ``every`` steps; the reverse sweep
recomputes one segment at a time from its checkpoint, so memory holds
nsteps/every checkpoints plus one segment of velocities.  Every step,
forward or adjoint, runs in libtc's kernels; this module only orders the
calls and holds the checkpoints.
"""
import torch


class TCSteps(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0_pert, solver, u_base, nsteps, every):
        u0 = (u_base + u0_pert).contiguous()
        solver.set_state(u0)
        checkpoints = []
        done = 0
        while done < nsteps:
            if done % every == 0:
                u, _ = solver.get_state()
                up, Np = solver.get_history()
                checkpoints.append((done, u, up, Np))
            k = min(every - done % every, nsteps - done)
            solver.step(k)
            done += k
        uT = solver.get_state(with_pressure=False)
        J = solver.diag()["perturbation_energy"]
        ctx.solver, ctx.nsteps, ctx.every = solver, nsteps, every
        ctx.checkpoints, ctx.uT, ctx.u0 = checkpoints, uT, u0
        return torch.tensor(J, dtype=torch.float64, device=u0.device)

    @staticmethod
    def backward(ctx, gJ):
        S = ctx.solver
        # cotangents of (u^{k+1}, u^k, N^k) in one 9-field buffer; two such
        # buffers in turn take the input and the output of each adjoint step
        bufs = [S.zeros(9), S.empty(9)]
        S.adjoint_seed(ctx.uT, float(gJ), out=bufs[0][0:3])
        cur = 0
        # one segment's velocities, newest first: fields 3m .. 3m+2 hold
        # u^{end-1-m}, so the inputs (u^k, u^{k-1}) of step k are the six
        # fields from 3 (end-1-k) on, with no copy
        seg = S.empty(3 * (ctx.every + 1))
        for start, cu, cup, cNp in reversed(ctx.checkpoints):
            end = min(start + ctx.every, ctx.nsteps)
            n = end - start
            # recompute the segment from its checkpoint
            S.set_state(cu, cup, cNp)
            seg[3 * n:3 * n + 3].copy_(cup)
            seg[3 * (n - 1):3 * n].copy_(cu)
            for k in range(start + 1, end):
                S.step(1)
                m = end - 1 - k
                S.get_state(with_pressure=False, out=seg[3 * m:3 * m + 3])
            for k in range(end - 1, start - 1, -1):
                m = end - 1 - k
                S.step_adjoint(seg[3 * m:3 * m + 6], bufs[cur], bufs[1 - cur])
                cur = 1 - cur
        # initial history: u^{-1} = u^0 and N^{-1} = N(u^0)
        g = S.adjoint_initial_history(ctx.u0, bufs[cur])
        return g, None, None, None, None


def final_energy_and_gradient(solver, u_base, u0_pert, nsteps, every=20):
    """(J, dJ/du0_pert) for J = E_pert after nsteps steps."""
    x = u0_pert.detach().clone().requires_grad_(True)
    J = TCSteps.apply(x, solver, u_base, nsteps, every)
    J.backward()
    return float(J.detach()), x.grad
