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
        ub = S.adjoint_seed(ctx.uT, float(gJ))
        upb = torch.zeros_like(ub)
        Nb = torch.zeros_like(ub)
        adj_in = S.empty(9)
        for start, cu, cup, cNp in reversed(ctx.checkpoints):
            end = min(start + ctx.every, ctx.nsteps)
            # recompute the segment: inputs (u^k, u^{k-1}) of every step in it
            S.set_state(cu, cup, cNp)
            inputs = [(cu, cup)]
            for _ in range(start, end - 1):
                S.step(1)
                u = S.get_state(with_pressure=False)
                inputs.append((u, inputs[-1][0]))
            for k in range(len(inputs) - 1, -1, -1):
                fwd = torch.cat([inputs[k][0], inputs[k][1]], 0)
                adj_in[0:3], adj_in[3:6], adj_in[6:9] = ub, upb, Nb
                out = S.step_adjoint(fwd, adj_in)
                ub, upb, Nb = out[0:3], out[3:6], out[6:9]
        # initial history: u^{-1} = u^0 and N^{-1} = N(u^0)
        adj_in[0:3], adj_in[3:6], adj_in[6:9] = ub, upb, Nb
        g = S.adjoint_initial_history(ctx.u0, adj_in)
        return g, None, None, None, None


def final_energy_and_gradient(solver, u_base, u0_pert, nsteps, every=20):
    """(J, dJ/du0_pert) for J = E_pert after nsteps steps."""
    x = u0_pert.detach().clone().requires_grad_(True)
    J = TCSteps.apply(x, solver, u_base, nsteps, every)
    J.backward()
    return float(J.detach()), x.grad
