"""Gradient of the final perturbation energy through the library's adjoint.

``TCSteps.apply(u0_pert, solver, u_base, nsteps, every, overlap)`` runs
``nsteps`` projection steps from u0 = u_base + u0_pert (history u^{-1} =
u^0, N^{-1} = N(u^0)) and returns J = E_pert(u^T).  Its backward pass is
the discrete adjoint of the steps (tc_step_adjoint): the forward keeps the
state (u^i, u^{i-1}, N^{i-1}) every ``every`` steps; the reverse sweep
recomputes one segment at a time from its checkpoint, so memory holds
nsteps/every checkpoints plus the velocities of one segment (two with the
overlap below).  Every step, forward or adjoint, runs in libtc's kernels;
this module only orders the calls and holds the checkpoints.

Overlap: the recomputation of the next (earlier) segment does not depend on
the adjoint steps of the current one, so with ``overlap`` a second context
(``Solver.twin``, same grid and factors) recomputes it on a second stream,
into the other of two segment buffers, while the current segment's adjoint
steps run; events order the hand-offs.  The arithmetic is the same, so the
gradient is the same bit for bit.  ``overlap=None`` takes it when the
context holds at most 4 GiB (the twin doubles that).
"""
import torch

TWIN_MAX_BYTES = 4 << 30


def _segment(solver, seg, start, end, cu, cup, cNp):
    """Recompute the velocities u^{start-1} .. u^{end-1} of one segment from
    its checkpoint into seg, newest first: fields 3m .. 3m+2 hold
    u^{end-1-m}, so the inputs (u^k, u^{k-1}) of step k are the six fields
    from 3 (end-1-k) on, with no copy."""
    n = end - start
    solver.set_state(cu, cup, cNp)
    seg[3 * n:3 * n + 3].copy_(cup)
    seg[3 * (n - 1):3 * n].copy_(cu)
    for k in range(start + 1, end):
        solver.step(1)
        m = end - 1 - k
        solver.get_state(with_pressure=False, out=seg[3 * m:3 * m + 3])


class TCSteps(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0_pert, solver, u_base, nsteps, every, overlap=None):
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
        ctx.overlap = solver.memory_bytes() <= TWIN_MAX_BYTES if overlap is None else bool(overlap)
        return torch.tensor(J, dtype=torch.float64, device=u0.device)

    @staticmethod
    def backward(ctx, gJ):
        S = ctx.solver
        main = S.stream
        # cotangents of (u^{k+1}, u^k, N^k) in one 9-field buffer; two such
        # buffers in turn take the input and the output of each adjoint step
        with torch.cuda.stream(main):
            bufs = [S.zeros(9), S.empty(9)]
            S.adjoint_seed(ctx.uT, float(gJ), out=bufs[0][0:3])
        cur = 0
        segs_desc = [(start, min(start + ctx.every, ctx.nsteps), cu, cup, cNp)
                     for start, cu, cup, cNp in reversed(ctx.checkpoints)]

        def adjoint_segment(seg, start, end):
            nonlocal cur
            for k in range(end - 1, start - 1, -1):
                m = end - 1 - k
                S.step_adjoint(seg[3 * m:3 * m + 6], bufs[cur], bufs[1 - cur])
                cur = 1 - cur

        if not ctx.overlap:
            with torch.cuda.stream(main):
                seg = S.empty(3 * (ctx.every + 1))
                for start, end, cu, cup, cNp in segs_desc:
                    _segment(S, seg, start, end, cu, cup, cNp)
                    adjoint_segment(seg, start, end)
        else:
            F = getattr(S, "_twin", None)
            if F is None:
                F = S.twin(torch.cuda.Stream(S.device))
                S._twin = F
            side = F.stream
            # allocated on main, which runs the last work on them
            with torch.cuda.stream(main):
                segs = [S.empty(3 * (ctx.every + 1)), S.empty(3 * (ctx.every + 1))]
            released = [None, None]  # event: the adjoint steps are done with segs[b]
            begin = torch.cuda.Event()
            begin.record(main)  # the checkpoints and seed are written on main

            def recompute(i):
                b = i % 2
                side.wait_event(begin)
                if released[b] is not None:
                    side.wait_event(released[b])
                with torch.cuda.stream(side):
                    _segment(F, segs[b], *segs_desc[i])
                ev = torch.cuda.Event()
                ev.record(side)
                return ev

            ready = recompute(0)
            for i, (start, end, _, _, _) in enumerate(segs_desc):
                nxt = recompute(i + 1) if i + 1 < len(segs_desc) else None
                main.wait_event(ready)
                with torch.cuda.stream(main):
                    adjoint_segment(segs[i % 2], start, end)
                released[i % 2] = torch.cuda.Event()
                released[i % 2].record(main)
                ready = nxt
        # initial history: u^{-1} = u^0 and N^{-1} = N(u^0)
        with torch.cuda.stream(main):
            g = S.adjoint_initial_history(ctx.u0, bufs[cur])
        return g, None, None, None, None, None


def final_energy_and_gradient(solver, u_base, u0_pert, nsteps, every=20, overlap=None):
    """(J, dJ/du0_pert) for J = E_pert after nsteps steps."""
    x = u0_pert.detach().clone().requires_grad_(True)
    J = TCSteps.apply(x, solver, u_base, nsteps, every, overlap)
    J.backward()
    return float(J.detach()), x.grad
