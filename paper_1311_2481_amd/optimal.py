"""Nonlinear optimal perturbation on the GPU: projected gradient ascent of
the final perturbation energy on the sphere of fixed initial perturbation
energy, with the control of libtc's control entry points (the initial
perturbation as the curl of a smooth vector potential; see include/tc.h).

Each iteration runs the forward steps with checkpoints and the reverse
sweep of the discrete adjoint (``autograd.final_energy_and_gradient``),
carries the gradient to the control (``tc_control_gradient``), and takes
the step on the sphere (``tc_control_ascent_update``).  This module only
orders the library calls and halves the step when the objective would
fall.
"""
from .autograd import final_energy_and_gradient


def objective_and_gradient(S, a, nsteps, every=20):
    """J = E_pert(u^T) from u^0 = U_c + B a, and dJ/da."""
    u0 = S.control_velocity(a)
    J, g = final_energy_and_gradient(S, u0, S.zeros(3), nsteps, every=every)
    return J, S.control_gradient(g)


def ascent(S, a0, E0, nsteps, iters, every=20, tau=None, min_tau=1e-12):
    """Projected gradient ascent; returns (a, [J of every accepted iterate])."""
    a, st = S.control_ascent_update(a0, None, None, 0.0, E0)
    J, G = objective_and_gradient(S, a, nsteps, every)
    history = [J]
    for _ in range(iters):
        gE = S.control_gradient(S.energy_gradient(S.control_velocity(a)))
        if tau is None:
            _, st = S.control_ascent_update(a, G, gE, 0.0, E0)
            tau = 0.1 * st["control_norm"] / max(st["step_norm"], 1e-300)
        while True:
            b, _ = S.control_ascent_update(a, G, gE, tau, E0)
            Jb, Gb = objective_and_gradient(S, b, nsteps, every)
            if Jb >= J or tau < min_tau:
                break
            tau *= 0.5
        a, J, G = b, Jb, Gb
        history.append(J)
    return a, history
