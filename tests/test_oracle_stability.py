"""Growth of the linearised step around circular Couette flow, one Fourier
mode at a time (power iteration of the tangent-linear step).

Around Couette flow (mode (0,0) only) the linearised nonlinear term couples
each mode to itself, so a grid whose single stored mode carries the mode's
wavenumbers (rescaled k_theta, k_z) gives that mode's step exactly.  The
parameters are those of the differentiation workload: eta = 0.71, Re_i =
1000, Re_o = 0, N_r = 64.  These tests record which reading of the paper
each time-step limit comes from:

* small dt: the correction of mode (0,0) must remove its radial velocity
  entirely (d_r phi = u*_r, the exact solution of eq. correction for that
  mode).  Taking d_r phi from the discrete phi solve instead (the FD
  Laplacian P is not the discrete divergence of the discrete gradient, so
  that projection is not idempotent) makes mode (0,0) grow below about
  dt = 5e-7, where viscous damping no longer outweighs it;
* large dt: the rotational form omega x u (the pressure then carries
  |u|^2/2 and its explicitly extrapolated wall condition a term U d_r u_theta)
  makes mode (n, l) = (1, 0) grow from dt = 1e-6 on; the paper's convective
  form u.grad u does not.
"""
import numpy as np
import pytest

import oracle
from oracle import adjoint as adj
from oracle import diagnostics as dg
from oracle import nonlinear as nl
from oracle import scheme

ETA, RE_I, RE_O, N_R = 0.71, 1000.0, 0.0, 64


def one_mode(dt, a, b):
    """Problem whose one stored mode has azimuthal and axial wavenumbers a, b."""
    if a == 0 and b == 0:
        return oracle.Problem(N_R, 1, 2, ETA, RE_I, RE_O, dt), (0, 0)
    P = oracle.Problem(N_R, 2, 4, ETA, RE_I, RE_O, dt, k_theta=a or 1.0, k_z=b or 1.0)
    return P, (1 if b else 0, 1 if a else 0)


def pc_linear_plain_gradient(P, Ne, u, up):
    """The linear part of steps 2-5 with the plain gradient of the discrete
    phi at every mode, (0,0) included (a reading the oracle does not take)."""
    I, Wm = adj._interior_mask(P), adj._wall_mask(P)
    z = scheme.zero_nyquist
    rhs_p = -scheme.div(P, Ne) * I + Wm * (-0.5 * (Ne[0] + Ne[1]) + scheme.vector_laplacian_r(P, 2 * u - up))
    p = P.solve("P", z(P, rhs_p))
    rhs_u = (-(4.0 * u - up) / (2.0 * P.dt) + Ne + scheme.grad(P, p)) * I
    us = np.stack([P.solve(k, z(P, rhs_u[c])) for c, k in enumerate(("Up", "Um", "Uz"))])
    phi = P.solve("P", z(P, scheme.div(P, us) * I))
    return z(P, us - scheme.grad(P, phi))


def growth(P, mode, form="rot", pc=None, steps=300, seed=0):
    """Mean growth factor per step of a random tangent over the last half of
    `steps` power iterations (the dominant |eigenvalue| when one mode grows)."""
    s, n = mode
    base = dg.couette_state(P)
    rng = np.random.default_rng(seed)
    pc = pc or adj.pc_linear

    def rnd():
        f = P.zeros(3)
        f[:, :, s, n] = rng.standard_normal((3, P.n_r)) + 1j * rng.standard_normal((3, P.n_r))
        return f

    if form == "conv":
        # the convective term is quadratic: a central difference is its
        # exact derivative
        tlm = lambda du: (nl.nonlinear_conv(P, base + du) - nl.nonlinear_conv(P, base - du)) / 2.0
    else:
        tlm = lambda du: adj.nonlinear_tlm(P, base, du)
    x = [rnd(), rnd(), rnd()]
    logs = []
    for _ in range(steps):
        du, dup, dNp = x
        dN = tlm(du)
        y = [pc(P, 2.0 * dN - dNp, du, dup), du, dN]
        ny = np.sqrt(sum(np.vdot(v, v).real for v in y))
        nx = np.sqrt(sum(np.vdot(v, v).real for v in x))
        logs.append(np.log(ny / nx))
        x = [v / ny for v in y]
    return float(np.exp(np.mean(logs[steps // 2:])))


@pytest.mark.parametrize("dt", [1e-7, 5e-7])
def test_small_time_steps_are_stable(dt):
    P, mode = one_mode(dt, 0, 0)
    assert growth(P, mode) < 1.0 + 1e-5


def test_plain_gradient_correction_grows_at_small_dt():
    # the same probe catches the other reading of mode (0,0)'s correction
    P, mode = one_mode(1e-7, 0, 0)
    assert growth(P, mode, pc=pc_linear_plain_gradient) > 1.1


def test_rotational_form_time_step_limit():
    # the differentiation workload's dt lies below the rotational form's
    # limit; twice the paper-style step above it, mode (1, 0) grows
    P, mode = one_mode(5e-7, 1, 0)
    assert growth(P, mode) < 1.0 + 1e-5
    P, mode = one_mode(2e-6, 1, 0)
    assert growth(P, mode) > 1.1


@pytest.mark.parametrize("dt", [1e-7, 2e-6, 1e-5])
def test_convective_form_is_stable(dt):
    for a, b in ((0, 0), (1, 0), (0, 1)):
        P, mode = one_mode(dt, a, b)
        assert growth(P, mode, form="conv") < 1.0 + 1e-5, (a, b)
