"""Tangent-linear model and discrete adjoint of one projection step, and the
gradient of the final perturbation energy (not in the paper; the discrete
adjoint of the scheme of Sec. 3.2 as implemented in ``scheme``).

Inner product: <x, y> = sum Re(conj(x) y) over every stored coefficient, so
the adjoint of a complex-linear map is its conjugate transpose and a
real-linear map (the transforms, which drop Im of the n = 0 bin) is
transposed as a real map:

* to_spectral (forward transform, 1/P, truncation) has the adjoint
  g -> to_physical(w * g) / P with w = 1 at n = 0 and 1/2 at n > 0;
* to_physical (inverse transform) has the adjoint
  f -> P * c * to_spectral(f) with c = 1 at n = 0 and 2 at n > 0;
* the product N = omega x u linearises to d omega x u + omega x du, whose
  adjoint gives omega_bar = u x N_bar and u_bar = N_bar x omega.

A step maps (u^i, u^{i-1}, N^{i-1}) to (u^{i+1}, u^i, N^i); its adjoint maps
cotangents of the outputs to cotangents of the inputs.
"""
import numpy as np

from . import nonlinear as nl
from .scheme import div, grad, zero_nyquist, vector_laplacian_r, correction_gradient


# ---------------------------------------------------------------- helpers
def ddr_t(prob, f):
    """Apply D1^T along the radial axis."""
    return prob._band_apply(prob.D1.T.copy(), f)


def ddr2_t(prob, f):
    return prob._band_apply(prob.D2.T.copy(), f)


def _cn(prob):
    c = np.full(prob.m_theta, 2.0)
    c[0] = 1.0
    return c


def _area(prob):
    return prob.p_theta * prob.p_z


def div_adjoint(prob, f):
    """Conjugate transpose of div: f -> (v+, v-, v_z)."""
    a, b, r = prob.bcast()
    d = 0.5 * ddr_t(prob, f)
    return np.stack([d + f / (2.0 * r) + a * f / (2.0 * r), d + f / (2.0 * r) - a * f / (2.0 * r), -1j * b * f])


def grad_adjoint(prob, v):
    """Conjugate transpose of grad: (v+, v-, v_z) -> f."""
    a, b, r = prob.bcast()
    return ddr_t(prob, v[0] + v[1]) - a * v[0] / r + a * v[1] / r - 1j * b * v[2]


def vector_laplacian_r_adjoint(prob, w):
    """Adjoint of u -> V_r(u) = (L+ u+ + L- u-)/2 (u_z does not enter)."""
    a, b, r = prob.bcast()
    out = []
    for sgn in (1.0, -1.0):
        t = ddr2_t(prob, w) + ddr_t(prob, w / r) - (a * a / r ** 2 + b * b) * w
        out.append(0.5 * (t - (1.0 + sgn * 2.0 * a) / r ** 2 * w))
    return np.stack([out[0], out[1], np.zeros_like(w)])


# ---------------------------------------------------------------- nonlinear term
def nonlinear_tlm(prob, u, du):
    """dN = (curl du) x u + omega x du."""
    U = nl.to_physical(prob, np.stack(nl.cylindrical(u)))
    W = nl.to_physical(prob, np.stack(nl.vorticity(prob, u)))
    dU = nl.to_physical(prob, np.stack(nl.cylindrical(du)))
    dW = nl.to_physical(prob, np.stack(nl.vorticity(prob, du)))
    return nl._omega_cross_u(prob, U, dW) + nl._omega_cross_u(prob, dU, W)


def _cross(A, B):
    return np.stack([A[1] * B[2] - A[2] * B[1], A[2] * B[0] - A[0] * B[2], A[0] * B[1] - A[1] * B[0]])


def nonlinear_adjoint(prob, u, Nbar):
    """u_bar = (dN/du)^T N_bar for N = omega x u."""
    P = _area(prob)
    c = _cn(prob)
    U = nl.to_physical(prob, np.stack(nl.cylindrical(u)))
    W = nl.to_physical(prob, np.stack(nl.vorticity(prob, u)))
    # (N+, N-) = (N_r + i N_t, N_r - i N_t): conjugate transpose
    cyl_bar = np.stack([Nbar[0] + Nbar[1], -1j * (Nbar[0] - Nbar[1]), Nbar[2]])
    # adjoint of to_spectral: Hermitian weights, inverse transform, 1/P
    w = np.full(prob.m_theta, 0.5)
    w[0] = 1.0
    G = nl.to_physical(prob, cyl_bar * w) / P
    Wbar = _cross(U, G)    # omega_bar
    Ubar = _cross(G, W)    # u_bar (direct part)
    # adjoint of to_physical: P * c * forward transform
    ub = P * c * nl.to_spectral(prob, Ubar)
    wb = P * c * nl.to_spectral(prob, Wbar)
    # adjoint of the curl (omega from the cylindrical components)
    a, b, r = prob.bcast()
    ur_b, ut_b, uz_b = ub[0].copy(), ub[1].copy(), ub[2].copy()
    uz_b += -1j * a * wb[0] / r
    ut_b += 1j * b * wb[0]
    ur_b += -1j * b * wb[1]
    uz_b += -ddr_t(prob, wb[1])
    ut_b += ddr_t(prob, wb[2]) + wb[2] / r
    ur_b += 1j * a * wb[2] / r
    # adjoint of (u+, u-) -> (u_r, u_theta)
    out = np.stack([0.5 * ur_b + 0.5j * ut_b, 0.5 * ur_b - 0.5j * ut_b, uz_b])
    return zero_nyquist(prob, out)


# ---------------------------------------------------------------- predictor-corrector (linear part)
def _wall_mask(prob):
    m = np.zeros((prob.n_r, prob.m_z, prob.m_theta))
    m[0] = 1.0
    m[-1] = 1.0
    m[-1, 0, 0] = 0.0
    return m


def _interior_mask(prob):
    m = np.ones((prob.n_r, prob.m_z, prob.m_theta))
    m[0] = 0.0
    m[-1] = 0.0
    return m


def pc_linear(prob, Ne, u, up):
    """Linear part of steps 2-5 (boundary constants dropped): (Ne, u, u_prev) -> u^{i+1}."""
    I, Wm = _interior_mask(prob), _wall_mask(prob)
    rhs_p = -div(prob, Ne) * I + Wm * (-0.5 * (Ne[0] + Ne[1]) + vector_laplacian_r(prob, 2.0 * u - up))
    p = prob.solve("P", zero_nyquist(prob, rhs_p))
    rhs_u = (-(4.0 * u - up) / (2.0 * prob.dt) + Ne + grad(prob, p)) * I
    us = np.stack([prob.solve(k, zero_nyquist(prob, rhs_u[c])) for c, k in enumerate(("Up", "Um", "Uz"))])
    phi = prob.solve("P", zero_nyquist(prob, div(prob, us) * I))
    return zero_nyquist(prob, us - correction_gradient(prob, phi, us))


def pc_adjoint(prob, ubar_next):
    """Adjoint of pc_linear: u^{i+1}_bar -> (Ne_bar, u_bar, u_prev_bar)."""
    I, Wm = _interior_mask(prob), _wall_mask(prob)
    ub = zero_nyquist(prob, ubar_next.copy())
    # u^{i+1} = u* - grad phi, except mode (0,0): u^{i+1}+- = u*+- - u*_r
    us_b = ub.copy()
    g00 = ub[0, :, 0, 0] + ub[1, :, 0, 0]
    us_b[0, :, 0, 0] -= 0.5 * g00
    us_b[1, :, 0, 0] -= 0.5 * g00
    gb = ub.copy()
    gb[0, :, 0, 0] = 0.0
    gb[1, :, 0, 0] = 0.0
    phi_b = -grad_adjoint(prob, gb)
    # phi = P^-1 rhs_phi, rhs_phi = div(u*) on interior rows
    rphi_b = zero_nyquist(prob, prob.solve("P", zero_nyquist(prob, phi_b), trans=1))
    us_b = us_b + div_adjoint(prob, rphi_b * I)
    # u* = H^-1 rhs_u
    ru_b = np.stack([zero_nyquist(prob, prob.solve(k, zero_nyquist(prob, us_b[c]), trans=1))
                     for c, k in enumerate(("Up", "Um", "Uz"))]) * I
    # rhs_u = -(4u - u_prev)/(2dt) + Ne + grad p
    u_b = -4.0 / (2.0 * prob.dt) * ru_b
    up_b = 1.0 / (2.0 * prob.dt) * ru_b
    Ne_b = ru_b.copy()
    p_b = grad_adjoint(prob, ru_b)
    # p = P^-1 rhs_p
    rp_b = zero_nyquist(prob, prob.solve("P", zero_nyquist(prob, p_b), trans=1))
    # rhs_p = -div(Ne) (interior) ; -(Ne+ + Ne-)/2 + V_r(2u - u_prev) (walls)
    Ne_b = Ne_b - div_adjoint(prob, rp_b * I)
    wall = rp_b * Wm
    Ne_b[0] = Ne_b[0] - 0.5 * wall
    Ne_b[1] = Ne_b[1] - 0.5 * wall
    vb = vector_laplacian_r_adjoint(prob, wall)
    u_b = u_b + 2.0 * vb
    up_b = up_b - vb
    return zero_nyquist(prob, Ne_b), zero_nyquist(prob, u_b), zero_nyquist(prob, up_b)


# ---------------------------------------------------------------- whole step
def step_tlm(prob, u, du, dup, dNp):
    """Tangent of (u^{i+1}, u^i, N^i) at (u^i) for input tangents (du, du_prev, dN_prev)."""
    dN = nonlinear_tlm(prob, u, du)
    dun = pc_linear(prob, 2.0 * dN - dNp, du, dup)
    return dun, du.copy(), dN


def step_adjoint(prob, u, ubar_next, ubar_keep, Nbar):
    """Cotangents of (u^i, u^{i-1}, N^{i-1}) from those of (u^{i+1}, u^i, N^i)."""
    Ne_b, u_b, up_b = pc_adjoint(prob, ubar_next)
    N_b = 2.0 * Ne_b + Nbar
    u_b = u_b + ubar_keep + nonlinear_adjoint(prob, u, N_b)
    return zero_nyquist(prob, u_b), up_b, zero_nyquist(prob, -Ne_b)


# ---------------------------------------------------------------- objective and gradient
def perturbation_energy_gradient(prob, u):
    """Gradient of E_pert = 1/2 int |u - U_c|^2 (trapezoid in r, Parseval in theta, z)."""
    from .diagnostics import couette_state, trapezoid_weights
    area = (2.0 * np.pi / prob.k_theta) * (2.0 * np.pi / prob.k_z)
    w = trapezoid_weights(prob.r) * prob.r
    c = _cn(prob)
    d = u - couette_state(prob)
    scale = area * w[:, None, None] * c[None, None, :]
    g = np.stack([0.5 * scale * d[0], 0.5 * scale * d[1], scale * d[2]])
    return zero_nyquist(prob, g)


def gradient(prob, u0, nsteps, checkpoint_every=20):
    """J = E_pert(u^T) after nsteps from u^0 (history u^{-1} = u^0,
    N^{-1} = N(u^0)); returns (J, dJ/du^0) by checkpointed reverse sweep."""
    from .diagnostics import perturbation_energy
    from .scheme import step
    from .nonlinear import nonlinear_rot
    # forward, keeping (u^i, u^{i-1}, N^{i-1}) every checkpoint_every steps
    u, up, Np = u0.copy(), u0.copy(), nonlinear_rot(prob, u0)
    checkpoints = {}
    for i in range(nsteps):
        if i % checkpoint_every == 0:
            checkpoints[i] = (u.copy(), up.copy(), Np.copy())
        un, _, N = step(prob, u, up, Np)
        up, u, Np = u, un, N
    J = perturbation_energy(prob, u)
    ub = perturbation_energy_gradient(prob, u)
    upb = np.zeros_like(ub)
    Nb = np.zeros_like(ub)
    # reverse: segment by segment, recomputing the segment's states
    for seg in sorted(checkpoints, reverse=True):
        end = min(seg + checkpoint_every, nsteps)
        cu, cup, cNp = checkpoints[seg]
        states = [(cu, cup, cNp)]
        for _ in range(seg, end - 1):
            a, b, c = states[-1]
            an, _, N = step(prob, a, b, c)
            states.append((an, a, N))
        for k in range(end - seg - 1, -1, -1):
            su, sup, sNp = states[k]
            # output cotangents of step k: (u^{k+1}: ub, u^k: upb, N^k: Nb)
            ub, upb, Nb = step_adjoint(prob, su, ub, upb, Nb)
    # initial history: u^{-1} = u^0, N^{-1} = N(u^0)
    g = ub + upb + nonlinear_adjoint(prob, u0, Nb)
    return J, zero_nyquist(prob, g)


def inner(x, y):
    return float(np.sum((np.conj(x) * y).real))
