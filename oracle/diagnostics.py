"""Diagnostics of a spectral state (energies, divergence, wall slip, CFL
bound, wall torque).

Volume integrals use trapezoid weights on the radial nodes and Parseval in
(theta, z): a real field's mean square over a (theta, z) plane is
sum_{l,n} c_n |f_ln|^2 with c_0 = 1 and c_n = 2 for n > 0 (the n < 0 half
is the complex conjugate of the stored one).
"""
import numpy as np

from .radial import couette_profile


def trapezoid_weights(r):
    w = np.zeros_like(r)
    h = np.diff(r)
    w[:-1] += h / 2.0
    w[1:] += h / 2.0
    return w


def plane_energy_density(prob, u):
    """Per-node sum_{l,n} c_n ((|u+|^2 + |u-|^2)/2 + |u_z|^2)/2 -> (n_r,)."""
    c = np.full(prob.m_theta, 2.0)
    c[0] = 1.0
    dens = 0.5 * (np.abs(u[0]) ** 2 + np.abs(u[1]) ** 2) + np.abs(u[2]) ** 2
    dens[:, prob.nyq, :] = 0.0
    return 0.5 * np.einsum("jsn,n->j", dens, c)


def energy(prob, u):
    """Kinetic energy 1/2 int |u|^2 r dr dtheta dz over the periodic box."""
    area = (2.0 * np.pi / prob.k_theta) * (2.0 * np.pi / prob.k_z)
    w = trapezoid_weights(prob.r)
    return area * np.sum(w * prob.r * plane_energy_density(prob, u))


def couette_state(prob):
    """Circular Couette flow in the stored layout: u+- = +-i U_theta at mode (0,0)."""
    u = prob.zeros(3)
    U = couette_profile(prob.r, prob.eta, prob.Re_i, prob.Re_o)
    u[0, :, 0, 0] = 1j * U
    u[1, :, 0, 0] = -1j * U
    return u


def perturbation_energy(prob, u):
    return energy(prob, u - couette_state(prob))


def wall_slip(prob, u, wall=0):
    """Tangential slip at a wall relative to Re: sqrt(<(u_theta - Re)^2 + u_z^2>).

    The integrand printed in Sec. 5.3 has (u_theta - Re_i)^2 - u_z^2 under
    the root; the minus sign is read as a plus (a norm of the tangential
    velocity error).
    """
    Re = prob.Re_i if wall == 0 else prob.Re_o
    j = 0 if wall == 0 else -1
    ut = -0.5j * (u[0, j] - u[1, j])
    uz = u[2, j].copy()
    ut = ut.copy()
    ut[0, 0] -= Re
    c = np.full(prob.m_theta, 2.0)
    c[0] = 1.0
    ut[prob.nyq] = 0.0
    uz[prob.nyq] = 0.0
    ms = np.sum(c * (np.abs(ut) ** 2 + np.abs(uz) ** 2))
    return np.sqrt(ms) / abs(Re)


def cfl_bound(prob, u):
    """Upper bound of the advective CFL number of a state,

        dt max_j max_(theta, z) ( |u_r|/dr_j + |u_theta|/(r_j dtheta) + |u_z|/dz ),

    on the radial nodes, with dr_j the distance from node j to its nearer
    neighbour and dtheta = 2 pi / (k_theta 2 m_theta), dz = 2 pi / (k_z m_z)
    the spacings of the physical grid (2 m_theta, m_z) that the stored modes
    resolve.  The maximum over a (theta, z) plane is replaced by its bound
    for a real field, max |f| <= sum_{l, n} c_n |f_ln| (c_0 = 1, c_n = 2:
    the n < 0 half is the conjugate of the stored one), taken per velocity
    component.  This is a diagnostic of the time step's explicit limit; the
    paper discusses that limit in Sec. 5.3 and 5.5 without a formula.
    """
    ur = 0.5 * (u[0] + u[1])
    ut = -0.5j * (u[0] - u[1])
    uz = u[2]
    c = np.full(prob.m_theta, 2.0)
    c[0] = 1.0

    def plane_bound(f):
        a = np.abs(f)
        a[:, prob.nyq, :] = 0.0
        return np.einsum("jsn,n->j", a, c)

    r = prob.r
    h = np.diff(r)
    dr = np.minimum(np.concatenate([h, [np.inf]]), np.concatenate([[np.inf], h]))
    dth = 2.0 * np.pi / (prob.k_theta * 2 * prob.m_theta)
    dz = 2.0 * np.pi / (prob.k_z * prob.m_z)
    rate = plane_bound(ur) / dr + plane_bound(ut) / (r * dth) + plane_bound(uz) / dz
    return prob.dt * float(np.max(rate))


def quasi_nusselt(prob, u):
    """Quasi-Nusselt number at the inner and outer cylinder (Sec. 5.5): the
    torque the fluid exerts on a cylinder divided by that of circular
    Couette flow at the same Reynolds numbers.

    On a cylinder the viscous torque is proportional to r^3 d<omega>/dr,
    with <omega> = <u_theta> / r the angular velocity averaged over theta and
    z, i.e. the (l, n) = (0, 0) coefficient of u_theta divided by r (u_r
    vanishes at the walls, so the convective part of the angular-velocity
    flux does not enter there).  For Couette flow <omega> = C1 + C2 / r^2
    and r^3 d<omega>/dr = -2 C2 on every radius, hence

        Nu_w = r^3 (D1 <omega>)(r) / (-2 C2)   at r = r_i and r = r_o,

    with D1 the finite-difference first derivative (its wall rows).
    Returns (Nu_inner, Nu_outer); NaN when C2 = 0 (no laminar torque).
    """
    eta, Re_i, Re_o = prob.eta, prob.Re_i, prob.Re_o
    C2 = eta * (Re_i - eta * Re_o) / ((1.0 - eta) * (1.0 - eta ** 2))
    if C2 == 0.0:
        return float("nan"), float("nan")
    ut_mean = (-0.5j * (u[0, :, 0, 0] - u[1, :, 0, 0])).real
    dw = prob.D1 @ (ut_mean / prob.r)
    r = prob.r
    return (float(r[0] ** 3 * dw[0] / (-2.0 * C2)), float(r[-1] ** 3 * dw[-1] / (-2.0 * C2)))
