"""Nonlinear optimal perturbation: ascent of the final perturbation energy
on a sphere of fixed initial perturbation energy (not in the paper's method;
the paper's quasi-Keplerian run of Sec. 5.5 starts from such a state, taken
from elsewhere).

Control.  The initial perturbation is the curl of a vector potential with
smooth radial profiles, the same family the synthetic inputs use:

    A_c(r; l, n) = g(r) sum_{q=0..3} a_{c,q,l,n} T_q(xi),
    g = 16 (r - r_i)^2 (r_o - r)^2,  xi = 2 (r - r_i) - 1,
    u' = curl A:  u_r = i a A_z / r - i b A_theta,
                  u_theta = i b A_r - d_r A_z,
                  u_z = d_r A_theta + A_theta / r - i a A_r / r,

with a = n k_theta, b = l k_z, radial derivatives taken exactly from the
polynomials.  u' vanishes at both walls and is divergence-free in the
continuum.  The coefficients a[c, q, slot, n] (complex) are the control;
mode (0,0) and the empty axial slot are not used, and the n = 0 column obeys
a(-l) = conj(a(l)) so that u' is real.  A control of low radial degree has no
unresolved near-wall directions, which make the ascent in the velocity
coefficients themselves ill-posed on the clustered grid.

Inner products: sum Re(conj(x) y) over the stored coefficients, in both
spaces.  The control gradient of a function of u' is then B^H applied to
its velocity gradient, projected on the Hermitian-consistent controls.

Ascent (projected gradient with rescaling, one iteration):
    G_J = grad_a J,  G_E = grad_a E0(a),
    p = G_J - (<G_J, G_E> / <G_E, G_E>) G_E         (tangent to the sphere)
    a <- a + tau p,  then a <- a sqrt(E0 / E(a))     (E is quadratic in a)
tau halves whenever J would decrease.
"""
import numpy as np

from .adjoint import gradient, perturbation_energy_gradient, inner
from .diagnostics import couette_state, perturbation_energy


def _basis(prob):
    """g T_q and its r-derivative at the nodes, shape (n_r, 4) each."""
    r = prob.r
    r_i, r_o = prob.r_i, prob.r_o
    xi = 2.0 * (r - r_i) - 1.0
    dxi = 2.0
    T = np.stack([np.ones_like(xi), xi, 2.0 * xi ** 2 - 1.0, 4.0 * xi ** 3 - 3.0 * xi], axis=1)
    dT = np.stack([np.zeros_like(xi), np.ones_like(xi), 4.0 * xi, 12.0 * xi ** 2 - 3.0], axis=1) * dxi
    g = 16.0 * (r - r_i) ** 2 * (r_o - r) ** 2
    dg = 32.0 * (r - r_i) * (r_o - r) ** 2 - 32.0 * (r - r_i) ** 2 * (r_o - r)
    return g[:, None] * T, dg[:, None] * T + g[:, None] * dT


def control_shape(prob):
    return (3, 4, prob.m_z, prob.m_theta)


def control_mask(prob):
    """1 on the control coefficients in use (not mode (0,0), not the empty slot)."""
    m = np.ones(control_shape(prob))
    m[:, :, 0, 0] = 0.0
    m[:, :, prob.nyq, :] = 0.0
    return m


def hermitian_projection(prob, x):
    """Orthogonal projection on controls with x(-l, 0) = conj(x(l, 0))."""
    y = x * control_mask(prob)
    h = prob.m_z // 2
    lpos = np.arange(1, h)
    lneg = prob.m_z - lpos
    avg = 0.5 * (y[:, :, lpos, 0] + np.conj(y[:, :, lneg, 0]))
    y[:, :, lpos, 0] = avg
    y[:, :, lneg, 0] = np.conj(avg)
    return y


def velocity(prob, a):
    """u' = B a in the stored layout (u+, u-, u_z)."""
    Bq, dBq = _basis(prob)
    a = a * control_mask(prob)
    A = np.einsum("jq,cqsn->cjsn", Bq, a)
    dA = np.einsum("jq,cqsn->cjsn", dBq, a)
    an, bl, r = prob.bcast()
    ur = 1j * an * A[2] / r - 1j * bl * A[1]
    ut = 1j * bl * A[0] - dA[2]
    uz = dA[1] + A[1] / r - 1j * an * A[0] / r
    u = np.stack([ur + 1j * ut, ur - 1j * ut, uz])
    u[:, :, prob.nyq] = 0.0
    return u


def control_gradient(prob, g):
    """Gradient in the control from a velocity gradient g: the Hermitian
    projection of B^H g."""
    Bq, dBq = _basis(prob)
    an, bl, r = prob.bcast()
    gr = g[0] + g[1]
    gt = -1j * (g[0] - g[1])
    gz = g[2]
    # cotangents of A_c and d_r A_c (conjugate transposes of the curl)
    GA = np.stack([-1j * bl * gt + 1j * an * gz / r, 1j * bl * gr + gz / r, -1j * an * gr / r])
    GdA = np.stack([np.zeros_like(gz), gz, -gt])
    G = np.einsum("jq,cjsn->cqsn", Bq, GA) + np.einsum("jq,cjsn->cqsn", dBq, GdA)
    return hermitian_projection(prob, G)


def control_energy(prob, a):
    """Initial perturbation energy E0(a) = E_pert(U_c + B a)."""
    return perturbation_energy(prob, couette_state(prob) + velocity(prob, a))


def objective_and_gradient(prob, a, nsteps, checkpoint_every=20):
    """J(a) = E_pert(u^T) from u^0 = U_c + B a and its control gradient."""
    u0 = couette_state(prob) + velocity(prob, a)
    J, g = gradient(prob, u0, nsteps, checkpoint_every)
    return J, control_gradient(prob, g)


def ascent(prob, a0, E0, nsteps, iters, tau=None, checkpoint_every=20):
    """Projected gradient ascent of J on {E0(a) = E0}; returns (a, [J per iterate])."""
    a = hermitian_projection(prob, a0)
    a = a * np.sqrt(E0 / control_energy(prob, a))
    J, G = objective_and_gradient(prob, a, nsteps, checkpoint_every)
    history = [J]
    for _ in range(iters):
        u0 = couette_state(prob) + velocity(prob, a)
        GE = control_gradient(prob, perturbation_energy_gradient(prob, u0))
        p = G - (inner(G, GE) / inner(GE, GE)) * GE
        if tau is None:
            tau = 0.1 * np.sqrt(inner(a, a) / inner(p, p))
        while True:
            b = a + tau * p
            b = b * np.sqrt(E0 / control_energy(prob, b))
            Jb, Gb = objective_and_gradient(prob, b, nsteps, checkpoint_every)
            if Jb >= J or tau < 1e-12:
                break
            tau *= 0.5
        a, J, G = b, Jb, Gb
        history.append(J)
    return a, history
