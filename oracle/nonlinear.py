"""Nonlinear term by the pseudospectral method with 3/2 dealiasing (Sec. 3.2, step 1).

The velocity and the fields the product needs are evaluated in spectral
space (radial derivatives with the FD matrix D1, azimuthal and axial ones by
multiplication with i a, i b), transformed to a (P_z, P_theta) physical
grid at each radial node, multiplied point by point, transformed back and
truncated to the stored modes.  With P >= 3 K + 1 for the largest stored
wavenumber K the retained coefficients of the quadratic products are free
of aliasing (Sec. 3.1, last paragraph).

Transform convention (eq. fourier): the inverse transform is the plain sum
over modes (no scaling); the forward transform carries 1/(P_theta P_z).
The azimuthal transform is real-to-complex on n >= 0; as in any c2r
transform the imaginary part of the n = 0 bin is discarded.

``nonlinear_rot`` evaluates N = omega x u (rotational form; the pressure
variable is then p + |u|^2/2).  ``nonlinear_conv`` evaluates the paper's own
convective form u.grad u with the curvature terms of eq. NS_cyl.
"""
import numpy as np
import scipy.fft as sfft

WORKERS = 8


def _pad(prob, f):
    """(..., m_z, m_theta) stored modes -> (..., P_z, P_theta/2+1) zero padded."""
    h = prob.m_z // 2
    out = np.zeros(f.shape[:-2] + (prob.p_z, prob.p_theta // 2 + 1), dtype=np.complex128)
    out[..., :h, :prob.m_theta] = f[..., :h, :]
    out[..., prob.p_z - (h - 1):, :prob.m_theta] = f[..., h + 1:, :]
    return out


def _truncate(prob, g):
    h = prob.m_z // 2
    out = np.zeros(g.shape[:-2] + (prob.m_z, prob.m_theta), dtype=np.complex128)
    out[..., :h, :] = g[..., :h, :prob.m_theta]
    out[..., h + 1:, :] = g[..., prob.p_z - (h - 1):, :prob.m_theta]
    return out


def to_physical(prob, f):
    """Unnormalised inverse transform of stored coefficients -> real grid values."""
    return sfft.irfft2(_pad(prob, f), s=(prob.p_z, prob.p_theta), axes=(-2, -1),
                       norm="forward", workers=WORKERS)


def to_spectral(prob, g):
    """Forward transform (scaled by 1/(P_theta P_z)) truncated to the stored modes."""
    return _truncate(prob, sfft.rfft2(g, axes=(-2, -1), norm="forward", workers=WORKERS))


def cylindrical(u):
    """(u+, u-, u_z) -> (u_r, u_theta, u_z)."""
    up, um, uz = u
    return (up + um) / 2.0, -0.5j * (up - um), uz


def plus_minus(vr, vt, vz):
    return np.stack([vr + 1j * vt, vr - 1j * vt, vz])


def _curl(prob, r, ur, ut, uz, d_ut, d_uz):
    """omega from the cylindrical components and their radial derivatives."""
    a = prob.a[None, :]
    b = prob.b[:, None]
    wr = 1j * a * uz / r - 1j * b * ut
    wt = 1j * b * ur - d_uz
    wz = d_ut + ut / r - 1j * a * ur / r
    return wr, wt, wz


def vorticity(prob, u):
    """omega = curl u in cylindrical components, spectral in (theta, z), FD in r."""
    ur, ut, uz = cylindrical(u)
    r = prob.r[:, None, None]
    return _curl(prob, r, ur, ut, uz, prob.ddr(ut), prob.ddr(uz))


def _omega_cross_u(prob, U, W):
    Nr = W[1] * U[2] - W[2] * U[1]
    Nt = W[2] * U[0] - W[0] * U[2]
    Nz = W[0] * U[1] - W[1] * U[0]
    return plus_minus(*to_spectral(prob, np.stack([Nr, Nt, Nz])))


def nonlinear_rot(prob, u):
    """N = omega x u; returns (N+, N-, N_z) in the stored layout."""
    ur, ut, uz = cylindrical(u)
    wr, wt, wz = vorticity(prob, u)
    U = to_physical(prob, np.stack([ur, ut, uz]))
    W = to_physical(prob, np.stack([wr, wt, wz]))
    return _omega_cross_u(prob, U, W)


def nonlinear_rot_at(prob, window, j):
    """N = omega x u at radial node j only.

    ``window`` holds the velocity at nodes max(0, j-4) .. min(M, j+4) (the
    support of FD row j), shape (3, rows, m_z, m_theta).
    """
    lo = max(0, j - 4)
    ur, ut, uz = cylindrical(window)
    w = prob.D1[j, lo:lo + window.shape[1]]
    d_ut = np.tensordot(w, ut, axes=(0, 0))
    d_uz = np.tensordot(w, uz, axes=(0, 0))
    k = j - lo
    wr, wt, wz = _curl(prob, prob.r[j], ur[k], ut[k], uz[k], d_ut, d_uz)
    U = to_physical(prob, np.stack([ur[k], ut[k], uz[k]]))
    W = to_physical(prob, np.stack([wr, wt, wz]))
    return _omega_cross_u(prob, U, W)


def nonlinear_conv(prob, u):
    """N = u.grad u with the curvature terms -u_theta^2/r, +u_theta u_r/r (eq. NS_cyl)."""
    comps = cylindrical(u)
    a, b, r = prob.bcast()
    U = to_physical(prob, np.stack(comps))
    rr = prob.r[:, None, None]
    out = []
    for c in comps:
        grads = np.stack([prob.ddr(c), 1j * a * c / r, 1j * b * c])
        G = to_physical(prob, grads)
        out.append(U[0] * G[0] + U[1] * G[1] + U[2] * G[2])
    out[0] = out[0] - U[1] * U[1] / rr
    out[1] = out[1] + U[1] * U[0] / rr
    S = to_spectral(prob, np.stack(out))
    return plus_minus(*S)


def kinetic_density(prob, u):
    """Coefficients of |u|^2 / 2 (dealiased), the Bernoulli term of the rotational form."""
    U = to_physical(prob, np.stack(cylindrical(u)))
    return to_spectral(prob, 0.5 * (U[0] ** 2 + U[1] ** 2 + U[2] ** 2))


def nonlinear_term(prob, u):
    """The nonlinear term in the problem's form (prob.form)."""
    return nonlinear_conv(prob, u) if prob.form == "conv" else nonlinear_rot(prob, u)
