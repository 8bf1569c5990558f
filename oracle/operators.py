"""Mode-decoupled operators and their banded LU solves (Sec. 3.1-3.2).

Spectral layout shared by every function in the oracle (a complex array):

    field[j, s, n]   j = 0..M radial node, s = 0..m_z-1 axial slot,
                     n = 0..m_theta-1 azimuthal wavenumber (n >= 0 stored,
                     the field being real).

Axial slot s holds l = s for s < m_z/2 and l = s - m_z above; slot m_z/2
(l = -m_z/2) is kept zero.  Velocity is stored as (u+, u-, u_z) with
u+- = u_r +- i u_theta (Sec. 3.1, Orszag-Patera change of variables).

For a mode with a = n k_theta, b = l k_z and R = diag(r) the operators are
(eq. modalNS and eq. modalNSdecoup, whose coefficients of u+- carry
-(1 +- 2a)/r^2; the sign printed in the theta equation of eq. modalNS is
read as +, the only sign consistent with eq. NS_cyl and eq. modalNSdecoup):

    Lap  = D2 + R^-1 D1 - a^2 R^-2 - b^2
    L+-  = Lap - (1 +- 2a) R^-2
    H+-  = L+- - 3/(2 dt),  H_z = Lap - 3/(2 dt)   (eq. vel, BDF2 weight 3/2)
    P    = Lap                                    (eqs. pressure, correction)

Boundary rows: H+-, H_z take Dirichlet rows (identity rows at j = 0, M,
eq. nsBC); P takes Neumann rows (the D1 rows at j = 0, M), except mode
(0, 0) whose row M is the identity (Dirichlet zero at the outer cylinder,
Sec. 3.2, last paragraph).

The systems are banded (kl = ku = 4) and are factored once with LAPACK
DGBTRF and solved with DGBTRS, the routines Sec. 4 names.
"""
import numpy as np
from scipy.linalg import lapack

from .radial import nodes, fd_matrices, radii, HALF

KL = KU = HALF
KINDS = ("P", "Up", "Um", "Uz")


class Problem:
    """Grid, parameters and cached per-mode LU factors of one configuration."""

    def __init__(self, n_r, m_theta, m_z, eta, Re_i, Re_o, dt, k_theta=1.0, k_z=1.0,
                 alpha=0.0, p_theta=0, p_z=0, form="rot"):
        if m_z % 2:
            raise ValueError("m_z must be even")
        if form not in ("rot", "conv"):
            raise ValueError("form must be 'rot' (omega x u) or 'conv' (u.grad u)")
        # form of the nonlinear term the step uses: rotational omega x u, or
        # the paper's convective u.grad u (Sec. 3.2, step 1)
        self.form = form
        self.n_r, self.m_theta, self.m_z = n_r, m_theta, m_z
        self.M = n_r - 1
        self.p_theta = p_theta or 3 * m_theta
        self.p_z = p_z or 3 * m_z // 2
        self.eta, self.Re_i, self.Re_o, self.dt = eta, Re_i, Re_o, dt
        self.k_theta, self.k_z, self.alpha = k_theta, k_z, alpha
        self.r_i, self.r_o = radii(eta)
        self.r = nodes(n_r, eta, alpha)
        self.D1, self.D2 = fd_matrices(self.r)
        self.n = np.arange(m_theta)
        slots = np.arange(m_z)
        self.l = np.where(slots < m_z // 2, slots, slots - m_z)
        self.nyq = m_z // 2
        self.a = self.n * k_theta
        self.b = self.l * k_z
        self._lu = {}

    # ------------------------------------------------------------------ shapes
    def zeros(self, *lead):
        return np.zeros(lead + (self.n_r, self.m_z, self.m_theta), dtype=np.complex128)

    # ------------------------------------------------------------------ operators
    def operator(self, kind, n, labs):
        """Dense n_r x n_r matrix of operator ``kind`` for mode (|l|, n)."""
        a = n * self.k_theta
        b = labs * self.k_z
        r = self.r
        lap = self.D2 + self.D1 / r[:, None] - np.diag(a * a / r ** 2 + b * b)
        c = 1.5 / self.dt
        if kind == "P":
            A = lap.copy()
            A[0] = self.D1[0]
            A[-1] = self.D1[-1]
            if n == 0 and labs == 0:
                A[-1] = 0.0
                A[-1, -1] = 1.0
            return A
        if kind == "Up":
            A = lap - np.diag((1.0 + 2.0 * a) / r ** 2) - c * np.eye(self.n_r)
        elif kind == "Um":
            A = lap - np.diag((1.0 - 2.0 * a) / r ** 2) - c * np.eye(self.n_r)
        elif kind == "Uz":
            A = lap - c * np.eye(self.n_r)
        else:
            raise ValueError(kind)
        A[0] = 0.0
        A[0, 0] = 1.0
        A[-1] = 0.0
        A[-1, -1] = 1.0
        return A

    def _band(self, A):
        """LAPACK band storage with KL extra rows for the pivoting fill-in."""
        N = A.shape[0]
        ab = np.zeros((2 * KL + KU + 1, N))
        for j in range(N):
            lo, hi = max(0, j - KU), min(N - 1, j + KL)
            ab[KL + KU + np.arange(lo, hi + 1) - j, j] = A[lo:hi + 1, j]
        return ab

    def factor(self, kind, n, labs):
        key = (kind, n, labs)
        f = self._lu.get(key)
        if f is None:
            lu, piv, info = lapack.dgbtrf(self._band(self.operator(kind, n, labs)), KL, KU)
            if info != 0:
                raise np.linalg.LinAlgError(f"singular operator {key}: info={info}")
            f = (lu, piv)
            self._lu[key] = f
        return f

    def solve_mode(self, kind, n, labs, rhs, trans=0):
        """Solve A x = rhs (trans=1: A^T x = rhs); rhs real (n_r, k)."""
        lu, piv = self.factor(kind, n, labs)
        x, info = lapack.dgbtrs(lu, KL, KU, rhs, piv, trans=trans)
        if info != 0:
            raise np.linalg.LinAlgError(f"dgbtrs failed: {info}")
        return x

    def solve(self, kind, rhs, trans=0, modes=None):
        """Solve operator ``kind`` for every stored mode.

        ``rhs`` is a complex (n_r, m_z, m_theta) array whose rows 0 and M hold
        the boundary values.  The slots +l and -l share one factorisation,
        the operators depending on l only through l^2.  ``modes`` optionally
        restricts the work to a list of (|l|, n); other entries of the
        result are zero.
        """
        x = np.zeros_like(rhs)
        if modes is None:
            modes = [(labs, n) for labs in range(self.m_z // 2) for n in range(self.m_theta)]
        for labs, n in modes:
            slots = [labs] if labs == 0 else [labs, self.m_z - labs]
            cols = np.concatenate([np.stack([rhs[:, s, n].real, rhs[:, s, n].imag], 1)
                                   for s in slots], axis=1)
            sol = self.solve_mode(kind, n, labs, np.ascontiguousarray(cols), trans)
            for k, s in enumerate(slots):
                x[:, s, n] = sol[:, 2 * k] + 1j * sol[:, 2 * k + 1]
        return x

    # ------------------------------------------------------------------ radial helpers
    def _band_apply(self, A, f):
        """Apply a banded (kl = ku = 4) radial matrix along axis -3 of f."""
        n = self.n_r
        out = np.zeros(np.broadcast_shapes(f.shape), dtype=np.result_type(f, A))
        for off in range(-HALF, HALF + 1):
            rows = np.arange(max(0, -off), min(n, n - off))
            coef = A[rows, rows + off]
            out[..., rows, :, :] += coef[:, None, None] * f[..., rows + off, :, :]
        return out

    def ddr(self, f):
        """Apply D1 along the radial axis of a (..., n_r, m_z, m_theta) array."""
        return self._band_apply(self.D1, f)

    def ddr2(self, f):
        return self._band_apply(self.D2, f)

    def bcast(self):
        """a, b and r broadcast against a (n_r, m_z, m_theta) array."""
        return (self.a[None, None, :], self.b[None, :, None], self.r[:, None, None])
