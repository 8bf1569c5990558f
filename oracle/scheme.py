"""AB2BD2 fractional-step projection scheme (Sec. 3.2, steps 1-6).

One step maps (u^i, u^{i-1}, N^{i-1}) to (u^{i+1}, p^{i+1}, N^i):

1. N^i = N(u^i) pseudospectrally, in the problem's form: omega x u (the
   pressure variable is then p + |u|^2/2) or the paper's u.grad u;
   Ne = 2 N^i - N^{i-1} (eq. timeScheme).
2. Pressure predictor (eq. pressure): P p* = -div(Ne) inside, with the
   consistent Neumann rows of eq. ppBC at both walls.  Discretely the wall
   rows read  d_r p* = -Ne_r + (2 V_r(u^i) - V_r(u^{i-1})),  where V_r is the
   r-component of the vector Laplacian and d_t u_r = 0 at a wall (u_r is
   held at zero there); the Laplacian term is extrapolated to i+1 like the
   nonlinear term.  Mode (0,0): the outer row is p* = 0 (Sec. 3.2).
3. Velocity predictor (eq. vel): three Helmholtz problems
   H u* = -(4 u^i - u^{i-1})/(2 dt) + Ne + grad p*, Dirichlet rows from
   eq. nsBC (u_theta = Re_i, Re_o; u_r = u_z = 0), i.e. u+- = +-i Re at the
   walls of mode (0,0) and zero for every other mode.
4. Correction (eq. correction): P phi = div(u*), homogeneous Neumann rows;
   phi uses the same operator P as the pressure (mode (0,0) again takes
   phi = 0 at the outer wall).
5. Update (eq. update): p^{i+1} = p* + 3 phi/(2 dt), u^{i+1} = u* - grad phi,
   applied at every node.  For mode (0,0) the radial part of grad phi is
   d_r phi = u*_r, the exact solution of eq. correction for that mode
   ((1/r) d_r (r d_r phi) = (1/r) d_r (r u*_r) with d_r phi = 0 = u*_r at
   both walls), so its radial velocity is removed entirely; the Dirichlet
   row only fixes phi's constant, which enters the pressure alone.  (Taking
   d_r phi from the discrete solve instead leaves this mode a projection
   that is not idempotent, and it grows for small dt.)
6. History shift.

The first step starts from u^{-1} = u^0 and N^{-1} = N(u^0).

In the (u+, u-, u_z) variables (Sec. 3.1):
   (grad f)+- = D1 f -+ a f / r,        (grad f)_z = i b f,
   div v      = D1 v_r + v_r / r + a (v+ - v-)/(2 r) + i b v_z,
                with v_r = (v+ + v-)/2.
"""
import numpy as np

from .nonlinear import nonlinear_term


def grad(prob, f):
    a, b, r = prob.bcast()
    d = prob.ddr(f)
    return np.stack([d - a * f / r, d + a * f / r, 1j * b * f])


def div(prob, v):
    a, b, r = prob.bcast()
    vr = 0.5 * (v[0] + v[1])
    return prob.ddr(vr) + vr / r + a * (v[0] - v[1]) / (2.0 * r) + 1j * b * v[2]


def vector_laplacian_r(prob, u):
    """r-component of the vector Laplacian, 1/2 (L+ u+ + L- u-)."""
    a, b, r = prob.bcast()
    out = []
    for sgn, f in ((1.0, u[0]), (-1.0, u[1])):
        lap = prob.ddr2(f) + prob.ddr(f) / r - (a * a / r ** 2 + b * b) * f
        out.append(lap - (1.0 + sgn * 2.0 * a) / r ** 2 * f)
    return 0.5 * (out[0] + out[1])


def correction_gradient(prob, phi, u_star):
    """grad phi of eq. update, with mode (0,0) taking d_r phi = u*_r."""
    g = grad(prob, phi)
    ur = 0.5 * (u_star[0, :, 0, 0] + u_star[1, :, 0, 0])
    g[0, :, 0, 0] = ur
    g[1, :, 0, 0] = ur
    return g


def zero_nyquist(prob, f):
    f[..., prob.nyq, :] = 0.0
    return f


def pressure_rhs(prob, Ne, u, u_prev):
    rhs = -div(prob, Ne)
    wall = -0.5 * (Ne[0] + Ne[1]) + 2.0 * vector_laplacian_r(prob, u) - vector_laplacian_r(prob, u_prev)
    rhs[0] = wall[0]
    rhs[-1] = wall[-1]
    rhs[-1, 0, 0] = 0.0
    return zero_nyquist(prob, rhs)


def velocity_rhs(prob, Ne, u, u_prev, p_star):
    rhs = -(4.0 * u - u_prev) / (2.0 * prob.dt) + Ne + grad(prob, p_star)
    rhs[:, 0] = 0.0
    rhs[:, -1] = 0.0
    rhs[0, 0, 0, 0] = 1j * prob.Re_i
    rhs[1, 0, 0, 0] = -1j * prob.Re_i
    rhs[0, -1, 0, 0] = 1j * prob.Re_o
    rhs[1, -1, 0, 0] = -1j * prob.Re_o
    return zero_nyquist(prob, rhs)


def correction_rhs(prob, u_star):
    rhs = div(prob, u_star)
    rhs[0] = 0.0
    rhs[-1] = 0.0
    return zero_nyquist(prob, rhs)


def predictor_corrector(prob, N, N_prev, u, u_prev, detail=False):
    """Steps 2-5 for given N^i: returns (u^{i+1}, p^{i+1})."""
    Ne = 2.0 * N - N_prev
    rhs_p = pressure_rhs(prob, Ne, u, u_prev)
    p_star = prob.solve("P", rhs_p)
    rhs_u = velocity_rhs(prob, Ne, u, u_prev, p_star)
    u_star = np.stack([prob.solve(k, rhs_u[c]) for c, k in enumerate(("Up", "Um", "Uz"))])
    rhs_phi = correction_rhs(prob, u_star)
    phi = prob.solve("P", rhs_phi)
    p_next = zero_nyquist(prob, p_star + 1.5 * phi / prob.dt)
    u_next = zero_nyquist(prob, u_star - correction_gradient(prob, phi, u_star))
    if detail:
        return u_next, p_next, dict(p_star=p_star, u_star=u_star, phi=phi, rhs_phi=rhs_phi)
    return u_next, p_next


def step(prob, u, u_prev, N_prev, N=None, detail=False):
    """One projection step.  Returns (u_next, p_next, N) (+ intermediates if detail)."""
    if N is None:
        N = nonlinear_term(prob, u)
    out = predictor_corrector(prob, N, N_prev, u, u_prev, detail=detail)
    if detail:
        return out[0], out[1], N, out[2]
    return out[0], out[1], N


def run(prob, u0, nsteps, u_prev=None, N_prev=None):
    """nsteps steps from u0 (history defaults to u^{-1} = u^0, N^{-1} = N(u^0))."""
    u = u0.copy()
    up = u.copy() if u_prev is None else u_prev.copy()
    Np = nonlinear_term(prob, up) if N_prev is None else N_prev.copy()
    p = None
    for _ in range(nsteps):
        un, p, N = step(prob, u, up, Np)
        up, u, Np = u, un, N
    return u, up, Np, p
