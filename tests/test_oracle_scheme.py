"""Pins of the oracle's projection step (Sec. 3.2, steps 1-6)."""
import numpy as np
import pytest
from scipy import optimize, special

import oracle
import tc_inputs
from oracle import diagnostics as dg
from oracle import scheme
from conftest import paper_value


@pytest.mark.parametrize("alpha", [0.0, 0.5])
def test_couette_drift_falls_with_resolution(alpha):
    # circular Couette flow (Sec. 5.1) is an exact steady solution; the
    # discrete drift is FD error and falls at high order with n_r
    drift = []
    for n_r in (16, 32):
        P = oracle.Problem(n_r, 4, 8, 0.5, 50.0, 200.0, 1e-3, alpha=alpha)
        u = dg.couette_state(P)
        un, _, _, _ = scheme.run(P, u, 20)
        drift.append(np.linalg.norm(un - u) / np.linalg.norm(u))
    assert drift[1] < drift[0] / 2 ** 7 and drift[1] < 1e-9, drift


def test_discrete_couette_stays_steady():
    # the discrete steady profile (D2 + D1/r - 1/r^2) u_theta = 0 is kept to
    # rounding: the centrifugal force of mode (0,0) is balanced by the
    # pressure, and the correction leaves that mode no radial velocity
    drift = []
    for n_r in (32, 64):
        P = oracle.Problem(n_r, 4, 8, 0.5, 50.0, 200.0, 1e-3)
        A = P.D2 + P.D1 / P.r[:, None] - np.diag(1.0 / P.r ** 2)
        A[0] = np.eye(n_r)[0]
        A[-1] = np.eye(n_r)[-1]
        b = np.zeros(n_r)
        b[0], b[-1] = 50.0, 200.0
        U = np.linalg.solve(A, b)
        u = P.zeros(3)
        u[0, :, 0, 0] = 1j * U
        u[1, :, 0, 0] = -1j * U
        un, _, _, _ = scheme.run(P, u, 20)
        drift.append(np.linalg.norm(un - u) / np.linalg.norm(u))
    assert max(drift) < 1e-12, drift


def test_divergence_identity(small_problem):
    # u^{i+1} = u* - grad phi with P phi = div u*: at interior nodes
    # div u^{i+1} = (D2 - D1 D1) phi exactly (eqs. correction and update),
    # except mode (0,0), whose radial velocity the correction removes
    # entirely: its divergence is zero at every node
    P, cfg = small_problem
    u0 = tc_inputs.initial_state(P.r, cfg)
    N0 = oracle.nonlinear_rot(P, u0)
    un, p, N, d = scheme.step(P, u0, u0, N0, detail=True)
    lhs = scheme.div(P, un)[1:-1]
    rhs = np.tensordot(P.D2 - P.D1 @ P.D1, d["phi"], axes=(1, 0))[1:-1]
    rhs[:, 0, 0] = 0.0
    ustar_div = np.abs(scheme.div(P, d["u_star"])[1:-1]).max()
    assert np.abs(lhs - rhs).max() <= 1e-12 * ustar_div
    assert np.abs(lhs).max() < 1e-2 * ustar_div
    assert np.abs(un[0, :, 0, 0] + un[1, :, 0, 0]).max() == 0.0


def test_mode_00_correction_solves_its_equation_exactly(small_problem):
    # for mode (0,0), (1/r) d_r (r d_r phi) = (1/r) d_r (r u*_r) with
    # d_r phi = u*_r = 0 at both walls has the solution d_r phi = u*_r:
    # the correction leaves u_theta, u_z and every other mode as the plain
    # gradient of the discrete phi does
    P, cfg = small_problem
    u0 = tc_inputs.initial_state(P.r, cfg)
    N0 = oracle.nonlinear_rot(P, u0)
    un, p, N, d = scheme.step(P, u0, u0, N0, detail=True)
    plain = d["u_star"] - scheme.grad(P, d["phi"])
    plain[:, :, P.nyq] = 0.0
    mask = np.ones(un.shape, bool)
    mask[:2, :, 0, 0] = False
    assert np.array_equal(un[mask], plain[mask])
    ut = un[0, :, 0, 0] - un[1, :, 0, 0]
    assert np.array_equal(ut, d["u_star"][0, :, 0, 0] - d["u_star"][1, :, 0, 0])


def _bessel_case(eta):
    r_i, r_o = oracle.radii(eta)
    f = lambda k: special.j1(k * r_i) * special.y1(k * r_o) - special.j1(k * r_o) * special.y1(k * r_i)
    k = optimize.brentq(f, 0.5, 4.5)
    w = lambda r: special.j1(k * r) * special.y1(k * r_i) - special.j1(k * r_i) * special.y1(k * r)
    return k, w


def _bessel_error(dt, exact_history):
    # axisymmetric azimuthal flow U_c + w(r) exp(-k^2 t): its nonlinear term is
    # purely radial (absorbed by the pressure), so u_theta must decay exactly
    eta = 0.5
    k, w = _bessel_case(eta)
    P = oracle.Problem(48, 2, 4, eta, 50.0, 20.0, dt)

    def state(t):
        u = dg.couette_state(P)
        ww = w(P.r) * np.exp(-k * k * t)
        u[0, :, 0, 0] += 1j * ww
        u[1, :, 0, 0] -= 1j * ww
        return u

    n = int(round(0.02 / dt))
    u, _, _, _ = scheme.run(P, state(0.0), n, u_prev=state(-dt) if exact_history else None)
    return np.abs(u[0, :, 0, 0] - state(n * dt)[0, :, 0, 0]).max()


def test_bdf2_order_bessel_mode():
    e = np.array([_bessel_error(dt, True) for dt in (2e-3, 1e-3, 5e-4)])
    ratios = e[:-1] / e[1:]
    assert np.all(ratios > 3.7) and np.all(ratios < 4.3), ratios


def test_default_start_is_first_order():
    # u^{-1} = u^0 makes the first step backward Euler with step 2 dt / 3:
    # the global error is then first order in dt
    e = np.array([_bessel_error(dt, False) for dt in (2e-3, 1e-3)])
    assert 1.8 < e[0] / e[1] < 2.2


def test_wall_slip_falls_with_dt():
    # Sec. 5.3: the projection leaves a tangential slip that falls with dt
    # (paper: exponent about 2.5 until spatial error takes over)
    cfg = dict(tc_inputs.CONFIGS["small"])
    cfg.update(amp=0.05, m_theta=8, m_z=8)
    slip = []
    for dt in (4e-4, 2e-4, 1e-4):
        P = oracle.Problem(32, 8, 8, cfg["eta"], cfg["Re_i"], cfg["Re_o"], dt)
        u, _, _, _ = scheme.run(P, tc_inputs.initial_state(P.r, cfg), int(round(0.004 / dt)))
        slip.append(dg.wall_slip(P, u))
    slope = np.log2(slip[0] / slip[1])
    assert slip[2] < slip[1] < slip[0] and slip[0] < 1e-5
    assert 2.0 < slope < 4.0 and abs(slope - paper_value("slip_exponent")) < 1.0


def test_nonlinear_term_changes_the_step(small_problem):
    # N enters the step: dropping it changes u^{i+1} well above roundoff
    P, cfg = small_problem
    u0 = tc_inputs.initial_state(P.r, cfg)
    N0 = oracle.nonlinear_rot(P, u0)
    a, _, _ = scheme.step(P, u0, u0, N0)
    b, _, _ = scheme.step(P, u0, u0, 0 * N0, N=0 * N0)
    pert = u0 - dg.couette_state(P)
    assert np.linalg.norm(a - b) > 1e-3 * np.linalg.norm(pert)


def _noise_floor(P, u0, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    N0 = oracle.nonlinear_rot(P, u0)
    ref, _, _ = scheme.step(P, u0, u0, N0)
    jig = u0 * (1 + 2.2e-16 * rng.choice([-1.0, 1.0], size=u0.shape))
    alt, _, _ = scheme.step(P, jig, jig, oracle.nonlinear_rot(P, jig))
    return np.linalg.norm(alt - ref) / np.linalg.norm(ref)


def test_parity_noise_floor_small(small_problem):
    # one-ulp input noise moves one step by far less than the 1e-11 parity bar
    P, cfg = small_problem
    floor = _noise_floor(P, tc_inputs.initial_state(P.r, cfg), 9)
    assert floor < 1e-12, floor


@pytest.mark.slow
def test_parity_noise_floor_medium():
    cfg = tc_inputs.CONFIGS["medium"]
    P = oracle.Problem(cfg.n_r, cfg.m_theta, cfg.m_z, cfg.eta, cfg.Re_i, cfg.Re_o, cfg.dt)
    floor = _noise_floor(P, tc_inputs.initial_state(P.r, cfg), 10)
    assert floor < 1e-11, floor


def test_axisymmetric_onset_brackets_textbook_value():
    # Linear onset of Taylor vortices for eta = 0.5, outer cylinder at rest:
    # Re_c = 68.19 at axial wavenumber 3.163 (standard linear-stability
    # result).  Growth rate of a small (l=1, n=0) disturbance changes sign
    # between Re_i = 64 and Re_i = 72.
    rates = []
    for Re in (64.0, 72.0):
        P = oracle.Problem(24, 1, 4, 0.5, Re, 0.0, 2e-3, k_z=3.163)
        u = dg.couette_state(P)
        x = P.r - P.r_i
        prof = x ** 2 * (1 - x) ** 2
        u[0, :, 1, 0] = 1e-6 * prof
        u[1, :, 1, 0] = 1e-6 * prof
        u[0, :, 3, 0] = 1e-6 * prof
        u[1, :, 3, 0] = 1e-6 * prof
        E = []
        up, Np = u.copy(), oracle.nonlinear_rot(P, u)
        for i in range(400):
            un, _, N = scheme.step(P, u, up, Np)
            up, u, Np = u, un, N
            if i >= 200 and i % 50 == 0:
                # energy of the disturbed modes (slots l = +-1) alone
                d = u.copy()
                d[:, :, 0] = 0.0
                E.append(dg.energy(P, d))
        rates.append(np.polyfit(np.arange(len(E)) * 50 * P.dt, np.log(E), 1)[0])
    assert rates[0] < 0 < rates[1], rates


def test_one_mode_problem_reproduces_full_step():
    # the production-size step test checks sampled modes with one-mode
    # problems (grid m_theta = 2, m_z = 4, wavenumbers rescaled so that a
    # stored slot carries the mode's a and b); on a small grid they must
    # give exactly what the full predictor-corrector gives, mode by mode
    from test_gpu_production import _mode_problem
    P = oracle.Problem(24, 6, 10, 0.6, 80.0, -20.0, 1e-3, k_theta=1.5, k_z=0.8)
    sh = (3, P.n_r, P.m_z, P.m_theta)
    u, up, N, Np = (tc_inputs.random_state(sh, s) for s in (1, 2, 3, 4))
    ref_u, ref_p = scheme.predictor_corrector(P, N, Np, u, up)
    T = oracle.Problem(24, 2, 4, 0.6, 80.0, -20.0, 1e-3)
    for labs in range(P.m_z // 2):
        for n in range(P.m_theta):
            slots = [labs] if labs == 0 else [labs, P.m_z - labs]
            Q, nq, sq = _mode_problem(T, labs, n, P.k_theta, P.k_z)
            ins = [Q.zeros(3) for _ in range(4)]
            for src, dst in zip((u, up, N, Np), ins):
                for m, s in enumerate(slots):
                    dst[:, :, sq[m], nq] = src[:, :, s, n]
            un, pn = scheme.predictor_corrector(Q, ins[2], ins[3], ins[0], ins[1])
            assert np.array_equal(un[:, :, sq, nq], ref_u[:, :, slots, n])
            assert np.array_equal(pn[:, sq, nq], ref_p[:, slots, n])
