"""Degenerate and extreme grids against the oracle, and the out-of-memory path.

* smallest grid: n_r = 9 (one full 9-point stencil), a single azimuthal mode
  (axisymmetric) and a single axial mode pair (m_z = 2: l = 0 and the empty
  slot), on the shortest supported transforms (16 x 16);
* tallest radial grid the library accepts (n_r = 4096) with few modes;
* the zero state, whose nonlinear term and step must be exactly zero;
* a grid too large for the device: tc_init must fail with TC_ENOMEM and
  leave the device usable;
* default dealiased grids, the curl fused into the last sweep on large
  grids, and the wall torque where circular Couette flow exerts none.
"""
import numpy as np
import pytest

import oracle
import tc_inputs
from oracle import scheme
from gpu_common import rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu


def _pair(n_r, m_theta, m_z, p_theta=16, p_z=16, Re_i=50.0, Re_o=10.0, dt=1e-3):
    from paper_1311_2481_amd import Solver
    args = (n_r, m_theta, m_z, 0.5, Re_i, Re_o, dt)
    S = Solver(*args, p_theta=p_theta, p_z=p_z)
    P = oracle.Problem(*args, p_theta=p_theta, p_z=p_z)
    return S, P


def _jittered(P, seed):
    """The same problem on nodes moved by independent one-ulp perturbations
    (walls fixed), with its FD weights rebuilt: the two sides round the node
    formula independently, and next to clustered walls a one-ulp move of a
    node is ~1e-9 of the local spacing, so this distance is the rounding
    floor of a result."""
    from oracle.radial import fd_matrices
    rng = np.random.Generator(np.random.PCG64(seed))
    Q = oracle.Problem(P.n_r, P.m_theta, P.m_z, P.eta, P.Re_i, P.Re_o, P.dt, p_theta=P.p_theta, p_z=P.p_z)
    r = P.r.copy()
    r[1:-1] *= 1.0 + 1.1e-16 * rng.choice([-1.0, 1.0], size=P.n_r - 2)
    Q.r = r
    Q.D1, Q.D2 = fd_matrices(r)
    return Q


@pytest.mark.parametrize("n_r,m_theta,m_z", [(9, 1, 2), (9, 2, 4), (4096, 3, 4)])
def test_extreme_grids_step(n_r, m_theta, m_z):
    S, P = _pair(n_r, m_theta, m_z)
    shape = (3, n_r, m_z, m_theta)
    u = tc_inputs.random_state(shape, n_r + m_theta)
    up = tc_inputs.random_state(shape, n_r + m_theta + 1)
    N = to_host(S.nonlinear(to_dev(u)))
    ref_N = oracle.nonlinear_rot(P, u)
    eN = rel_l2(N, ref_N)
    Np = oracle.nonlinear_rot(P, up)
    S.set_state(to_dev(u), to_dev(up), to_dev(Np))
    S.step(1)
    got, p = S.get_state()
    ref_u, ref_p, _ = scheme.step(P, u, up, Np)
    eu, ep = rel_l2(to_host(got), ref_u), rel_l2(to_host(p), ref_p)
    # rounding floor: unstructured radial data meets D1 weights of order
    # 1/h_min near the clustered walls (h_min ~ 3e-7 at n_r = 4096), and the
    # correction phi of unstructured input is as large as u itself
    Q = _jittered(P, 11)
    fN = rel_l2(oracle.nonlinear_rot(Q, u), ref_N)
    qu, qp, _ = scheme.step(Q, u, up, Np)
    fu, fp = rel_l2(qu, ref_u), rel_l2(qp, ref_p)
    print(f"n_r={n_r} m_theta={m_theta} m_z={m_z}: nonlinear {eN:.2e} (floor {fN:.1e}), "
          f"step u {eu:.2e} (floor {fu:.1e}), p {ep:.2e} (floor {fp:.1e})")
    assert eN < max(1e-12, 10 * fN)
    assert eu < max(1e-10, 10 * fu) and ep < max(1e-9, 10 * fp)
    # the empty axial slot stays zero
    assert np.all(to_host(got)[:, :, m_z // 2] == 0)
    S.close()


def test_zero_state_is_a_fixed_point():
    # with both cylinders at rest the zero flow is a solution of the discrete
    # step: the nonlinear term and every right-hand side vanish exactly
    S, P = _pair(16, 4, 8, Re_i=0.0, Re_o=0.0)
    z = S.zeros(3)
    assert to_host(S.nonlinear(z)).any() == False  # noqa: E712
    S.set_state(z)
    S.step(3)
    u, p = S.get_state()
    assert not to_host(u).any() and not to_host(p).any()
    S.close()


def test_step_zero_and_history_defaults():
    # tc_step(0) changes nothing; u_prev = NULL means u_prev = u, N_prev =
    # NULL means N(u_prev)
    S, P = _pair(12, 3, 6)
    u = tc_inputs.random_state((3, 12, 6, 3), 77)
    S.set_state(to_dev(u))
    S.step(0)
    assert np.array_equal(to_host(S.get_state(with_pressure=False)), u)
    up, Np = S.get_history()
    assert np.array_equal(to_host(up), u)
    assert rel_l2(to_host(Np), oracle.nonlinear_rot(P, u)) < 1e-12
    S.close()


def test_out_of_memory_is_reported_and_recoverable():
    from paper_1311_2481_amd import Solver, TcError
    # one field of this grid is 61 GB; the state alone needs 16 of them
    with pytest.raises(TcError) as err:
        Solver(4096, 683, 1366, 0.5, 100.0, 0.0, 1e-4, p_theta=2048, p_z=2048)
    assert "ENOMEM" in str(err.value)
    # the device is still usable afterwards
    S, P = _pair(9, 1, 2)
    u = tc_inputs.random_state((3, 9, 2, 1), 3)
    assert rel_l2(to_host(S.nonlinear(to_dev(u))), oracle.nonlinear_rot(P, u)) < 1e-12
    S.close()


def test_default_dealiased_grid_rounds_up():
    # p_theta = p_z = 0 picks the smallest supported lengths that meet the
    # 3/2 rule: m_theta = 24 needs 70 -> 80, m_z = 40 needs 58 -> 64; the
    # result must equal the oracle's on that grid (any grid meeting the rule
    # gives the same truncated product, up to rounding)
    from paper_1311_2481_amd import Solver
    args = (12, 24, 40, 0.6, 70.0, -10.0, 1e-3)
    S = Solver(*args)
    P = oracle.Problem(*args, p_theta=80, p_z=64)
    u = tc_inputs.random_state((3, 12, 40, 24), 5)
    err = rel_l2(to_host(S.nonlinear(to_dev(u))), oracle.nonlinear_rot(P, u))
    print(f"default grid: nonlinear rel_l2 {err:.2e}")
    assert err < 1e-12
    S.close()


def test_fused_curl_matches_standalone():
    # On large grids (at least 2048 waves of predictor-corrector lanes) the
    # last sweep of a step also forms the curl of the new velocity, and the
    # next step skips its curl kernel.  Two steps in one call (the second
    # using that curl) must equal one step, a reload of the state (which
    # discards it) and one more step (which computes the curl on its own).
    from paper_1311_2481_amd import Solver
    n_r, m_theta, m_z = 16, 128, 1040      # 128 * 520 distinct modes -> 2080 waves
    args = (n_r, m_theta, m_z, 0.6, 300.0, -50.0, 1e-4)
    cfg = tc_inputs.Config(n_r=n_r, m_theta=m_theta, m_z=m_z, eta=0.6, Re_i=300.0, Re_o=-50.0, dt=1e-4,
                           amp=0.05, envelope="k53", seed=9, k_theta=1.0, k_z=1.0, alpha=0.0)
    A = Solver(*args)
    u0 = to_dev(tc_inputs.initial_state(A.radial_nodes(), cfg))
    A.set_state(u0)
    A.step(2)
    ua, pa = A.get_state()
    B = Solver(*args)
    B.set_state(u0)
    B.step(1)
    u1 = B.get_state(with_pressure=False)
    up1, Np1 = B.get_history()
    B.set_state(u1, up1, Np1)
    B.step(1)
    ub, pb = B.get_state()
    eu, ep = rel_l2(to_host(ua), to_host(ub)), rel_l2(to_host(pa), to_host(pb))
    print(f"fused vs standalone curl after two steps: u {eu:.2e}, p {ep:.2e}")
    assert eu < 1e-14 and ep < 1e-13
    A.close()
    B.close()


def test_wall_torque_undefined_without_laminar_torque():
    # Re_i = eta Re_o: circular Couette flow is a solid-body rotation
    # (C2 = 0) and exerts no torque, so Nu_omega has no reference: NaN,
    # while the other diagnostics stay defined
    from paper_1311_2481_amd import Solver
    S = Solver(12, 3, 6, 0.5, 10.0, 20.0, 1e-3)
    S.set_state(to_dev(tc_inputs.random_state((3, 12, 6, 3), 8)))
    d = S.diag()
    assert np.isnan(d["nu_inner"]) and np.isnan(d["nu_outer"])
    assert all(np.isfinite(d[k]) for k in ("energy", "perturbation_energy", "max_div", "slip", "cfl"))
    S.close()


@pytest.mark.parametrize("name", ["small", "medium", "adjoint"])
def test_factor_backward_error_is_at_rounding(name):
    # tc_init accepts the unpivoted factors only below 1e-12; on the
    # workloads they sit at a few units of rounding
    from paper_1311_2481_amd import Solver
    cfg = tc_inputs.CONFIGS[name]
    S = Solver(cfg.n_r, cfg.m_theta, cfg.m_z, cfg.eta, cfg.Re_i, cfg.Re_o, cfg.dt)
    err = S.factor_backward_error()
    print(f"{name}: largest componentwise backward error of the factors {err:.2e}")
    assert 0.0 < err < 1e-14
    S.close()
