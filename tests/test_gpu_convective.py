"""GPU parity of the paper's convective form N = u.grad u (Sec. 3.2, step 1,
with the curvature terms of eq. NS_cyl) against the oracle, and the time-step
range it buys over the rotational form."""
import numpy as np
import pytest

import oracle
import tc_inputs
from oracle import scheme
from gpu_common import rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu

LENGTHS = [16, 24, 32, 40, 48, 64, 80, 96, 120, 128, 144, 160, 192, 240, 256, 288, 320, 384, 480, 512, 576,
           640, 768, 960, 1024, 1152, 1280, 1536, 1920, 2048]
CASES = [(LENGTHS[i], LENGTHS[(i + 5) % len(LENGTHS)]) for i in range(len(LENGTHS))]


def _pair(name, **over):
    from paper_1311_2481_amd import Solver
    cfg = tc_inputs.Config(tc_inputs.CONFIGS[name])
    cfg.update(over)
    args = (cfg.n_r, cfg.m_theta, cfg.m_z, cfg.eta, cfg.Re_i, cfg.Re_o, cfg.dt)
    S = Solver(*args, k_theta=cfg.k_theta, k_z=cfg.k_z, form="conv")
    P = oracle.Problem(*args, k_theta=cfg.k_theta, k_z=cfg.k_z, form="conv")
    return S, P, cfg


@pytest.mark.parametrize("name", ["small", "medium"])
@pytest.mark.parametrize("hermitian", [True, False])
def test_convective_nonlinear(name, hermitian):
    S, P, cfg = _pair(name)
    if hermitian:
        u = tc_inputs.initial_state(P.r, cfg)
    else:
        u = tc_inputs.random_state((3, cfg.n_r, cfg.m_z, cfg.m_theta), 91, hermitian=False)
    N = to_host(S.nonlinear(to_dev(u)))
    ref = oracle.nonlinear_conv(P, u)
    err = rel_l2(N, ref)
    print(f"{name} convective nonlinear (hermitian={hermitian}) rel_l2={err:.3e}")
    assert err < 1e-12
    assert np.all(N[:, :, cfg.m_z // 2] == 0)
    S.close()


@pytest.mark.parametrize("p_theta,p_z", CASES)
def test_convective_nonlinear_all_lengths(p_theta, p_z):
    from paper_1311_2481_amd import Solver
    m_theta, m_z = (p_theta + 2) // 3, 2 * ((p_z + 2) // 3)
    args = (11, m_theta, m_z, 0.6, 80.0, -20.0, 1e-3)
    S = Solver(*args, k_theta=1.5, k_z=0.8, p_theta=p_theta, p_z=p_z, form="conv")
    P = oracle.Problem(*args, k_theta=1.5, k_z=0.8, p_theta=p_theta, p_z=p_z, form="conv")
    u = tc_inputs.random_state((3, P.n_r, P.m_z, P.m_theta), 5 * p_theta + p_z)
    err = rel_l2(to_host(S.nonlinear(to_dev(u))), oracle.nonlinear_conv(P, u))
    print(f"P_theta={p_theta} P_z={p_z}: convective nonlinear rel_l2 {err:.2e}")
    assert err < 1e-12
    S.close()


@pytest.mark.parametrize("name", ["small", "medium"])
def test_convective_one_step(name):
    S, P, cfg = _pair(name)
    u0 = tc_inputs.initial_state(P.r, cfg)
    N0 = oracle.nonlinear_conv(P, u0)
    S.set_state(to_dev(u0), None, to_dev(N0))
    S.step(1)
    ug, pg = S.get_state()
    ur, pr, Nr = scheme.step(P, u0, u0, N0)
    err, perr = rel_l2(to_host(ug), ur), rel_l2(to_host(pg), pr)
    print(f"{name} convective one step: u rel_l2={err:.3e}, p rel_l2={perr:.3e}")
    assert err <= 1e-11
    _, Np = S.get_history()
    assert rel_l2(to_host(Np), Nr) < 1e-12
    S.close()


def test_convective_small_trajectory():
    S, P, cfg = _pair("small")
    u0 = tc_inputs.initial_state(P.r, cfg)
    S.set_state(to_dev(u0))
    S.step(cfg.steps)
    ref, _, _, _ = scheme.run(P, u0, cfg.steps)
    err = rel_l2(to_host(S.get_state(with_pressure=False)), ref)
    print(f"small convective {cfg.steps}-step trajectory rel_l2={err:.3e}")
    assert err < 1e-11
    S.close()


def test_convective_form_runs_where_the_rotational_form_grows():
    # the differentiation workload's flow at dt = 2e-6: the rotational form
    # has a growing mode (n, l) = (1, 0) there (the oracle's per-mode probe),
    # the paper's convective form none; 2000 steps on the GPU
    from paper_1311_2481_amd import Solver
    cfg = tc_inputs.Config(tc_inputs.CONFIGS["adjoint"])
    res = {}
    for form in ("rot", "conv"):
        S = Solver(cfg.n_r, cfg.m_theta, cfg.m_z, cfg.eta, cfg.Re_i, cfg.Re_o, 2e-6, form=form)
        S.set_state(tc_inputs.initial_state(S.radial_nodes(), cfg, device="cuda"))
        e0 = S.diag()["perturbation_energy"]
        S.step(2000)
        e1 = S.diag()["perturbation_energy"] if S.check_finite() else float("inf")
        res[form] = e1 / e0
        print(f"{form}: perturbation energy x{res[form]:.3e} over 2000 steps at dt = 2e-6")
        S.close()
    assert res["conv"] < 10.0
    assert res["rot"] > 1e6


def test_convective_form_limits():
    from paper_1311_2481_amd import Solver, TcError
    cfg = tc_inputs.CONFIGS["small"]
    args = (cfg.n_r, cfg.m_theta, cfg.m_z, cfg.eta, cfg.Re_i, cfg.Re_o, cfg.dt)
    with pytest.raises(TcError, match="FP64 only"):
        Solver(*args, precision="fp32_bulk", form="conv")
    S = Solver(*args, form="conv")
    u = S.zeros(3)
    with pytest.raises(TcError, match="rotational form"):
        S.step_adjoint(S.zeros(6), S.zeros(9))
    S.close()
