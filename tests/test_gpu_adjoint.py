"""GPU discrete adjoint: one adjoint step against the oracle's, the
checkpointed gradient against the oracle's gradient and against central
finite differences of the GPU forward map (the differentiation workload:
N_r = 64, 128 x 128 physical, Re_i = 1000, T = 400 steps, checkpoints every
20 steps)."""
import numpy as np
import pytest

import oracle
import tc_inputs
from oracle import adjoint as adj
from oracle import diagnostics as dg
from gpu_common import make_pair, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["small", "medium"])
@pytest.mark.parametrize("hermitian", [True, False])
def test_adjoint_step_matches_oracle(name, hermitian):
    S, P, cfg = make_pair(name)
    u = tc_inputs.initial_state(P.r, cfg)
    shape = (3, cfg.n_r, cfg.m_z, cfg.m_theta)
    a, b, c = (tc_inputs.random_state(shape, 60 + k, hermitian=hermitian) for k in range(3))
    out = to_host(S.step_adjoint(to_dev(np.concatenate([u, u])), to_dev(np.concatenate([a, b, c]))))
    ref = adj.step_adjoint(P, u, a, b, c)
    errs = [rel_l2(out[3 * k:3 * k + 3], ref[k]) for k in range(3)]
    print(f"{name} adjoint step (hermitian={hermitian}): rel_l2 u {errs[0]:.2e}, u_prev {errs[1]:.2e}, N_prev {errs[2]:.2e}")
    assert max(errs) < (1e-12 if name == "small" else 1e-9)
    S.close()


def test_energy_gradient_matches_oracle():
    S, P, cfg = make_pair("small")
    u = tc_inputs.initial_state(P.r, cfg)
    g = to_host(S.energy_gradient(to_dev(u)))
    assert rel_l2(g, adj.perturbation_energy_gradient(P, u)) < 1e-13
    S.close()


def test_gradient_matches_oracle_gradient():
    from paper_1311_2481_amd.autograd import final_energy_and_gradient
    S, P, cfg = make_pair("small", dt=2e-4)
    u0 = tc_inputs.initial_state(P.r, cfg)
    base = dg.couette_state(P)
    J, g = final_energy_and_gradient(S, to_dev(base), to_dev(u0 - base), 8, every=3)
    Jr, gr = adj.gradient(P, u0, 8, checkpoint_every=3)
    err = rel_l2(to_host(g), gr)
    print(f"gradient vs oracle (8 steps): J {J:.6e} / {Jr:.6e}, rel_l2 {err:.2e}")
    assert abs(J - Jr) <= 1e-11 * abs(Jr)
    assert err < 1e-10
    S.close()


def test_differentiation_workload_gradient_vs_finite_differences():
    import torch
    from paper_1311_2481_amd.autograd import final_energy_and_gradient
    S, P, cfg = make_pair("adjoint")
    r = P.r
    u0 = tc_inputs.initial_state(r, cfg)
    base = dg.couette_state(P)
    pert = u0 - base
    T, every = cfg.steps, cfg.checkpoint_every
    J, g = final_energy_and_gradient(S, to_dev(base), to_dev(pert), T, every=every)
    g = to_host(g)

    def J_of(x):
        S.set_state(to_dev(x))
        S.step(T)
        return S.diag()["perturbation_energy"]

    worst = 0.0
    for seed in range(1000, 1008):
        v = tc_inputs.random_direction(r, cfg, seed)
        v *= np.linalg.norm(pert) / np.linalg.norm(v)
        ad = adj.inner(g, v)
        best = np.inf
        for eps in (1e-3, 1e-4, 1e-5):
            fd = (J_of(u0 + eps * v) - J_of(u0 - eps * v)) / (2 * eps)
            best = min(best, abs(fd - ad) / abs(ad))
        worst = max(worst, best)
        print(f"direction {seed}: adjoint {ad:.10e}, best relative FD mismatch {best:.2e}")
    print(f"J = {J:.10e}; worst over 8 directions: {worst:.2e}")
    assert worst < 1e-6
    S.close()
