"""Pins of the oracle's optimal-perturbation ascent (control map, its
adjoint, the control gradient and the ascent itself)."""
import numpy as np
import pytest

import oracle
import tc_inputs
from oracle import adjoint as adj
from oracle import optimal as opt
from oracle import scheme


def _prob(n_r=17, m_theta=4, m_z=8, dt=1e-3, Re_i=100.0):
    return oracle.Problem(n_r, m_theta, m_z, 0.5, Re_i, 0.0, dt, k_theta=2.0, k_z=1.5)


def _control(P, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.standard_normal(opt.control_shape(P)) + 1j * rng.standard_normal(opt.control_shape(P))
    return opt.hermitian_projection(P, a)


def test_control_velocity_matches_the_input_generator():
    # the synthetic inputs are the same family: for the generator's own
    # coefficients, the control map reproduces its perturbation up to the
    # generator's amplitude scale (two independent implementations)
    cfg = tc_inputs.Config(tc_inputs.CONFIGS["small"])
    cfg.update(envelope="k53", k_theta=2.0, k_z=1.5)
    P = oracle.Problem(cfg.n_r, cfg.m_theta, cfg.m_z, cfg.eta, cfg.Re_i, cfg.Re_o, cfg.dt, k_theta=2.0, k_z=1.5)
    a = tc_inputs.perturbation_coefficients(cfg.m_theta, cfg.m_z, cfg.envelope, cfg.seed, 2.0, 1.5)
    v = opt.velocity(P, a)
    w = tc_inputs.initial_state(P.r, cfg, with_couette=False)
    c = adj.inner(v, w) / adj.inner(v, v)
    assert np.linalg.norm(w - c * v) <= 1e-13 * np.linalg.norm(w)


def test_control_gradient_is_the_adjoint_of_the_control_map():
    P = _prob()
    a = _control(P, 3)
    g = tc_inputs.random_state((3, P.n_r, P.m_z, P.m_theta), 4, hermitian=False)
    lhs = adj.inner(g, opt.velocity(P, a))
    rhs = adj.inner(opt.control_gradient(P, g), a)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_control_velocity_is_divergence_free_and_real():
    # divergence-free in the continuum: the FD divergence falls at high
    # order with n_r; zero at the walls; real field (n = 0 symmetry)
    errs = []
    for n_r in (24, 48):
        P = _prob(n_r=n_r)
        u = opt.velocity(P, _control(P, 5))
        errs.append(np.abs(scheme.div(P, u)).max() / np.abs(u).max())
        assert np.abs(u[:, 0]).max() == 0.0 and np.abs(u[:, -1]).max() < 1e-12 * np.abs(u).max()
        ur = 0.5 * (u[0] + u[1])
        h = P.m_z // 2
        np.testing.assert_allclose(ur[:, P.m_z - np.arange(1, h), 0], np.conj(ur[:, np.arange(1, h), 0]),
                                   rtol=0, atol=1e-13 * np.abs(u).max())
    assert errs[1] < errs[0] / 2 ** 5 and errs[1] < 1e-5, errs


def test_control_gradient_matches_central_differences():
    P = _prob()
    a = 0.05 * _control(P, 7)
    nsteps = 6
    J, G = opt.objective_and_gradient(P, a, nsteps, checkpoint_every=4)
    for seed in (8, 9):
        d = _control(P, seed)
        eps = 1e-4 * np.sqrt(adj.inner(a, a) / adj.inner(d, d))
        Jp, _ = opt.objective_and_gradient(P, a + eps * d, nsteps)
        Jm, _ = opt.objective_and_gradient(P, a - eps * d, nsteps)
        fd = (Jp - Jm) / (2 * eps)
        assert abs(fd - adj.inner(G, d)) <= 1e-6 * abs(fd)


def test_ascent_raises_the_final_energy_on_the_energy_sphere():
    P = _prob(Re_i=300.0)
    a0 = _control(P, 11)
    E0 = 1e-3
    a, hist = opt.ascent(P, a0, E0, nsteps=10, iters=4)
    assert all(hist[k + 1] >= hist[k] for k in range(len(hist) - 1)), hist
    assert hist[-1] > 1.02 * hist[0], hist
    assert abs(opt.control_energy(P, a) - E0) <= 1e-12 * E0
