"""Pins of the oracle's tangent-linear model and discrete adjoint."""
import numpy as np
import pytest

import oracle
import tc_inputs
from oracle import adjoint as adj
from oracle import diagnostics as dg
from oracle import scheme


@pytest.fixture(scope="module")
def setup():
    cfg = dict(tc_inputs.CONFIGS["small"])
    cfg.update(amp=0.05, envelope="k53", m_theta=8, m_z=8, n_r=20, dt=2e-4)
    P = oracle.Problem(cfg["n_r"], cfg["m_theta"], cfg["m_z"], cfg["eta"], cfg["Re_i"], cfg["Re_o"], cfg["dt"],
                       k_theta=2.0, k_z=1.5)
    u = tc_inputs.initial_state(P.r, cfg)
    return P, cfg, u


def rnd(P, seed, k=3, hermitian=False):
    return tc_inputs.random_state((k, P.n_r, P.m_z, P.m_theta), seed, hermitian=hermitian)


def test_pc_linear_is_the_step_minus_its_constant(setup):
    P, cfg, u = setup
    N, Np, up = rnd(P, 1, hermitian=True), rnd(P, 2, hermitian=True), rnd(P, 3, hermitian=True)
    full, _ = scheme.predictor_corrector(P, N, Np, u, up)
    const, _ = scheme.predictor_corrector(P, 0 * N, 0 * N, 0 * u, 0 * u)
    lin = adj.pc_linear(P, 2 * N - Np, u, up)
    np.testing.assert_allclose(full - const, lin, rtol=0, atol=1e-10 * np.abs(lin).max())


def test_nonlinear_tlm_is_the_derivative(setup):
    P, cfg, u = setup
    du = rnd(P, 5, hermitian=True)
    eps = 1e-6 * np.linalg.norm(u) / np.linalg.norm(du)
    fd = (oracle.nonlinear_rot(P, u + eps * du) - oracle.nonlinear_rot(P, u - eps * du)) / (2 * eps)
    tl = adj.nonlinear_tlm(P, u, du)
    assert np.linalg.norm(fd - tl) / np.linalg.norm(tl) < 1e-7


@pytest.mark.parametrize("hermitian", [True, False])
def test_nonlinear_adjoint_dot_product(setup, hermitian):
    P, cfg, u = setup
    du, w = rnd(P, 11, hermitian=hermitian), rnd(P, 12, hermitian=hermitian)
    lhs = adj.inner(w, adj.nonlinear_tlm(P, u, du))
    rhs = adj.inner(adj.nonlinear_adjoint(P, u, w), du)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_pc_adjoint_dot_product(setup):
    P, cfg, u = setup
    Ne, uu, up, w = rnd(P, 21), rnd(P, 22), rnd(P, 23), rnd(P, 24)
    lhs = adj.inner(w, adj.pc_linear(P, Ne, uu, up))
    a, b, c = adj.pc_adjoint(P, w)
    rhs = adj.inner(a, Ne) + adj.inner(b, uu) + adj.inner(c, up)
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_sub_operator_adjoints(setup):
    P, cfg, u = setup
    f, v = rnd(P, 31, k=1)[0], rnd(P, 32)
    assert abs(adj.inner(f, scheme.div(P, v)) - adj.inner(adj.div_adjoint(P, f), v)) < 1e-10 * np.abs(f).max() * np.abs(v).max() * f.size
    assert abs(adj.inner(v, scheme.grad(P, f)) - adj.inner(adj.grad_adjoint(P, v), f)) < 1e-10 * np.abs(f).max() * np.abs(v).max() * f.size
    lhs = adj.inner(f, scheme.vector_laplacian_r(P, v))
    rhs = adj.inner(adj.vector_laplacian_r_adjoint(P, f), v)
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs) * 100 + 1e-8


def test_step_adjoint_dot_product(setup):
    P, cfg, u = setup
    du, dup, dNp = rnd(P, 41), rnd(P, 42), rnd(P, 43)
    a, b, c = rnd(P, 44), rnd(P, 45), rnd(P, 46)
    t1, t2, t3 = adj.step_tlm(P, u, du, dup, dNp)
    lhs = adj.inner(a, t1) + adj.inner(b, t2) + adj.inner(c, t3)
    x, y, z = adj.step_adjoint(P, u, a, b, c)
    rhs = adj.inner(x, du) + adj.inner(y, dup) + adj.inner(z, dNp)
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_step_tlm_matches_finite_difference(setup):
    P, cfg, u = setup
    up, Np = u.copy(), oracle.nonlinear_rot(P, u)
    du, dup, dNp = rnd(P, 51, hermitian=True), rnd(P, 52, hermitian=True), rnd(P, 53, hermitian=True)
    eps = 1e-6 * np.linalg.norm(u) / np.linalg.norm(du)
    plus = scheme.step(P, u + eps * du, up + eps * dup, Np + eps * dNp)
    minus = scheme.step(P, u - eps * du, up - eps * dup, Np - eps * dNp)
    fd = (plus[0] - minus[0]) / (2 * eps)
    tl = adj.step_tlm(P, u, du, dup, dNp)[0]
    assert np.linalg.norm(fd - tl) / np.linalg.norm(tl) < 1e-6


def test_gradient_matches_central_differences(setup):
    # T15: dJ/du0 . v against central differences along divergence-free
    # directions (same recipe as the initial perturbation)
    P, cfg, u = setup
    J, g = adj.gradient(P, u, 6, checkpoint_every=4)
    for seed in (1000, 1001):
        v = tc_inputs.random_direction(P.r, cfg, seed)
        v *= 1e-2 * np.linalg.norm(u - dg.couette_state(P)) / np.linalg.norm(v)
        fds = []
        for eps in (1e-1, 1e-2):
            Jp = dg.perturbation_energy(P, scheme.run(P, u + eps * v, 6)[0])
            Jm = dg.perturbation_energy(P, scheme.run(P, u - eps * v, 6)[0])
            fds.append((Jp - Jm) / (2 * eps))
        ad = adj.inner(g, v)
        err = min(abs(f - ad) for f in fds) / abs(ad)
        assert err < 1e-6, (seed, fds, ad)


def test_checkpointing_does_not_change_the_gradient(setup):
    P, cfg, u = setup
    J1, g1 = adj.gradient(P, u, 5, checkpoint_every=1)
    J2, g2 = adj.gradient(P, u, 5, checkpoint_every=20)
    assert J1 == J2
    np.testing.assert_allclose(g1, g2, rtol=0, atol=1e-13 * np.abs(g1).max())
