"""GPU parity: every C-ABI entry point against the FP64 oracle on identical inputs."""
import numpy as np
import pytest

import oracle
import tc_inputs
from oracle import scheme
from gpu_common import floor_tol, make_pair, rel_l2, to_dev, to_host, twin_floor

pytestmark = pytest.mark.gpu

SIZES = ["small", "medium"]
_pairs = {}


def pair(name, precision="fp64"):
    key = (name, precision)
    if key not in _pairs:
        _pairs[key] = make_pair(name, precision)
    return _pairs[key]


@pytest.mark.parametrize("name", SIZES)
def test_radial_nodes(name):
    S, P, cfg = pair(name)
    np.testing.assert_allclose(S.radial_nodes(), P.r, rtol=0, atol=4e-16 * P.r_o)


# Tolerances: 10x the floor of each solve, the difference between the
# oracle's banded LAPACK solve and a dense LU of the same operators.  The
# Helmholtz operators are well conditioned (floor ~1e-16); the Neumann
# Poisson operator P is not (condition number ~ (1/h_min)^2 / |lambda_min|),
# and any two backward-stable solvers, the GPU's unpivoted row-scaled LU
# among them, differ at that conditioning level.


@pytest.mark.parametrize("name", SIZES)
@pytest.mark.parametrize("kind", ["P", "Up", "Um", "Uz", "Phi"])
@pytest.mark.parametrize("transposed", [False, True])
def test_helmholtz_solve(name, kind, transposed):
    S, P, cfg = pair(name)
    rhs = tc_inputs.random_state((cfg.n_r, cfg.m_z, cfg.m_theta), 100 + len(kind), hermitian=False)
    out = S.empty(1).fill_(complex(7.0, -3.0))
    x = to_host(S.solve(kind, to_dev(rhs), out=out, transposed=transposed))
    k = "P" if kind == "Phi" else kind
    ref = P.solve(k, rhs, trans=1 if transposed else 0)
    floor = twin_floor(P, lambda Q: Q.solve(k, rhs, trans=1 if transposed else 0), ref)
    err = rel_l2(x, ref)
    print(f"{name} {kind} trans={transposed} rel_l2={err:.3e} (floor {floor:.2e})")
    assert err < floor_tol(floor)
    # the empty axial slot is written as zero (the output array is not cleared first)
    assert np.all(x[:, cfg.m_z // 2] == 0)


@pytest.mark.parametrize("name", SIZES)
def test_nonlinear(name):
    S, P, cfg = pair(name)
    u = tc_inputs.initial_state(P.r, cfg)
    N = to_host(S.nonlinear(to_dev(u)))
    ref = oracle.nonlinear_rot(P, u)
    err = rel_l2(N, ref)
    print(f"{name} nonlinear rel_l2={err:.3e}")
    assert err < 1e-12
    assert np.all(N[:, :, cfg.m_z // 2] == 0)


@pytest.mark.parametrize("name", SIZES)
def test_nonlinear_non_hermitian_input(name):
    # the n = 0 handling must reproduce the plain transform for ANY input
    S, P, cfg = pair(name)
    u = tc_inputs.random_state((3, cfg.n_r, cfg.m_z, cfg.m_theta), 77, hermitian=False)
    N = to_host(S.nonlinear(to_dev(u)))
    ref = oracle.nonlinear_rot(P, u)
    err = rel_l2(N, ref)
    print(f"{name} nonlinear (non-Hermitian) rel_l2={err:.3e}")
    assert err < 1e-12


@pytest.mark.parametrize("name", SIZES)
def test_nonlinear_energy_neutral(name):
    S, P, cfg = pair(name)
    u = tc_inputs.initial_state(P.r, cfg)
    N = to_host(S.nonlinear(to_dev(u)))
    c = np.full(cfg.m_theta, 2.0)
    c[0] = 1.0
    dens = 0.5 * (np.conj(u[0]) * N[0] + np.conj(u[1]) * N[1]) + np.conj(u[2]) * N[2]
    work = np.einsum("n,jsn->j", c, dens.real)
    assert np.abs(work).max() <= 1e-13 * np.linalg.norm(u) * np.linalg.norm(N)


@pytest.mark.parametrize("name", SIZES)
def test_one_step(name):
    # R21: relative field error after one step from an identical state
    S, P, cfg = pair(name)
    u0 = tc_inputs.initial_state(P.r, cfg)
    N0 = oracle.nonlinear_rot(P, u0)
    S.set_state(to_dev(u0), None, to_dev(N0))
    S.step(1)
    ug, pg = S.get_state()
    ug, pg = to_host(ug), to_host(pg)
    ur, pr, Nr = scheme.step(P, u0, u0, N0)
    err = rel_l2(ug, ur)
    pert = rel_l2(ug - oracle.diagnostics.couette_state(P), ur - oracle.diagnostics.couette_state(P))
    perr = rel_l2(pg, pr)
    fu = twin_floor(P, lambda Q: scheme.step(Q, u0, u0, N0)[0], ur)
    fp = twin_floor(P, lambda Q: scheme.step(Q, u0, u0, N0)[1], pr)
    print(f"{name} one step: u rel_l2={err:.3e} (perturbation-relative {pert:.3e}), p rel_l2={perr:.3e}; "
          f"floors u {fu:.2e}, p {fp:.2e}")
    assert err <= 1e-11
    assert err <= floor_tol(fu) and perr <= floor_tol(fp)
    up, Np = S.get_history()
    assert rel_l2(to_host(Np), Nr) < 1e-12
    assert rel_l2(to_host(up), u0) == 0.0


@pytest.mark.parametrize("name", SIZES)
def test_diagnostics(name):
    # tc_get_diag against the oracle's definitions on the workload's state
    # (sums in a different order: relative agreement to ~1e-13)
    from oracle import diagnostics as dg
    S, P, cfg = pair(name)
    u = tc_inputs.initial_state(P.r, cfg)
    S.set_state(to_dev(u))
    d = S.diag()
    div = np.abs(scheme.div(P, u)[1:-1]).max()
    ref = dict(energy=dg.energy(P, u), perturbation_energy=dg.perturbation_energy(P, u), max_div=div,
               slip=dg.wall_slip(P, u), cfl=dg.cfl_bound(P, u))
    # the divergence of a divergence-free field is a cancellation: bound its
    # difference by the size of the terms summed, sum |D1_jk| |u_r,k| + |u_r|/r
    # + a |u+ - u-|/(2r) + |b u_z| at the worst node
    a, b, r = P.bcast()
    ur = 0.5 * np.abs(u[0] + u[1])
    terms = (np.einsum("jk,ksn->jsn", np.abs(P.D1), ur) + ur / r + a * np.abs(u[0] - u[1]) / (2 * r)
             + np.abs(b * u[2]))
    tol = dict(max_div=1e-14 * terms[1:-1].max())
    ref.update(nu_tol(P, u, tol))
    for k, v in ref.items():
        print(f"{name} {k}: gpu {d[k]:.15e} oracle {v:.15e}")
        assert abs(d[k] - v) <= tol.get(k, 1e-12 * abs(v)), k
    assert d["steps"] == 0
    # a mean flow sheared away from Couette's at both walls (Nu != 1)
    x = (P.r - P.r[0]) / (P.r[-1] - P.r[0])
    bump = 0.3 * abs(P.Re_i) * x * (1 - x) * np.cos(3 * x)
    u[0, :, 0, 0] += 1j * bump
    u[1, :, 0, 0] -= 1j * bump
    S.set_state(to_dev(u))
    d, tol = S.diag(), {}
    for k, v in nu_tol(P, u, tol).items():
        print(f"{name} sheared mean {k}: gpu {d[k]:.15e} oracle {v:.15e}")
        assert abs(v - 1) > 0.1 and abs(d[k] - v) <= tol[k], k


def nu_tol(P, u, tol):
    """Oracle wall torques of u, with their tolerances put into tol: the D1
    wall row sums terms far larger than the result (weights ~ 1 / h_wall),
    and the two sides' weights differ by rounding."""
    from oracle import diagnostics as dg
    nu = dg.quasi_nusselt(P, u)
    C2 = P.eta * (P.Re_i - P.eta * P.Re_o) / ((1 - P.eta) * (1 - P.eta ** 2))
    om = np.abs((-0.5j * (u[0, :, 0, 0] - u[1, :, 0, 0])).real / P.r)
    out = {}
    for key, j, v in (("nu_inner", 0, nu[0]), ("nu_outer", -1, nu[1])):
        out[key] = v
        tol[key] = 1e-14 * abs(P.r[j]) ** 3 * (np.abs(P.D1[j]) @ om) / abs(2 * C2) + 1e-13 * abs(v)
    return out


def test_trajectory_small():
    S, P, cfg = pair("small")
    u0 = tc_inputs.initial_state(P.r, cfg)
    S.set_state(to_dev(u0))
    S.step(cfg.steps)
    ug = to_host(S.get_state(with_pressure=False))
    ur, _, _, _ = scheme.run(P, u0, cfg.steps)
    err = rel_l2(ug, ur)
    pert = rel_l2(ug - oracle.diagnostics.couette_state(P), ur - oracle.diagnostics.couette_state(P))
    print(f"small {cfg.steps} steps: rel_l2={err:.3e} perturbation-relative={pert:.3e}")
    assert err < 1e-11
