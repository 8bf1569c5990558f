"""The line predictor-corrector (each mode's radial line spread over 4, 8 or
16 lanes and held on chip; grids of 32, 64 and 128 radial nodes) against the
FP64 oracle, and against the four-sweep kernels on the same inputs (a
context created with TC_PC_LINE=0 uses those)."""
import numpy as np
import pytest

import oracle
import tc_inputs
from oracle import scheme
from gpu_common import floor_tol, make_pair, rel_l2, to_dev, to_host, twin_floor

pytestmark = pytest.mark.gpu

# (workload, overrides): 4, 8 and 16 lanes per slot; the (12, 20) shapes
# leave a ragged last tile and waves whose slots straddle two |l|.
CASES = [
    ("small", {}),
    ("medium", {}),
    ("medium", dict(m_theta=12, m_z=20)),
    ("medium", dict(n_r=128, m_theta=12, m_z=20)),
]
IDS = ["nr32", "nr64", "nr64-ragged", "nr128-ragged"]


def _inputs(P, cfg, seed):
    """u^i, u^{i-1} and N^{i-1} that differ from one another, so that every
    input of the step enters the result."""
    shape = (3, cfg.n_r, cfg.m_z, cfg.m_theta)
    u0 = tc_inputs.initial_state(P.r, cfg)
    up = u0 + 1e-3 * tc_inputs.random_state(shape, seed)
    up[:, 0] = u0[:, 0]
    up[:, -1] = u0[:, -1]
    Np = oracle.nonlinear_rot(P, u0) + 0.1 * tc_inputs.random_state(shape, seed + 1)
    return u0, up, Np


def _pair(case, monkeypatch, line=True, **extra):
    name, over = case
    if not line:
        monkeypatch.setenv("TC_PC_LINE", "0")
    try:
        return make_pair(name, **over, **extra)
    finally:
        monkeypatch.delenv("TC_PC_LINE", raising=False)


@pytest.mark.parametrize("case", CASES, ids=IDS)
@pytest.mark.parametrize("dt", [1e-6, 1e-4])
def test_line_step_matches_oracle(case, dt, monkeypatch):
    S, P, cfg = _pair(case, monkeypatch, dt=dt)
    u0, up, Np = _inputs(P, cfg, 71)
    S.set_state(to_dev(u0), to_dev(up), to_dev(Np))
    S.step(1)
    ug, pg = (to_host(x) for x in S.get_state())
    ur, pr, Nr = scheme.step(P, u0, up, Np)
    eu, ep = rel_l2(ug, ur), rel_l2(pg, pr)
    fu = twin_floor(P, lambda Q: scheme.step(Q, u0, up, Np)[0], ur)
    fp = twin_floor(P, lambda Q: scheme.step(Q, u0, up, Np)[1], pr)
    print(f"line step {case} dt={dt:g}: u rel_l2 {eu:.2e} (floor {fu:.2e}), p {ep:.2e} (floor {fp:.2e})")
    assert eu <= floor_tol(fu) and ep <= floor_tol(fp)
    # the Nyquist slot stays empty
    assert np.abs(ug[:, :, cfg.m_z // 2]).max() == 0.0 and np.abs(pg[:, cfg.m_z // 2]).max() == 0.0
    S.close()


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_line_matches_four_sweep_kernels(case, monkeypatch):
    """Five steps of both predictor-corrector forms from the same state: the
    states, pressures and histories agree within the one-step rounding floor
    of each quantity (velocity, pressure, and the nonlinear term of the new
    velocity, which the next step keeps as N^{i-1}) times the number of
    steps; the line context holds the second factor copy."""
    S, P, cfg = _pair(case, monkeypatch, dt=1e-5)
    R, _, _ = _pair(case, monkeypatch, line=False, dt=1e-5)
    assert S.memory_bytes() > R.memory_bytes()
    u0, up, Np = _inputs(P, cfg, 81)
    u1, p1, _ = scheme.step(P, u0, up, Np)
    fu = twin_floor(P, lambda Q: scheme.step(Q, u0, up, Np)[0], u1)
    fp = twin_floor(P, lambda Q: scheme.step(Q, u0, up, Np)[1], p1)
    fN = twin_floor(P, lambda Q: oracle.nonlinear_rot(Q, scheme.step(Q, u0, up, Np)[0]), oracle.nonlinear_rot(P, u1))
    for X in (S, R):
        X.set_state(to_dev(u0), to_dev(up), to_dev(Np))
    worst = 0.0
    for k in range(1, 6):
        for X in (S, R):
            X.step(1)
        (ua, pa), (ub, pb) = ([to_host(x) for x in X.get_state()] for X in (S, R))
        (ha, na), (hb, nb) = ([to_host(x) for x in X.get_history()] for X in (S, R))
        errs = [rel_l2(ua, ub), rel_l2(pa, pb), rel_l2(ha, hb), rel_l2(na, nb)]
        bounds = [floor_tol(fu), floor_tol(fp), floor_tol(fu), floor_tol(fN)]
        worst = max(worst, max(e / (k * f) for e, f in zip(errs, bounds)))
        print(f"step {k}: line vs four-sweep rel_l2 u {errs[0]:.2e}, p {errs[1]:.2e}, "
              f"u_prev {errs[2]:.2e}, N_prev {errs[3]:.2e}")
        for e, f in zip(errs, bounds):
            assert e <= k * f
    print(f"one-step floors u {fu:.2e}, p {fp:.2e}, N {fN:.2e}; worst difference over its bound {worst:.2f}")
    S.close()
    R.close()


@pytest.mark.parametrize("case", CASES, ids=IDS)
@pytest.mark.parametrize("kind", ["P", "Up", "Um", "Uz"])
def test_line_transposed_solve_matches_oracle(case, kind, monkeypatch):
    """The adjoint step's transposed solves on the line layout, one operator
    at a time, against the oracle's LAPACK transposed solve."""
    S, P, cfg = _pair(case, monkeypatch, dt=1e-5)
    rhs = tc_inputs.random_state((cfg.n_r, cfg.m_z, cfg.m_theta), 91, hermitian=False)
    out = S.empty(1).fill_(complex(7.0, -3.0))
    x = to_host(S.solve(kind, to_dev(rhs), out=out, transposed=True))
    ref = P.solve(kind, rhs, trans=1)
    floor = twin_floor(P, lambda Q: Q.solve(kind, rhs, trans=1), ref)
    err = rel_l2(x, ref)
    print(f"line transposed solve {case} {kind}: rel_l2 {err:.2e} (floor {floor:.2e})")
    assert err <= floor_tol(floor)
    # the empty axial slot is written as zero (the output array is not cleared first)
    assert np.all(x[:, cfg.m_z // 2] == 0)
    S.close()


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_line_adjoint_step_matches_oracle(case, monkeypatch):
    """The adjoint step with its predictor-corrector part on the line layout
    (one fused launch) against the oracle's adjoint step, and against the
    same step through the separate stencil and solve kernels."""
    from oracle import adjoint as adj
    S, P, cfg = _pair(case, monkeypatch, dt=1e-5)
    R, _, _ = _pair(case, monkeypatch, line=False, dt=1e-5)
    u = tc_inputs.initial_state(P.r, cfg)
    shape = (3, cfg.n_r, cfg.m_z, cfg.m_theta)
    a, b, c = (tc_inputs.random_state(shape, 60 + k, hermitian=False) for k in range(3))
    fwd, adj_in = to_dev(np.concatenate([u, u])), to_dev(np.concatenate([a, b, c]))
    out = to_host(S.step_adjoint(fwd, adj_in))
    alt = to_host(R.step_adjoint(fwd, adj_in))
    ref = adj.step_adjoint(P, u, a, b, c)
    errs = [rel_l2(out[3 * k:3 * k + 3], ref[k]) for k in range(3)]
    alts = [rel_l2(out[3 * k:3 * k + 3], alt[3 * k:3 * k + 3]) for k in range(3)]
    floors = [twin_floor(P, lambda Q: adj.step_adjoint(Q, u, a, b, c)[k], ref[k]) for k in range(3)]
    print(f"line adjoint step {case}: rel_l2 vs oracle u {errs[0]:.2e}, u_prev {errs[1]:.2e}, N_prev {errs[2]:.2e} "
          f"(floors {floors[0]:.2e} {floors[1]:.2e} {floors[2]:.2e}); vs separate kernels "
          f"{alts[0]:.2e} {alts[1]:.2e} {alts[2]:.2e}")
    for e, f, x in zip(errs, floors, alts):
        assert e <= floor_tol(f) and x <= floor_tol(f)
    S.close()
    R.close()


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_line_multistep_call_equals_single_steps(case, monkeypatch):
    """tc_step(5) (the pressure written on the last step only) gives the same
    bits as five tc_step(1) calls from the same state: state, pressure,
    history and the fused curl the next step uses."""
    S, P, cfg = _pair(case, monkeypatch, dt=1e-5)
    R, _, _ = _pair(case, monkeypatch, dt=1e-5)
    u0, up, Np = _inputs(P, cfg, 85)
    for X in (S, R):
        X.set_state(to_dev(u0), to_dev(up), to_dev(Np))
    S.step(5)
    for _ in range(5):
        R.step(1)
    for a, b in zip(S.get_state() + S.get_history(), R.get_state() + R.get_history()):
        assert np.array_equal(to_host(a), to_host(b))
    # one more step each: the curl each kept for it is the same
    S.step(1)
    R.step(1)
    assert np.array_equal(to_host(S.get_state()[0]), to_host(R.get_state()[0]))
    S.close()
    R.close()
