"""Parity at the production size (N_r = 512, 1536 x 1536 dealiased planes),
sampled where the oracle cannot afford the whole field: the nonlinear term
on 8 radial planes (each depends on its plane and 4 neighbours) and every
solve kind on 256 distinct modes (each independent)."""
import numpy as np
import pytest

import oracle
import tc_inputs
from oracle import nonlinear as nl

pytestmark = pytest.mark.gpu

PLANES = [0, 1, 4, 100, 255, 256, 507, 511]
_state = {}


def solver():
    if "S" not in _state:
        from paper_1311_2481_amd import Solver
        cfg = tc_inputs.Config(tc_inputs.CONFIGS["production"])
        S = Solver(cfg.n_r, cfg.m_theta, cfg.m_z, cfg.eta, cfg.Re_i, cfg.Re_o, cfg.dt)
        P = oracle.Problem(cfg.n_r, cfg.m_theta, cfg.m_z, cfg.eta, cfg.Re_i, cfg.Re_o, cfg.dt)
        _state.update(S=S, P=P, cfg=cfg)
    return _state["S"], _state["P"], _state["cfg"]


def _jittered(P, seed):
    """Copy of P whose D1 weights carry independent one-ulp perturbations."""
    import copy
    Q = copy.copy(P)
    rng = np.random.Generator(np.random.PCG64(seed))
    Q.D1 = P.D1 * (1.0 + 2.2e-16 * rng.choice([-1.0, 1.0], size=P.D1.shape))
    return Q


def test_production_nonlinear_sampled_planes():
    # Near the walls the 9-point weights reach ~1/h_min ~ 1e5 and u_theta ~
    # Re ~ 1e4, so omega there carries a rounding floor set by the weights
    # themselves: it is measured by re-running the oracle with D1 perturbed
    # by one ulp, and the GPU must sit within a small multiple of it.
    import torch
    S, P, cfg = solver()
    Q = _jittered(P, 17)
    u = tc_inputs.initial_state(P.r, cfg, device="cuda")
    N = S.nonlinear(u)
    torch.cuda.synchronize()
    num = den = 0.0
    for j in PLANES:
        lo, hi = max(0, j - 4), min(cfg.n_r - 1, j + 4)
        window = u[:, lo:hi + 1].cpu().numpy()
        ref = nl.nonlinear_rot_at(P, window, j)
        floor = np.linalg.norm(nl.nonlinear_rot_at(Q, window, j) - ref) / np.linalg.norm(ref)
        got = N[:, j].cpu().numpy()
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        num += np.sum(np.abs(got - ref) ** 2)
        den += np.sum(np.abs(ref) ** 2)
        print(f"production nonlinear plane {j}: rel_l2={err:.2e} (one-ulp D1 floor {floor:.2e})")
        assert err <= max(20.0 * floor, 1e-12)
        assert np.all(got[:, cfg.m_z // 2] == 0)
    total = np.sqrt(num / den)
    print(f"production nonlinear, 8 sampled planes together: rel_l2={total:.2e}")
    assert total < 1e-11
    del u, N
    torch.cuda.empty_cache()


@pytest.mark.parametrize("kind", ["P", "Up", "Um", "Uz"])
def test_production_solve_sampled_modes(kind):
    import torch
    S, P, cfg = solver()
    rhs = tc_inputs.random_field_torch((cfg.n_r, cfg.m_z, cfg.m_theta), 31 + len(kind), "cuda")
    x = S.solve(kind, rhs)
    torch.cuda.synchronize()
    rng = np.random.Generator(np.random.PCG64(8))
    picks = [(0, 0), (0, 1), (1, 0), (cfg.m_z // 2 - 1, cfg.m_theta - 1)]
    picks += [(int(rng.integers(cfg.m_z // 2)), int(rng.integers(cfg.m_theta))) for _ in range(252)]
    num = den = 0.0
    for labs, n in picks:
        slots = [labs] if labs == 0 else [labs, cfg.m_z - labs]
        b = rhs[:, slots, n].cpu().numpy()
        cols = np.concatenate([np.stack([b[:, k].real, b[:, k].imag], 1) for k in range(len(slots))], 1)
        ref = P.solve_mode(kind, n, labs, np.ascontiguousarray(cols))
        got = x[:, slots, n].cpu().numpy()
        for k in range(len(slots)):
            r = ref[:, 2 * k] + 1j * ref[:, 2 * k + 1]
            num += np.sum(np.abs(got[:, k] - r) ** 2)
            den += np.sum(np.abs(r) ** 2)
    err = np.sqrt(num / den)
    print(f"production solve {kind}, 256 sampled modes rel_l2={err:.3e}")
    # the Neumann Poisson operator is ill conditioned at n_r = 512 (smallest
    # near-wall spacing ~1e-5): two LU solvers differ at ~1e-10 there
    assert err < (1e-8 if kind == "P" else 1e-12)
    del rhs, x
    torch.cuda.empty_cache()
