"""Helpers shared by the GPU parity tests: solver/oracle pairs on identical inputs."""
import numpy as np

import oracle
import tc_inputs


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def to_host(t):
    return t.detach().cpu().numpy()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def make_pair(name, precision="fp64", **over):
    """(GPU solver, oracle Problem, config) for a named workload."""
    from paper_1311_2481_amd import Solver
    cfg = tc_inputs.Config(tc_inputs.CONFIGS[name])
    cfg.update(over)
    S = Solver(cfg.n_r, cfg.m_theta, cfg.m_z, cfg.eta, cfg.Re_i, cfg.Re_o, cfg.dt,
               k_theta=cfg.k_theta, k_z=cfg.k_z, alpha=cfg.alpha, precision=precision)
    P = oracle.Problem(cfg.n_r, cfg.m_theta, cfg.m_z, cfg.eta, cfg.Re_i, cfg.Re_o, cfg.dt,
                       k_theta=cfg.k_theta, k_z=cfg.k_z, alpha=cfg.alpha)
    return S, P, cfg


def dense_twin(P):
    """Copy of an oracle problem whose per-mode solves use a dense LU with
    partial pivoting (numpy) instead of LAPACK's banded one.  Both are
    backward stable, so their difference measures the rounding floor of a
    solve, or of a whole step, at the operators' conditioning: the bar a
    third solver (the GPU's) is held to."""
    import copy
    Q = copy.copy(P)
    Q._lu = {}

    def solve_mode(kind, n, labs, rhs, trans=0):
        A = P.operator(kind, n, labs)
        return np.linalg.solve(A.T if trans else A, rhs)

    Q.solve_mode = solve_mode
    return Q


def node_jitter_twin(P, seed):
    """Copy of an oracle problem on nodes moved by independent one-ulp
    relative perturbations (walls fixed), with D1 and D2 rebuilt: every
    operator entry moves at the level of its rounding, so the twin's
    results differ from P's by the conditioning of the computation."""
    import copy
    from oracle.radial import fd_matrices
    Q = copy.copy(P)
    rng = np.random.Generator(np.random.PCG64(seed))
    r = P.r.copy()
    r[1:-1] *= 1.0 + 1.1e-16 * rng.choice([-1.0, 1.0], size=P.n_r - 2)
    Q.r = r
    Q.D1, Q.D2 = fd_matrices(r)
    Q._lu = {}
    return Q


def twin_floor(P, fn, ref, seeds=(1, 2)):
    """Rounding floor of a computation fn(problem) with result ref: the
    largest relative difference over a dense-LU twin and one-ulp node
    twins of the problem."""
    twins = [dense_twin(P)] + [node_jitter_twin(P, s) for s in seeds]
    return max(rel_l2(fn(Q), ref) for Q in twins)


def floor_tol(floor, factor=10.0, minimum=1e-14):
    """Tolerance of a parity check: a small multiple of its measured floor,
    never below a few units of double rounding."""
    return max(factor * floor, minimum)
