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
