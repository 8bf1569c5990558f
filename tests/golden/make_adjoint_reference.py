"""Write the FP64 oracle reference for the gradient of the differentiation
workload.

Runs only oracle/ and tc_inputs: N_r = 64, 128 x 128 physical, eta = 0.71,
Re_i = 1000, Re_o = 0, perturbation 1e-3 with a k^-5/3 envelope (seed 5),
dt and T from the workload (T steps, checkpoints every 20), the objective
J = E_pert(u^T) from u^0 = Couette + perturbation (history u^{-1} = u^0,
N^{-1} = N(u^0)), and its gradient g = dJ/du^0 by the oracle's
checkpointed discrete adjoint.

Output: adjoint_reference.txt with J, the projections <g, v_k> on the 8
seeded divergence-free directions v_k (seeds 1000..1007, the ones the
finite-difference check uses), |g|, and 256 sampled coefficients of g at
fixed (seeded) positions.

    python tests/golden/make_adjoint_reference.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import tc_inputs  # noqa: E402
from oracle import adjoint as adj  # noqa: E402

NSAMPLE = 256
DIRECTIONS = range(1000, 1008)


def sample_positions(shape, n=NSAMPLE, seed=5151):
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.integers(0, shape[0], n)
    j = rng.integers(0, shape[1], n)
    s = rng.integers(0, shape[2], n)
    s = np.where(s == shape[2] // 2, 0, s)
    k = rng.integers(0, shape[3], n)
    return c, j, s, k


def main():
    cfg = tc_inputs.Config(tc_inputs.CONFIGS["adjoint"])
    P = oracle.Problem(cfg.n_r, cfg.m_theta, cfg.m_z, cfg.eta, cfg.Re_i, cfg.Re_o, cfg.dt,
                       k_theta=cfg.k_theta, k_z=cfg.k_z, alpha=cfg.alpha)
    u0 = tc_inputs.initial_state(P.r, cfg)
    J, g = adj.gradient(P, u0, cfg.steps, cfg.checkpoint_every)
    proj = [adj.inner(g, tc_inputs.random_direction(P.r, cfg, seed)) for seed in DIRECTIONS]
    c, j, s, k = sample_positions(g.shape)
    out = os.path.join(HERE, "adjoint_reference.txt")
    with open(out, "w") as fh:
        fh.write(f"# FP64 oracle gradient of E_pert(u^T), T = {cfg.steps} steps, dt = {cfg.dt:g}, "
                 f"differentiation workload (see make_adjoint_reference.py)\n")
        fh.write(f"J = {J:.17e}\n")
        fh.write(f"grad_norm = {np.sqrt(adj.inner(g, g)):.17e}\n")
        for seed, p in zip(DIRECTIONS, proj):
            fh.write(f"proj_{seed} = {p:.17e}\n")
        fh.write("# c j s n re im\n")
        for a, b, e, f in zip(c, j, s, k):
            v = g[a, b, e, f]
            fh.write(f"{a} {b} {e} {f} {v.real:.17e} {v.imag:.17e}\n")
    print(f"wrote {out}: J = {J:.6e}")


if __name__ == "__main__":
    main()
