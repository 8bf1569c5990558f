"""Write the FP64 oracle reference for the FP32-bulk error statement.

Runs the oracle (only oracle/ and tc_inputs are used) for 500 steps on the
medium grid (N_r = 64, 128 x 128 physical, eta = 0.71, Re_i = 1000,
Re_o = -500, perturbation 1e-2 with a k^-5/3 envelope, seed 2) at
dt = 1e-5.  The workload's nominal dt = 2e-4 is far above the advective
stability limit (the oracle's fields overflow within ~15 steps there), so
the error statement is made at a stable step.

Output: fp32_reference_medium.txt with the final kinetic and perturbation
energies, the norm of the perturbation, and 512 sampled coefficients of
the final velocity at fixed (seeded) positions.

    python tests/golden/make_fp32_reference.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import tc_inputs  # noqa: E402
from oracle import diagnostics as dg  # noqa: E402
from oracle import scheme  # noqa: E402

DT = 1e-5
STEPS = 500
NSAMPLE = 512


def sample_positions(shape, n=NSAMPLE, seed=4242):
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.integers(0, shape[0], n)
    j = rng.integers(0, shape[1], n)
    s = rng.integers(0, shape[2], n)
    s = np.where(s == shape[2] // 2, 0, s)
    k = rng.integers(0, shape[3], n)
    return c, j, s, k


def main():
    cfg = tc_inputs.Config(tc_inputs.CONFIGS["medium_fp32"])
    P = oracle.Problem(cfg.n_r, cfg.m_theta, cfg.m_z, cfg.eta, cfg.Re_i, cfg.Re_o, DT)
    u0 = tc_inputs.initial_state(P.r, cfg)
    u, _, _, _ = scheme.run(P, u0, STEPS)
    pos = sample_positions(u.shape)
    vals = u[pos]
    pert = u - dg.couette_state(P)
    with open(os.path.join(HERE, "fp32_reference_medium.txt"), "w") as fh:
        fh.write("# FP64 oracle after %d steps, dt = %g, medium grid (see make_fp32_reference.py)\n" % (STEPS, DT))
        fh.write("energy = %.17e\n" % dg.energy(P, u))
        fh.write("perturbation_energy = %.17e\n" % dg.perturbation_energy(P, u))
        fh.write("perturbation_norm = %.17e\n" % np.linalg.norm(pert))
        fh.write("# c j s n re im\n")
        for i in range(len(vals)):
            fh.write("%d %d %d %d %.17e %.17e\n" % (pos[0][i], pos[1][i], pos[2][i], pos[3][i], vals[i].real, vals[i].imag))


if __name__ == "__main__":
    main()
