"""Wall torque of turbulent flow at Re_i = 8000 (Sec. 5.5), with the paper's
convective form: eta = 0.5, outer cylinder at rest, Gamma = pi (k_z = 2),
k_theta = 2, (n_r, n_theta, n_z) = (128, 192, 320) physical points
(m_theta = 96, m_z = 320 stored modes, 288 x 480 dealiased), Chebyshev
nodes (alpha -> 0), dt = 2e-7.  The paper's quasi-Nusselt number converges
to 8.815 at this resolution (8.81 +- 0.05 over alpha = 0, 0.5, 0.99).

The run starts from Couette flow with a seeded perturbation, lets the
turbulence develop for 50 000 steps (t = 0.01) and averages Nu_omega at
both cylinders over the next 250 000 (t = 0.01 ... 0.06), sampled every
1000 steps.  About 11 minutes on one MI355X, so it runs only when
TC_LONG_PHYSICS=1 is set.
"""
import os

import numpy as np
import pytest

import tc_inputs

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(os.environ.get("TC_LONG_PHYSICS") != "1",
                                 reason="11-minute run: set TC_LONG_PHYSICS=1")]


def test_turbulent_torque_matches_paper():
    from paper_1311_2481_amd import Solver
    cfg = tc_inputs.Config(n_r=128, m_theta=96, m_z=320, eta=0.5, Re_i=8000.0, Re_o=0.0, dt=2e-7,
                           amp=0.05, envelope="k53", seed=8, k_theta=2.0, k_z=2.0, alpha=0.0)
    S = Solver(cfg.n_r, cfg.m_theta, cfg.m_z, cfg.eta, cfg.Re_i, cfg.Re_o, cfg.dt,
               k_theta=cfg.k_theta, k_z=cfg.k_z, form="conv")
    try:
        assert (S.m_theta, S.m_z) == (96, 320)
        S.set_state(tc_inputs.initial_state(S.radial_nodes(), cfg, device="cuda"))
        transient, total, every = 50_000, 300_000, 1000
        nu_i, nu_o = [], []
        done = 0
        while done < total:
            S.step(every)
            done += every
            d = S.diag()
            assert np.isfinite(d["energy"]), f"not finite at step {done}"
            if done > transient:
                nu_i.append(d["nu_inner"])
                nu_o.append(d["nu_outer"])
            if done % 10_000 == 0:
                print(f"step {done} t={done * cfg.dt:.4f}: Nu_omega inner {d['nu_inner']:.4f}, "
                      f"outer {d['nu_outer']:.4f}, CFL bound {d['cfl']:.2f}", flush=True)
        nu_i, nu_o = np.array(nu_i), np.array(nu_o)
        # standard errors from 10 blocks of consecutive samples
        blk = lambda x: np.std([b.mean() for b in np.array_split(x, 10)], ddof=1) / np.sqrt(10)
        mi, mo = nu_i.mean(), nu_o.mean()
        print(f"Nu_omega over t = {transient * cfg.dt:.3f}..{total * cfg.dt:.3f}: inner {mi:.4f} +- {blk(nu_i):.4f}, "
              f"outer {mo:.4f} +- {blk(nu_o):.4f}, both {0.5 * (mi + mo):.4f} (paper: 8.815)")
        assert abs(mi - 8.815) < 0.2 and abs(mo - 8.815) < 0.2
    finally:
        S.close()
