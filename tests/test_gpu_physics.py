"""Physics checks of the whole GPU path against what the paper reports:
the onset of wavy vortex flow and the wave speed of wavy vortices (Sec. 5.2),
the order in dt of the wall slip (Sec. 5.3), and the balance of the wall
torques (quasi-Nusselt numbers, Sec. 5.5) in a steady pattern.

Onset
-----

For eta = 0.56, Gamma = 2.2 (k_z = 2 pi / 2.2), k_theta = 1 and a resting
outer cylinder, the paper disturbs Taylor vortex flow with an n = 1 mode and
finds the Reynolds number where the energy of that mode stops decaying:
Re_i^c in [408.09, 408.1], at n_r = 64 and dt = 2e-5, confirmed by an
independent Petrov-Galerkin code.

Recipe (every step runs in the library's kernels; the test only sets up
states and takes mode energies):

1. axisymmetric Taylor vortex flow: m_theta = 1, Re_i = 408, from circular
   Couette flow plus a seeded divergence-free axisymmetric disturbance, run
   to t = 1 (the vortex energy then changes by ~3e-6 per 0.1 time units);
2. for Re_i = 408.0 and 408.2: that state in the n = 0 plane of a grid with
   m_theta = 4, a seeded divergence-free n = 1 disturbance of energy ~1e-9
   of the vortices (so that it stays linear: its n = 2 harmonic stays ~1e-12
   of it), run to t = 1.2; the growth rate sigma of the n = 1 mode is half
   the slope of log E_1 over t in [0.8, 1.2], after the transients of the
   base flow and of the disturbance have died out;
3. Re_i^c by linear interpolation of sigma between the two Reynolds numbers.

The paper gives the bracket to 0.01; the test accepts Re_i^c within 0.02 of
it (5e-5 relative), well inside the 2% by which the older literature value
differs.

Wave speed
----------
For eta = 0.868, Gamma = 2.4, k_theta = 6, Re_i = 458.1, Re_o = 0, on
(n_r, n_theta, n_z) = (32, 32, 32) physical points (m_theta = 16, m_z = 32)
and dt = 2e-5, wavy vortices are a pattern rotating rigidly at angular speed
omega; the paper gives c = omega / Omega_i = 0.34432, Omega_i = Re_i / r_i
being the inner cylinder's angular speed.  A rigidly rotating pattern has
azimuthal coefficients u_n(t) = u_n(0) exp(-i n k_theta omega t), so omega
follows from the phase of sum conj(u_1(t)) u_1(t + tau) over all radial
nodes, axial slots and components.  From Couette flow plus a seeded
disturbance the flow settles by t ~ 1.2; c is taken over two windows 0.1
apart, which must agree (a relative equilibrium).
"""
import math

import numpy as np
import pytest

import tc_inputs

pytestmark = pytest.mark.gpu

ETA, GAMMA, DT, N_R = 0.56, 2.2, 2e-5, 64
K_Z = 2 * math.pi / GAMMA
RE_LO, RE_HI = 408.0, 408.2
BASE_STEPS = 50000                       # t = 1.0
FIT_STEPS = [40000, 45000, 50000, 55000, 60000]   # t = 0.8 .. 1.2


def mode_energy(u, r, n):
    """Kinetic energy of azimuthal mode n (trapezoid rule in r dr, summed
    over axial slots; u_r^2 + u_theta^2 = (|u+|^2 + |u-|^2) / 2)."""
    import torch
    w = np.zeros_like(r)
    h = np.diff(r)
    w[:-1] += h / 2
    w[1:] += h / 2
    tw = torch.from_numpy(w * r).to(u.device)
    a = u[:, :, :, n].abs() ** 2
    return float(torch.einsum("j,js->", tw, 0.5 * (a[0] + a[1]) + a[2]))


def taylor_vortex_state(m_z):
    import torch
    from paper_1311_2481_amd import Solver
    cfg = tc_inputs.Config(n_r=N_R, m_theta=1, m_z=m_z, eta=ETA, Re_i=RE_LO, Re_o=0.0, dt=DT, amp=1e-2,
                           envelope="low4", seed=7, k_theta=1.0, k_z=K_Z, alpha=0.0)
    S = Solver(N_R, 1, m_z, ETA, RE_LO, 0.0, DT, k_z=K_Z)
    r = S.radial_nodes()
    S.set_state(torch.from_numpy(tc_inputs.initial_state(r, cfg)).to(S.device))
    S.step(BASE_STEPS - 5000)
    e_before = S.diag()["perturbation_energy"]
    S.step(5000)
    d_end = S.diag()
    base = S.get_state(with_pressure=False)
    S.close()
    return r, base, cfg, e_before, d_end


def growth_rate(Re, r, base, cfg, m_z):
    """sigma of the n = 1 mode on the given vortex state, with E_2 / E_1 at
    the end of the run."""
    import torch
    from paper_1311_2481_amd import Solver
    S = Solver(N_R, 4, m_z, ETA, Re, 0.0, DT, k_z=K_Z)
    c2 = tc_inputs.Config(cfg)
    c2["m_theta"] = 2
    d = torch.from_numpy(tc_inputs.random_direction(r, c2, 11)).to(S.device)
    u = S.zeros(3)
    u[..., 0] = base[..., 0]
    u[..., 1] = 1e-3 * d[..., 1]
    S.set_state(u)
    done, ts, logs = 0, [], []
    for k in FIT_STEPS:
        S.step(k - done)
        done = k
        st = S.get_state(with_pressure=False)
        ts.append(k * DT)
        logs.append(math.log(mode_energy(st, r, 1)))
    ratio = mode_energy(st, r, 2) / mode_energy(st, r, 1)
    assert S.check_finite()
    S.close()
    return 0.5 * np.polyfit(ts, logs, 1)[0], ratio


def critical_reynolds(m_z):
    r, base, cfg, e_before, d_end = taylor_vortex_state(m_z)
    s_lo, q_lo = growth_rate(RE_LO, r, base, cfg, m_z)
    s_hi, q_hi = growth_rate(RE_HI, r, base, cfg, m_z)
    re_c = RE_LO - s_lo * (RE_HI - RE_LO) / (s_hi - s_lo)
    return dict(re_c=re_c, sigma=(s_lo, s_hi), harmonic=(q_lo, q_hi),
                vortex_energy=(e_before, d_end["perturbation_energy"]), nu=(d_end["nu_inner"], d_end["nu_outer"]))


def test_wavy_vortex_onset_matches_paper():
    out = critical_reynolds(64)
    e_before, e_end = out["vortex_energy"]
    print(f"Taylor vortex energy at t = 0.9, 1.0: {e_before:.7e}, {e_end:.7e}; "
          f"sigma(408.0) = {out['sigma'][0]:.6f}, sigma(408.2) = {out['sigma'][1]:.6f}; "
          f"E2/E1 = {out['harmonic'][0]:.1e}, {out['harmonic'][1]:.1e}; Re_c = {out['re_c']:.4f}")
    # the vortices have formed and settled (energy changing by less than
    # 1e-5 over the last 0.1 time units), the disturbance stayed linear, and
    # the two runs straddle the onset
    assert e_end > 1e5 and abs(e_end - e_before) < 1e-5 * e_end
    # the settled vortices carry more angular momentum than laminar flow, the
    # same through both cylinders
    nu_i, nu_o = out["nu"]
    print(f"Taylor vortex flow at Re_i = {RE_LO}: Nu_omega inner {nu_i:.8f}, outer {nu_o:.8f}")
    assert nu_i > 1.05 and abs(nu_i - nu_o) < 1e-4 * nu_i
    assert max(out["harmonic"]) < 1e-9
    assert out["sigma"][0] < 0 < out["sigma"][1]
    assert 408.07 <= out["re_c"] <= 408.12


WAVE = dict(eta=0.868, Re_i=458.1, k_theta=6.0, k_z=2 * math.pi / 2.4, m_theta=16, m_z=32)
C_PAPER = 0.34432


def wavy_solver(n_r, dt):
    from paper_1311_2481_amd import Solver
    W = WAVE
    return Solver(n_r, W["m_theta"], W["m_z"], W["eta"], W["Re_i"], 0.0, dt, k_theta=W["k_theta"], k_z=W["k_z"])


def start_wavy(S):
    """Circular Couette flow plus the seeded low-mode disturbance."""
    import torch
    W = WAVE
    cfg = tc_inputs.Config(n_r=S.n_r, m_theta=W["m_theta"], m_z=W["m_z"], eta=W["eta"], Re_i=W["Re_i"], Re_o=0.0,
                           dt=S.dt, amp=1e-2, envelope="low4", seed=7, k_theta=W["k_theta"], k_z=W["k_z"], alpha=0.0)
    S.set_state(torch.from_numpy(tc_inputs.initial_state(S.radial_nodes(), cfg)).to(S.device))


def wave_speed(n_r, dt=2e-5, settle=60000, tau=500, apart=5000):
    """c from two windows [t1, t1 + tau dt], t1 = settle dt and settle dt +
    apart dt, with the |phase correlation| / energy ratio of the second."""
    import torch
    W = WAVE
    S = wavy_solver(n_r, dt)
    start_wavy(S)
    r_i = W["eta"] / (1 - W["eta"])
    out = []
    for gap in (settle, apart - tau):
        S.step(gap)
        a = S.get_state(with_pressure=False)[..., 1]
        S.step(tau)
        b = S.get_state(with_pressure=False)[..., 1]
        z = torch.sum(torch.conj(a) * b).item()
        omega = -math.atan2(z.imag, z.real) / (W["k_theta"] * tau * dt)
        out.append(omega * r_i / W["Re_i"])
    ratio = abs(z) / float((a.abs() ** 2).sum())
    diag = S.diag()
    assert S.check_finite()
    S.close()
    return out[0], out[1], ratio, diag


@pytest.mark.parametrize("n_r,tol", [(32, 3e-5), (64, 1e-5)])
def test_wavy_vortex_wave_speed_matches_paper(n_r, tol):
    c1, c2, ratio, diag = wave_speed(n_r)
    nu_i, nu_o = diag["nu_inner"], diag["nu_outer"]
    print(f"n_r = {n_r}: c = {c1:.7f}, {c2:.7f} (paper {C_PAPER}); |correlation| / energy {ratio:.8f}; "
          f"relative slip {diag['slip']:.2e}; Nu_omega inner {nu_i:.8f}, outer {nu_o:.8f}")
    # a rigidly rotating pattern: the speed is steady and the n = 1 shape
    # only turns
    assert abs(c1 - c2) < 1e-6 and abs(ratio - 1) < 1e-6
    # its theta-z mean is then steady, so the angular-velocity flux is the
    # same through every cylinder: equal torques on both walls (up to the
    # radial discretisation), above the laminar one (Sec. 5.5)
    assert nu_i > 1.05 and abs(nu_i - nu_o) < 1e-4 * nu_i
    # the phase advance per window (k_theta omega tau dt ~ 1.4 rad) is below
    # pi, so the measured speed is not aliased
    assert abs(c2 - C_PAPER) < tol


def test_wall_slip_decreases_as_dt_cubed():
    """Sec. 5.3: the projection leaves a tangential slip of order dt^3 at
    the cylinders (|grad phi|, phi = 2 dt (p^{i+1} - p*) / 3); with finite
    differences a part of order dt times the spatial error adds to it (the
    FD divergence and vector Laplacian do not commute), which the paper
    sees as the low-resolution curve levelling off.  At n_r = 128 the dt^3
    part dominates for dt >= 5e-6.  The wavy vortex state settled at
    dt = 2e-5 is restarted at each dt (u_prev = u) and the slip read after
    1000 steps, when it is steady to 1e-5 (the pattern only rotates)."""
    import torch
    S = wavy_solver(128, 2e-5)
    start_wavy(S)
    S.step(60000)
    u = S.get_state(with_pressure=False)
    S.close()
    dts, slips = (2e-5, 1e-5, 5e-6), []
    for dt in dts:
        S = wavy_solver(128, dt)
        S.set_state(u)
        S.step(1000)
        slips.append(S.diag()["slip"])
        assert S.check_finite()
        S.close()
    p = [math.log(slips[k] / slips[k + 1]) / math.log(2.0) for k in range(2)]
    print(f"relative slip at dt = {dts}: {slips}; exponents {p[0]:.2f}, {p[1]:.2f}")
    assert all(2.5 < e < 3.3 for e in p)
    assert slips[0] < 1e-8
