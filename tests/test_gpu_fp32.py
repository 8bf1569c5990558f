"""FP32-bulk form: transforms and products in float, solves and state in
double.  Checked against the FP64 oracle."""
import os

import numpy as np
import pytest

import oracle
import tc_inputs
from oracle import diagnostics as dg
from oracle import scheme
from gpu_common import make_pair, rel_l2, to_dev, to_host

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fp32_reference_medium.txt")


@pytest.mark.parametrize("name", ["small", "medium"])
def test_fp32_nonlinear_and_step(name):
    S, P, cfg = make_pair(name, "fp32_bulk")
    u0 = tc_inputs.initial_state(P.r, cfg)
    N = to_host(S.nonlinear(to_dev(u0)))
    ref = oracle.nonlinear_rot(P, u0)
    err = rel_l2(N, ref)
    # energy neutrality holds to float rounding
    c = np.full(cfg.m_theta, 2.0)
    c[0] = 1.0
    dens = 0.5 * (np.conj(u0[0]) * N[0] + np.conj(u0[1]) * N[1]) + np.conj(u0[2]) * N[2]
    work = np.abs(np.einsum("n,jsn->j", c, dens.real)).max() / (np.linalg.norm(u0) * np.linalg.norm(N))
    S.set_state(to_dev(u0), None, to_dev(ref))
    S.step(1)
    ug = to_host(S.get_state(with_pressure=False))
    ur, _, _ = scheme.step(P, u0, u0, ref)
    serr = rel_l2(ug, ur)
    print(f"{name} fp32-bulk: nonlinear rel_l2={err:.3e}, neutrality={work:.2e}, one step rel_l2={serr:.3e}")
    assert err < 2e-6
    assert work < 1e-6
    assert serr < 1e-7
    S.close()


def _golden():
    vals, pos = {}, []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        if "=" in line:
            k, v = line.split("=")
            vals[k.strip()] = float(v)
        else:
            p = line.split()
            pos.append(tuple(int(x) for x in p[:4]) + (float(p[4]) + 1j * float(p[5]),))
    return vals, pos


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="oracle reference not generated")
def test_fp32_bulk_500_steps_against_oracle():
    # medium grid at a stable dt = 1e-5 (the nominal 2e-4 overflows): the FP64
    # GPU trajectory must reproduce the oracle's sampled coefficients; the
    # FP32-bulk trajectory's error is stated against the same reference
    vals, pos = _golden()
    out = {}
    for prec in ("fp64", "fp32_bulk"):
        S, P, cfg = make_pair("medium_fp32", prec, dt=1e-5)
        S.set_state(to_dev(tc_inputs.initial_state(P.r, cfg)))
        S.step(500)
        u = to_host(S.get_state(with_pressure=False))
        S.close()
        got = np.array([u[c, j, s, n] for c, j, s, n, _ in pos])
        ref = np.array([v for *_, v in pos])
        pert = u - dg.couette_state(P)
        out[prec] = dict(u=u, sample_err=np.linalg.norm(got - ref) / np.linalg.norm(ref),
                         E=dg.energy(P, u), Ep=dg.perturbation_energy(P, u), pnorm=np.linalg.norm(pert))
    f64, f32 = out["fp64"], out["fp32_bulk"]
    field = np.linalg.norm(f32["u"] - f64["u"]) / np.linalg.norm(f64["u"])
    pfield = np.linalg.norm(f32["u"] - f64["u"]) / f64["pnorm"]
    eerr = abs(f32["E"] - vals["energy"]) / vals["energy"]
    perr = abs(f32["Ep"] - vals["perturbation_energy"]) / vals["perturbation_energy"]
    print(f"500 steps: fp64 sample err {f64['sample_err']:.2e}, fp64 Ep err "
          f"{abs(f64['Ep'] - vals['perturbation_energy']) / vals['perturbation_energy']:.2e}; fp32-bulk: "
          f"sample err {f32['sample_err']:.2e}, field err vs fp64 {field:.2e} (perturbation-relative {pfield:.2e}), "
          f"kinetic energy err {eerr:.2e}, perturbation energy err {perr:.2e}")
    assert f64["sample_err"] < 1e-10
    assert abs(f64["Ep"] - vals["perturbation_energy"]) / vals["perturbation_energy"] < 1e-10
    assert f32["sample_err"] < 1e-5 and eerr < 1e-6 and perr < 1e-4
