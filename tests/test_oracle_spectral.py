"""Pins of the oracle's pseudospectral nonlinear term (Sec. 3.2, step 1)."""
import numpy as np
import pytest

import oracle
import tc_inputs
from oracle import nonlinear as nl


def _tiny(m_theta=4, m_z=6, n_r=9):
    return oracle.Problem(n_r, m_theta, m_z, 0.5, 10.0, 0.0, 1e-3, k_theta=2.0, k_z=1.5)


def _full_spectrum(P, f):
    """Dict (l, n) -> coefficient over the full +-n range of a real field."""
    out = {}
    for s in range(P.m_z):
        if s == P.nyq:
            continue
        l = int(P.l[s])
        for n in range(P.m_theta):
            out[(l, n)] = f[s, n]
            if n > 0:
                out[(-l, -n)] = np.conj(f[s, n])
    return out


def test_transform_matches_direct_dft():
    P = _tiny()
    f = tc_inputs.random_state((P.m_z, P.m_theta), 7)
    g = nl.to_physical(P, f)
    zz = 2 * np.pi * np.arange(P.p_z) / P.p_z
    tt = 2 * np.pi * np.arange(P.p_theta) / P.p_theta
    direct = np.zeros((P.p_z, P.p_theta), dtype=complex)
    for (l, n), c in _full_spectrum(P, f).items():
        direct += c * np.exp(1j * (l * zz[:, None] + n * tt[None, :]))
    assert np.abs(direct.imag).max() < 1e-13
    np.testing.assert_allclose(g, direct.real, rtol=0, atol=1e-13)


def test_transform_roundtrip_and_parseval():
    P = oracle.Problem(8, 16, 32, 0.5, 10.0, 0.0, 1e-3)
    f = tc_inputs.random_state((3, P.m_z, P.m_theta), 11)
    g = nl.to_physical(P, f)
    np.testing.assert_allclose(nl.to_spectral(P, g), f, rtol=0, atol=1e-14)
    c = np.full(P.m_theta, 2.0)
    c[0] = 1.0
    ms_spec = np.einsum("ksn,n->k", np.abs(f) ** 2, c)
    np.testing.assert_allclose(np.mean(g ** 2, axis=(-2, -1)), ms_spec, rtol=1e-13)


def test_dealiased_product_equals_truncated_convolution():
    P = _tiny(m_theta=5, m_z=8)
    f = tc_inputs.random_state((P.m_z, P.m_theta), 3)
    g = tc_inputs.random_state((P.m_z, P.m_theta), 4)
    prod = nl.to_spectral(P, nl.to_physical(P, f) * nl.to_physical(P, g))
    F, G = _full_spectrum(P, f), _full_spectrum(P, g)
    for s in range(P.m_z):
        if s == P.nyq:
            assert prod[s].max() == 0
            continue
        l = int(P.l[s])
        for n in range(P.m_theta):
            ref = sum(cf * G.get((l - l1, n - n1), 0.0) for (l1, n1), cf in F.items())
            assert abs(prod[s, n] - ref) < 1e-13


def test_curl_exact_on_polynomial_profiles():
    # every FD row (5 to 9 points) differentiates quartics exactly, so the
    # oracle's omega must equal the analytic curl for such profiles
    P = oracle.Problem(20, 6, 8, 0.6, 10.0, 0.0, 1e-3, k_theta=3.0, k_z=0.7)
    rng = np.random.Generator(np.random.PCG64(5))
    coef = rng.standard_normal((3, 5, P.m_z, P.m_theta)) + 1j * rng.standard_normal((3, 5, P.m_z, P.m_theta))
    r = P.r
    pw = np.stack([r ** k for k in range(5)])
    dpw = np.stack([k * r ** (k - 1) if k else 0 * r for k in range(5)])
    ur, ut, uz = (np.einsum("kj,ksn->jsn", pw, coef[c]) for c in range(3))
    dut, duz = (np.einsum("kj,ksn->jsn", dpw, coef[c]) for c in (1, 2))
    u = np.stack([ur + 1j * ut, ur - 1j * ut, uz])
    a, b, rr = P.bcast()
    exact = (1j * a * uz / rr - 1j * b * ut, 1j * b * ur - duz, dut + ut / rr - 1j * a * ur / rr)
    got = nl.vorticity(P, u)
    for e, g in zip(exact, got):
        np.testing.assert_allclose(g, e, rtol=0, atol=1e-10 * np.abs(e).max())


def _plane_work(P, u, N):
    c = np.full(P.m_theta, 2.0)
    c[0] = 1.0
    dens = 0.5 * (np.conj(u[0]) * N[0] + np.conj(u[1]) * N[1]) + np.conj(u[2]) * N[2]
    return np.einsum("n,jsn->j", c, dens.real)


@pytest.mark.parametrize("seed", [1, 2])
def test_energy_neutrality(seed):
    # int u.(omega x u) = 0 holds exactly on every radial node because the
    # 3/2 rule keeps the retained coefficients of the product exact
    cfg = dict(tc_inputs.CONFIGS["small"])
    cfg["envelope"] = "k53"
    cfg["seed"] = seed
    cfg["amp"] = 0.3
    P = oracle.Problem(cfg["n_r"], cfg["m_theta"], cfg["m_z"], cfg["eta"], cfg["Re_i"], cfg["Re_o"], cfg["dt"])
    u = tc_inputs.initial_state(P.r, cfg)
    N = oracle.nonlinear_rot(P, u)
    w = _plane_work(P, u, N)
    assert np.abs(w).max() <= 1e-13 * np.linalg.norm(u) * np.linalg.norm(N)
    # a planted error (u_theta component dropped from N_r) breaks it
    U = nl.to_physical(P, np.stack(nl.cylindrical(u)))
    W = nl.to_physical(P, np.stack(nl.vorticity(P, u)))
    S = nl.to_spectral(P, np.stack([W[1] * U[2], W[2] * U[0] - W[0] * U[2], W[0] * U[1] - W[1] * U[0]]))
    bad = _plane_work(P, u, nl.plus_minus(*S))
    assert np.abs(bad).max() > 1e-6 * np.linalg.norm(u) * np.linalg.norm(N)


def test_rotational_matches_convective_up_to_bernoulli_gradient():
    # u.grad u = omega x u + grad(|u|^2/2); discretely the difference is FD
    # error, which must shrink at high order as n_r grows
    errs = []
    for n_r in (24, 48):
        cfg = dict(tc_inputs.CONFIGS["small"])
        cfg.update(n_r=n_r, amp=0.2, m_theta=8, m_z=8)
        P = oracle.Problem(n_r, 8, 8, cfg["eta"], cfg["Re_i"], cfg["Re_o"], cfg["dt"])
        u = tc_inputs.initial_state(P.r, cfg)
        K = nl.kinetic_density(P, u)
        from oracle.scheme import grad
        diff = nl.nonlinear_conv(P, u) - nl.nonlinear_rot(P, u) - grad(P, K)
        errs.append(np.abs(diff).max() / np.abs(nl.nonlinear_conv(P, u)).max())
    assert errs[1] < errs[0] / 2 ** 6, errs
    assert errs[1] < 1e-4


def test_single_plane_nonlinear_matches_full():
    # the per-node evaluation (used for sampled parity at full size) is the
    # same computation restricted to one radial node
    cfg = dict(tc_inputs.CONFIGS["small"])
    cfg.update(amp=0.2, envelope="k53")
    P = oracle.Problem(cfg["n_r"], cfg["m_theta"], cfg["m_z"], cfg["eta"], cfg["Re_i"], cfg["Re_o"], cfg["dt"])
    u = tc_inputs.initial_state(P.r, cfg)
    full = oracle.nonlinear_rot(P, u)
    for j in (0, 2, 15, P.n_r - 1):
        lo, hi = max(0, j - 4), min(P.n_r - 1, j + 4)
        Nj = nl.nonlinear_rot_at(P, u[:, lo:hi + 1], j)
        np.testing.assert_allclose(Nj, full[:, j], rtol=0, atol=1e-12 * np.abs(full).max())


def test_energy_matches_physical_space_quadrature():
    """Kinetic energy from the spectral formula (Parseval with c_n weights,
    +- components) equals 1/2 sum_j w_j r_j * mean over an explicit (theta, z)
    grid of u_r^2 + u_theta^2 + u_z^2 times the box area, with the physical
    values summed term by term from the coefficients."""
    from oracle import diagnostics as dg
    P = _tiny(m_theta=3, m_z=4, n_r=7)
    u = tc_inputs.random_state((3, P.n_r, P.m_z, P.m_theta), 21)
    # u_r = (u+ + u-)/2, u_theta = -i (u+ - u-)/2 are real fields: their
    # coefficients must obey the n = 0 symmetry for the comparison to hold
    up, um = u[0].copy(), u[1].copy()
    ur_c, ut_c = (up + um) / 2, -0.5j * (up - um)
    for c in (ur_c, ut_c):
        for s in range(1, P.m_z):
            if s != P.nyq:
                c[:, P.m_z - s, 0] = np.conj(c[:, s, 0])
        c[:, 0, 0] = c[:, 0, 0].real
    u = np.stack([ur_c + 1j * ut_c, ur_c - 1j * ut_c, u[2]])
    nt, nz = 2 * P.m_theta + 1, P.m_z + 1          # enough points for exact quadrature of squares
    th = 2 * np.pi / P.k_theta * np.arange(nt) / nt
    z = 2 * np.pi / P.k_z * np.arange(nz) / nz

    def values(c):
        g = np.zeros((P.n_r, nz, nt))
        spec = {}
        for s in range(P.m_z):
            if s == P.nyq:
                continue
            for n in range(P.m_theta):
                spec[(int(P.l[s]), n)] = c[:, s, n]
        for (l, n), v in spec.items():
            ph = np.exp(1j * (n * P.k_theta * th[None, :] + l * P.k_z * z[:, None]))
            term = v[:, None, None] * ph[None]
            g += term.real if n == 0 else 2 * term.real
        return g

    comp = [values(ur_c), values(ut_c), values(u[2])]
    ms = sum((g ** 2).mean(axis=(1, 2)) for g in comp)
    area = (2 * np.pi / P.k_theta) * (2 * np.pi / P.k_z)
    w = np.zeros(P.n_r)
    h = np.diff(P.r)
    w[:-1] += h / 2
    w[1:] += h / 2
    ref = 0.5 * area * np.sum(w * P.r * ms)
    assert abs(dg.energy(P, u) - ref) <= 1e-13 * ref


def _physical_cfl(P, u):
    """dt max over the nodes and an explicit (P_z, P_theta) grid of
    |u_r|/dr_j + |u_theta|/(r_j dtheta) + |u_z|/dz, the values synthesised
    from the coefficients by inverse FFTs."""
    import scipy.fft as sfft
    ur, ut, uz = nl.cylindrical(u)

    def phys(f):
        return sfft.irfft2(nl._pad(P, f), s=(P.p_z, P.p_theta), axes=(-2, -1), norm="forward")
    h = np.diff(P.r)
    dr = np.minimum(np.concatenate([h, [np.inf]]), np.concatenate([[np.inf], h]))
    dth = 2 * np.pi / (P.k_theta * 2 * P.m_theta)
    dz = 2 * np.pi / (P.k_z * P.m_z)
    rate = (np.abs(phys(ur)) / dr[:, None, None] + np.abs(phys(ut)) / (P.r * dth)[:, None, None]
            + np.abs(phys(uz)) / dz)
    return P.dt * rate.max()


def test_cfl_bound_is_an_upper_bound():
    # the mode-sum bound can only overestimate the physical-grid value, and
    # for a smooth low-mode state it stays within a small factor of it
    from oracle import diagnostics as dg
    cfg = dict(tc_inputs.CONFIGS["small"])
    P = oracle.Problem(cfg["n_r"], cfg["m_theta"], cfg["m_z"], cfg["eta"], cfg["Re_i"], cfg["Re_o"], cfg["dt"])
    u = tc_inputs.initial_state(P.r, dict(cfg, amp=0.2))
    b, c = dg.cfl_bound(P, u), _physical_cfl(P, u)
    assert c <= b * (1 + 1e-12) and b < 3 * c


def test_cfl_bound_exact_for_one_aligned_mode():
    # Couette flow plus u_theta = 2 A(r) cos(k_z z) (slots l = +-1, n = 0,
    # A > 0): u_r = u_z = 0 and the largest |u_theta| on every node, at
    # z = 0, is U + 2A, which is exactly the mode sum
    from oracle import diagnostics as dg
    P = oracle.Problem(17, 3, 8, 0.5, 40.0, 0.0, 1e-3, k_theta=2.0, k_z=1.5)
    u = dg.couette_state(P)
    A = 3.0 + np.sin(P.r)
    for s in (1, P.m_z - 1):
        u[0, :, s, 0] = 1j * A
        u[1, :, s, 0] = -1j * A
    b, c = dg.cfl_bound(P, u), _physical_cfl(P, u)
    assert abs(b - c) <= 1e-13 * c


def test_quasi_nusselt_of_couette_flow_tends_to_one():
    # circular Couette flow is the laminar reference, so both cylinders give
    # Nu = 1 up to the error of the 5-point wall rows of D1, which is
    # O(h^4) in the wall spacing h
    from oracle import diagnostics as dg
    errs, hs = [], []
    for n_r in (17, 33, 65):
        P = oracle.Problem(n_r, 2, 4, 0.5, 100.0, -30.0, 1e-3)
        nu = dg.quasi_nusselt(P, dg.couette_state(P))
        errs.append(max(abs(nu[0] - 1.0), abs(nu[1] - 1.0)))
        hs.append(P.r[1] - P.r[0])
    orders = [np.log(errs[k] / errs[k + 1]) / np.log(hs[k] / hs[k + 1]) for k in range(2)]
    assert errs[-1] < 1e-9 and min(orders) > 3.5


def test_quasi_nusselt_exact_for_quartic_angular_velocity():
    # <u_theta> = r q(r) with q quartic: the wall rows of D1 (5 points) are
    # exact on it, so Nu at each wall is -r^3 q'(r) / (2 C2) to rounding.
    # A radial mean flow and every other mode must not enter.
    from oracle import diagnostics as dg
    P = oracle.Problem(21, 3, 6, 0.6, 80.0, 25.0, 1e-3)
    c = np.array([0.7, -1.3, 0.4, 2.1, -0.9])             # q(x) = sum c_k x^k, x = r - r_i
    x = P.r - P.r[0]
    q = np.polyval(c[::-1], x)
    dq = np.polyval((c[1:] * np.arange(1, 5))[::-1], x)
    u = tc_inputs.random_state((3, P.n_r, P.m_z, P.m_theta), 19)
    ur = np.cos(P.r)                                       # a radial (0, 0) component
    u[0, :, 0, 0] = ur + 1j * P.r * q
    u[1, :, 0, 0] = ur - 1j * P.r * q
    C2 = P.eta * (P.Re_i - P.eta * P.Re_o) / ((1 - P.eta) * (1 - P.eta ** 2))
    want = -P.r ** 3 * dq / (2 * C2)
    got = dg.quasi_nusselt(P, u)
    assert abs(got[0] - want[0]) <= 1e-11 * abs(want[0])
    assert abs(got[1] - want[-1]) <= 1e-11 * abs(want[-1])
    # no laminar torque (C2 = 0 on Re_i = eta Re_o): undefined
    Q = oracle.Problem(9, 1, 2, 0.5, 10.0, 20.0, 1e-3)
    assert all(np.isnan(dg.quasi_nusselt(Q, dg.couette_state(Q))))


def _physical_values(P, c, th, z):
    """Real field values on an explicit (z, theta) grid from its stored
    coefficients c[s, n], summed term by term (the n < 0 half is the
    conjugate of the stored one)."""
    g = np.zeros((len(z), len(th)))
    for s in range(P.m_z):
        if s == P.nyq:
            continue
        for n in range(P.m_theta):
            ph = np.exp(1j * (n * P.k_theta * th[None, :] + P.l[s] * P.k_z * z[:, None]))
            term = c[s, n] * ph
            g += term.real if n == 0 else 2 * term.real
    return g


def _hermitian_velocity(P, seed):
    """Random velocity whose cylindrical components are real fields."""
    u = tc_inputs.random_state((3, P.n_r, P.m_z, P.m_theta), seed)
    ur_c, ut_c, uz_c = (u[0] + u[1]) / 2, -0.5j * (u[0] - u[1]), u[2].copy()
    for c in (ur_c, ut_c, uz_c):
        for s in range(1, P.m_z):
            if s != P.nyq:
                c[:, P.m_z - s, 0] = np.conj(c[:, s, 0])
        c[:, 0, 0] = c[:, 0, 0].real
        c[:, P.nyq, :] = 0.0
    return np.stack([ur_c + 1j * ut_c, ur_c - 1j * ut_c, uz_c]), ut_c, uz_c


@pytest.mark.parametrize("wall", [0, 1])
def test_wall_slip_matches_physical_space_quadrature(wall):
    """Relative wall slip from the spectral formula equals
    sqrt(mean((u_theta - Re)^2 + u_z^2)) / |Re| with the mean taken over an
    explicit (theta, z) grid at the wall, the values synthesised term by
    term from the coefficients (enough points to integrate squares of the
    stored modes exactly)."""
    from oracle import diagnostics as dg
    P = oracle.Problem(9, 3, 6, 0.6, 7.0, -3.0, 1e-3, k_theta=2.0, k_z=1.5)
    u, ut_c, uz_c = _hermitian_velocity(P, 31)
    j = 0 if wall == 0 else -1
    Re = P.Re_i if wall == 0 else P.Re_o
    # add the wall speed to the mean azimuthal velocity so that the slip is
    # a small difference of large values, as in a real state
    u[0, j, 0, 0] += 1j * Re
    u[1, j, 0, 0] -= 1j * Re
    ut_c = -0.5j * (u[0] - u[1])
    nt, nz = 2 * P.m_theta + 1, P.m_z + 1
    th = 2 * np.pi / P.k_theta * np.arange(nt) / nt
    z = 2 * np.pi / P.k_z * np.arange(nz) / nz
    ut = _physical_values(P, ut_c[j], th, z)
    uz = _physical_values(P, uz_c[j], th, z)
    want = np.sqrt(np.mean((ut - Re) ** 2 + uz ** 2)) / abs(Re)
    got = dg.wall_slip(P, u, wall=wall)
    assert abs(got - want) <= 1e-13 * want


def test_wall_slip_closed_form_of_single_modes():
    """u_theta = Re_i + e1 cos(l k_z z) and u_z = e2 cos(n k_theta theta) at
    r_i: the mean squares are e1^2/2 and e2^2/2, so the slip is
    sqrt((e1^2 + e2^2)/2) / Re_i.  u_r and the outer wall do not enter."""
    from oracle import diagnostics as dg
    P = oracle.Problem(9, 4, 8, 0.5, 20.0, 5.0, 1e-3)
    u = dg.couette_state(P)
    e1, e2 = 0.3, 0.7
    # u_theta: slots l = +-2 at n = 0 carry e1/2 each (u+- = +-i u_theta)
    for s in (2, P.m_z - 2):
        u[0, 0, s, 0] += 1j * e1 / 2
        u[1, 0, s, 0] -= 1j * e1 / 2
    # u_z: n = 3, l = 0 carries e2/2 (its conjugate n = -3 is implied)
    u[2, 0, 0, 3] = e2 / 2
    # a radial velocity at the wall and anything at the other wall are ignored
    u[0, 0, 1, 1] += 0.4
    u[1, 0, 1, 1] += 0.4
    u[:, -1] += 5.0
    assert abs(dg.wall_slip(P, u) - np.sqrt((e1 ** 2 + e2 ** 2) / 2) / P.Re_i) <= 1e-14
