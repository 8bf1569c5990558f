"""Seeded synthetic inputs for the Taylor-Couette step (shared by tests and benchmark).

This module builds input states only.  It holds none of the method's
arithmetic (no finite differences, transforms or solves): radial
derivatives of the synthetic fields are taken analytically from their
polynomial profiles, and the radial nodes are supplied by the caller.

Initial state = circular Couette flow (closed form, Sec. 5.1 of the paper)
plus a divergence-free perturbation u' = curl A with

    A_c(r; l, n) = g(r) sum_{q=0..3} a_{c,q,l,n} T_q(xi),
    g = 16 (r - r_i)^2 (r_o - r)^2,   xi = 2 (r - r_i) - 1   (gap d = 1),

a ~ CN(0, 1) x envelope(l, n) drawn from numpy's PCG64(seed).  g and g'
vanish at both walls, so u' = 0 there.  Envelopes: "low4" is 1 for n <= 3,
|l| <= 3 and 0 elsewhere; "k53" is (1 + |k|)^(-5/3) with
|k| = sqrt((n k_theta)^2 + (l k_z)^2).  Mode (0,0) and the Nyquist slot
are excluded, and the n = 0 coefficients satisfy a(-l) = conj(a(l)) so the
field is real.  The perturbation is scaled so that its volume RMS equals
amp * |Re_i| (trapezoid weights in r).

Layout: complex128 (3, n_r, m_z, m_theta) holding (u+, u-, u_z),
u+- = u_r +- i u_theta; axial slot s holds l = s (s < m_z/2) or s - m_z.
"""
import numpy as np

__all__ = ["Config", "CONFIGS", "perturbation_coefficients", "initial_state",
           "random_state", "random_field_torch", "random_direction"]


class Config(dict):
    __getattr__ = dict.__getitem__


# The five workloads: small (oracle-sized), medium, production size for one
# GPU, the FP32-bulk form of the medium case and the differentiation case.
CONFIGS = {
    "small": Config(n_r=32, m_theta=16, m_z=32, eta=0.5, Re_i=100.0, Re_o=0.0, dt=1e-3,
                    steps=20, amp=1e-3, envelope="low4", seed=1),
    "medium": Config(n_r=64, m_theta=64, m_z=128, eta=0.71, Re_i=1000.0, Re_o=-500.0, dt=2e-4,
                     steps=200, amp=1e-2, envelope="k53", seed=2),
    "production": Config(n_r=512, m_theta=512, m_z=1024, eta=0.5, Re_i=1e4,
                         Re_o=1e4 * 0.5 ** 1.5, dt=5e-5, steps=50, amp=0.1, envelope="k53", seed=3),
    "medium_fp32": Config(n_r=64, m_theta=64, m_z=128, eta=0.71, Re_i=1000.0, Re_o=-500.0,
                          dt=2e-4, steps=500, amp=1e-2, envelope="k53", seed=2),
    # dt: no step is given for this workload; 5e-7 lies below the rotational
    # form's limit for it (mode (n, l) = (1, 0) grows from about 1e-6 on)
    "adjoint": Config(n_r=64, m_theta=64, m_z=128, eta=0.71, Re_i=1000.0, Re_o=0.0, dt=5e-7,
                      steps=400, amp=1e-3, envelope="k53", seed=5, checkpoint_every=20),
}
for _c in CONFIGS.values():
    _c.setdefault("k_theta", 1.0)
    _c.setdefault("k_z", 1.0)
    _c.setdefault("alpha", 0.0)


def _slot_l(m_z):
    s = np.arange(m_z)
    return np.where(s < m_z // 2, s, s - m_z)


def _envelope(kind, m_theta, m_z, k_theta, k_z):
    n = np.arange(m_theta)[None, :]
    l = _slot_l(m_z)[:, None]
    if kind == "low4":
        env = ((n <= 3) & (np.abs(l) <= 3)).astype(np.float64)
    elif kind == "k53":
        k = np.sqrt((n * k_theta) ** 2 + (l * k_z) ** 2)
        env = (1.0 + k) ** (-5.0 / 3.0)
    else:
        raise ValueError(kind)
    env = env.copy()
    env[0, 0] = 0.0
    env[m_z // 2, :] = 0.0
    return env


def perturbation_coefficients(m_theta, m_z, envelope, seed, k_theta=1.0, k_z=1.0):
    """Random vector-potential coefficients a[c, q, slot, n] (complex128)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (3, 4, m_z, m_theta)
    a = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)
    a *= _envelope(envelope, m_theta, m_z, k_theta, k_z)[None, None]
    # real field: n = 0 coefficients Hermitian in l
    h = m_z // 2
    a[:, :, 0, 0] = a[:, :, 0, 0].real
    a[:, :, m_z - np.arange(1, h), 0] = np.conj(a[:, :, np.arange(1, h), 0])
    return a


def _radial_basis(r, r_i, r_o):
    """g T_q(xi) and its r-derivative at the nodes, shape (n_r, 4) each."""
    xi = 2.0 * (r - r_i) - 1.0
    T = np.stack([np.ones_like(xi), xi, 2 * xi ** 2 - 1, 4 * xi ** 3 - 3 * xi], 1)
    dT = np.stack([np.zeros_like(xi), np.ones_like(xi), 4 * xi, 12 * xi ** 2 - 3], 1) * 2.0
    g = 16.0 * (r - r_i) ** 2 * (r_o - r) ** 2
    dg = 32.0 * (r - r_i) * (r_o - r) ** 2 - 32.0 * (r - r_i) ** 2 * (r_o - r)
    return g[:, None] * T, dg[:, None] * T + g[:, None] * dT


def _torch():
    import torch
    return torch


def initial_state(r, cfg, device=None, with_couette=True):
    """Perturbed circular Couette state for config ``cfg`` on nodes ``r``.

    Returns a numpy array when ``device`` is None, else a torch tensor on
    ``device`` (the assembly is then done there; large configurations
    need this).
    """
    r = np.asarray(r, dtype=np.float64)
    eta = cfg["eta"]
    r_i, r_o = eta / (1 - eta), 1 / (1 - eta)
    m_theta, m_z = cfg["m_theta"], cfg["m_z"]
    a = perturbation_coefficients(m_theta, m_z, cfg["envelope"], cfg["seed"],
                                  cfg.get("k_theta", 1.0), cfg.get("k_z", 1.0))
    B, dB = _radial_basis(r, r_i, r_o)
    kn = np.arange(m_theta) * cfg.get("k_theta", 1.0)
    kl = _slot_l(m_z) * cfg.get("k_z", 1.0)
    w = np.zeros_like(r)
    h = np.diff(r)
    w[:-1] += h / 2
    w[1:] += h / 2
    cn = np.full(m_theta, 2.0)
    cn[0] = 1.0
    C1 = (cfg["Re_o"] - eta * cfg["Re_i"]) / (1.0 + eta)
    C2 = eta * (cfg["Re_i"] - eta * cfg["Re_o"]) / ((1.0 - eta) * (1.0 - eta ** 2))
    U = C1 * r + C2 / r

    if device is None:
        xp_B, xp_dB, A = B, dB, a
        ein = np.einsum
        rr = r[:, None, None]
        an, bl = kn[None, None, :], kl[None, :, None]
        Ar, At, Az = (ein("jq,qsn->jsn", xp_B, A[c]) for c in range(3))
        dAt, dAz = (ein("jq,qsn->jsn", xp_dB, A[c]) for c in (1, 2))
        ur = 1j * an * Az / rr - 1j * bl * At
        ut = 1j * bl * Ar - dAz
        uz = dAt + At / rr - 1j * an * Ar / rr
        ms = np.einsum("j,jsn,n->", w * r, np.abs(ur) ** 2 + np.abs(ut) ** 2 + np.abs(uz) ** 2, cn)
        scale = cfg["amp"] * abs(cfg["Re_i"]) / np.sqrt(ms / np.sum(w * r))
        u = np.stack([ur + 1j * ut, ur - 1j * ut, uz]) * scale
        if with_couette:
            u[0, :, 0, 0] += 1j * U
            u[1, :, 0, 0] -= 1j * U
        return u

    torch = _torch()
    dev = torch.device(device)
    tB = torch.from_numpy(B).to(dev, torch.complex128)
    tdB = torch.from_numpy(dB).to(dev, torch.complex128)
    ta = torch.from_numpy(a).to(dev)
    rr = torch.from_numpy(r).to(dev)[:, None, None]
    an = torch.from_numpy(kn).to(dev)[None, None, :]
    bl = torch.from_numpy(kl.astype(np.float64)).to(dev)[None, :, None]

    def prof(basis, c):
        return torch.einsum("jq,qsn->jsn", basis, ta[c].contiguous())

    Az = prof(tB, 2)
    At = prof(tB, 1)
    ur = 1j * an * Az / rr - 1j * bl * At
    Ar = prof(tB, 0)
    ut = 1j * bl * Ar - prof(tdB, 2)
    uz = prof(tdB, 1) + At / rr - 1j * an * Ar / rr
    del Az, At, Ar
    tw = torch.from_numpy(w * r).to(dev)
    tcn = torch.from_numpy(cn).to(dev)
    ms = 0.0
    for f in (ur, ut, uz):
        ms += float(torch.einsum("j,jsn,n->", tw, f.abs() ** 2, tcn))
    scale = cfg["amp"] * abs(cfg["Re_i"]) / np.sqrt(ms / np.sum(w * r))
    u = torch.empty((3,) + tuple(ur.shape), dtype=torch.complex128, device=dev)
    u[0] = (ur + 1j * ut) * scale
    u[1] = (ur - 1j * ut) * scale
    u[2] = uz * scale
    del ur, ut, uz
    if with_couette:
        tU = torch.from_numpy(U).to(dev)
        u[0, :, 0, 0] += 1j * tU
        u[1, :, 0, 0] -= 1j * tU
    return u


def random_state(shape, seed, hermitian=True):
    """Unstructured complex test array (3 or more leading fields) with a
    real-field-consistent n = 0 plane and an empty Nyquist slot."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2.0)
    m_z = shape[-2]
    h = m_z // 2
    x[..., h, :] = 0.0
    if hermitian:
        x[..., 0, 0] = x[..., 0, 0].real
        x[..., m_z - np.arange(1, h), 0] = np.conj(x[..., np.arange(1, h), 0])
    return x


def random_field_torch(shape, seed, device):
    """Large unstructured complex128 test array drawn on ``device`` with a
    seeded torch generator (for sizes where NumPy generation is too slow);
    the empty axial slot (axis -2 midpoint) is zero."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    x = torch.randn(tuple(shape) + (2,), dtype=torch.float64, device=device, generator=g)
    x = torch.view_as_complex(x) / np.sqrt(2.0)
    x[..., shape[-2] // 2, :] = 0
    return x


def random_direction(r, cfg, seed):
    """Divergence-free unit-RMS perturbation direction (same recipe, no Couette part)."""
    c = Config(cfg)
    c["seed"] = seed
    c["amp"] = 1.0
    c["Re_i"] = 1.0
    return initial_state(r, c, with_couette=False)
