"""Pins of the oracle's banded Helmholtz/Poisson solves (Sec. 3.2, steps 2-4)."""
import numpy as np
import pytest

import oracle
from oracle.operators import KINDS


@pytest.fixture(scope="module")
def prob():
    return oracle.Problem(24, 5, 8, 0.6, 30.0, -10.0, 3e-3, k_theta=2.0, k_z=1.3, alpha=0.4)


def test_operators_structure(prob):
    A = prob.operator("Up", 2, 1)
    i, j = np.nonzero(A)
    assert np.max(np.abs(i - j)) <= 4
    np.testing.assert_array_equal(A[0], np.eye(prob.n_r)[0])
    P = prob.operator("P", 0, 0)
    np.testing.assert_array_equal(P[-1], np.eye(prob.n_r)[-1])
    np.testing.assert_array_equal(P[0], prob.D1[0])
    P = prob.operator("P", 1, 0)
    np.testing.assert_array_equal(P[-1], prob.D1[-1])
    # L+ - L- = -4a/r^2 on the diagonal (eq. modalNSdecoup)
    a = 2 * prob.k_theta
    d = np.diag(prob.operator("Up", 2, 1) - prob.operator("Um", 2, 1))[1:-1]
    scale = np.abs(np.diag(prob.operator("Up", 2, 1))).max()
    np.testing.assert_allclose(d, -4 * a / prob.r[1:-1] ** 2, rtol=0, atol=1e-13 * scale)


@pytest.mark.parametrize("kind", KINDS)
def test_banded_lu_matches_dense(prob, kind, rng):
    rhs = rng.standard_normal((prob.n_r, prob.m_z, prob.m_theta)) + 1j * rng.standard_normal((prob.n_r, prob.m_z, prob.m_theta))
    rhs[:, prob.nyq] = 0
    for trans in (0, 1):
        x = prob.solve(kind, rhs, trans=trans)
        for s in range(prob.m_z):
            if s == prob.nyq:
                assert np.all(x[:, s] == 0)
                continue
            for n in range(prob.m_theta):
                A = prob.operator(kind, n, abs(int(prob.l[s])))
                if trans:
                    A = A.T
                ref = np.linalg.solve(A, rhs[:, s, n])
                err = np.abs(x[:, s, n] - ref).max() / np.abs(ref).max()
                assert err < 1e-12, (kind, s, n, err)


def _manufactured(n_r, kind, n, labs):
    P = oracle.Problem(n_r, 4, 8, 0.5, 1.0, 0.0, 1e-2, k_theta=1.0, k_z=1.0)
    r, r_i = P.r, P.r_i
    a, b = n * P.k_theta, labs * P.k_z
    if kind == "P":
        k = 2 * np.pi
        u = np.cos(k * (r - r_i))
        du = -k * np.sin(k * (r - r_i))
        d2u = -k * k * np.cos(k * (r - r_i))
    else:
        s, c = np.sin(np.pi * (r - r_i)), np.cos(np.pi * (r - r_i))
        e = np.exp(r)
        u = s * e
        du = (np.pi * c + s) * e
        d2u = (-np.pi ** 2 * s + 2 * np.pi * c + s) * e
    lap = d2u + du / r - (a * a / r ** 2 + b * b) * u
    shift = {"P": 0.0, "Up": (1 + 2 * a) / r ** 2, "Um": (1 - 2 * a) / r ** 2, "Uz": 0.0}[kind]
    f = lap - shift * u - (0.0 if kind == "P" else 1.5 / P.dt) * u
    if kind == "P":
        f[0], f[-1] = du[0], du[-1]
    else:
        f[0], f[-1] = u[0], u[-1]
    x = P.solve_mode(kind, n, labs, f[:, None])[:, 0]
    return np.abs(x - u).max()


@pytest.mark.parametrize("kind,n,labs", [("Up", 2, 1), ("Um", 3, 0), ("Uz", 1, 2), ("P", 2, 1)])
def test_manufactured_order(kind, n, labs):
    sizes = np.array([24, 32, 48])
    errs = np.array([_manufactured(k, kind, n, labs) for k in sizes])
    order = -np.polyfit(np.log(sizes), np.log(errs), 1)[0]
    assert order >= 6.0, (order, errs)
    assert errs[-1] < 1e-7


def _lu_without_pivoting(A):
    A = A.copy()
    for k in range(len(A) - 1):
        A[k + 1:, k] /= A[k, k]
        A[k + 1:, k + 1:] -= np.outer(A[k + 1:, k], A[k, k + 1:])
    return A


def _lu_solve(LU, b):
    y = b.copy()
    for i in range(len(b)):
        y[i] -= LU[i, :i] @ y[:i]
    for i in range(len(b) - 1, -1, -1):
        y[i] = (y[i] - LU[i, i + 1:] @ y[i + 1:]) / LU[i, i]
    return y


@pytest.mark.parametrize("n_r,eta,Re,dt", [(64, 0.71, 1000.0, 5e-7), (512, 0.5, 1e4, 5e-5)])
def test_operators_need_no_pivoting(n_r, eta, Re, dt):
    # Sec. 4 factors with DGBTRF (partial pivoting).  Elimination without
    # pivoting, with P's Neumann rows scaled to the size of the Laplacian
    # rows, is backward stable for every operator of the workloads: its
    # componentwise backward error on A x = A x0 stays at a few units of
    # rounding (the GPU factorisation checks the same bound at set-up)
    P = oracle.Problem(n_r, 2, 4, eta, Re, 0.0, dt)
    x0 = 1.0 + 0.5 * np.sin(0.7 * np.arange(n_r))
    for kind in ("P", "Up", "Um", "Uz"):
        for n, labs in [(0, 0), (0, 1), (1, 0), (7, 3), (300, 200)]:
            A = P.operator(kind, n, labs)
            if kind == "P":
                scale = np.abs(A[1]).max()
                A[0] *= scale / np.abs(A[0]).max()
                if not (n == 0 and labs == 0):
                    A[-1] *= scale / np.abs(A[-1]).max()
            b = A @ x0
            x = _lu_solve(_lu_without_pivoting(A), b)
            berr = np.max(np.abs(A @ x - b) / (np.abs(A) @ np.abs(x) + np.abs(b)))
            assert berr < 1e-15, (kind, n, labs, berr)
