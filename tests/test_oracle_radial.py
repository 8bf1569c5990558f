"""Pins of the oracle's radial discretisation (nodes, FD weights, operators)."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle.radial import fornberg_weights, fd_matrices, nodes, radii
from conftest import read_golden, paper_value


def test_nodes_walls_and_limits():
    # eq. nodeDist: j = 0 and j = M land on the walls; alpha = 1 is uniform,
    # alpha -> 0 gives the Chebyshev points.
    for eta in (0.5, 0.71, 0.993):
        r_i, r_o = radii(eta)
        for alpha in (0.0, 0.3, 0.5, 1.0):
            r = nodes(33, eta, alpha)
            assert abs(r[0] - r_i) <= 4e-15 * r_o and abs(r[-1] - r_o) <= 4e-15 * r_o
            assert np.all(np.diff(r) > 0)
        u = nodes(33, eta, 1.0)
        np.testing.assert_allclose(np.diff(u), (r_o - r_i) / 32, rtol=1e-12)
        M = 32
        cheb = (1 + eta) / (2 * (1 - eta)) - np.cos(np.pi * np.arange(33) / M) / 2
        np.testing.assert_allclose(nodes(33, eta, 0.0), cheb, rtol=0, atol=1e-14 * r_o)
        np.testing.assert_allclose(nodes(33, eta, 1e-7), cheb, rtol=0, atol=1e-12 * r_o)


def test_fornberg_textbook_weights():
    rows = read_golden("fd_weights_uniform9.txt")
    x = np.arange(-4.0, 5.0)
    w = fornberg_weights(0.0, x, 2)
    for row in rows:
        parts = row.split()
        k = int(parts[0])
        exact = np.array([float(Fraction(p)) for p in parts[1:]])
        np.testing.assert_allclose(w[k], exact, rtol=0, atol=1e-14)


def test_fornberg_polynomial_exactness(rng):
    # weights from n nodes differentiate every polynomial of degree < n exactly
    for n in range(5, 10):
        x = np.sort(rng.uniform(-1, 1, n))
        z = rng.uniform(-0.5, 0.5)
        w = fornberg_weights(z, x, 2)
        for deg in range(n):
            f = x ** deg
            d1 = deg * z ** (deg - 1) if deg >= 1 else 0.0
            d2 = deg * (deg - 1) * z ** (deg - 2) if deg >= 2 else 0.0
            scale = np.max(np.abs(w)) * 1.0
            assert abs(w[0] @ f - z ** deg) <= 1e-10 * scale
            assert abs(w[1] @ f - d1) <= 1e-10 * scale
            assert abs(w[2] @ f - d2) <= 1e-9 * scale


def test_fd_matrices_banded_and_exact():
    r = nodes(40, 0.5, 0.0)
    D1, D2 = fd_matrices(r)
    i, j = np.nonzero(D1)
    assert np.max(np.abs(i - j)) == 4
    i, j = np.nonzero(D2)
    assert np.max(np.abs(i - j)) == 4
    # shortest stencil (5 points at the walls) is exact up to degree 4
    for deg in range(5):
        f = r ** deg
        d1 = deg * r ** (deg - 1) if deg else 0 * r
        d2 = deg * (deg - 1) * r ** (deg - 2) if deg > 1 else 0 * r
        np.testing.assert_allclose(D1 @ f, d1, rtol=0, atol=1e-9 * max(1, np.abs(d1).max()))
        np.testing.assert_allclose(D2 @ f, d2, rtol=0, atol=1e-7 * max(1, np.abs(d2).max()))
    # row lengths 5,6,7,8,9,...,9,8,7,6,5 (stencils shortened towards the walls)
    lengths = np.count_nonzero(D1 != 0, axis=1) + (np.diag(D1) == 0)
    assert list(lengths[:5]) == [5, 6, 7, 8, 9] and list(lengths[-5:]) == [9, 8, 7, 6, 5]


def _laminar_error(n_r, alpha):
    eta = paper_value("laminar_eta")
    Re_i, Re_o = paper_value("laminar_Re_i"), paper_value("laminar_Re_o")
    P = oracle.Problem(n_r, 2, 4, eta, Re_i, Re_o, 1.0, alpha=alpha)
    # steady azimuthal momentum of mode (0,0): D2 + D1/r - 1/r^2 acting on
    # u_theta (eq. NS_cyl), with the wall values Re_i, Re_o
    A = P.D2 + P.D1 / P.r[:, None] - np.diag(1.0 / P.r ** 2)
    A[0] = 0.0
    A[0, 0] = 1.0
    A[-1] = 0.0
    A[-1, -1] = 1.0
    b = np.zeros(n_r)
    b[0], b[-1] = Re_i, Re_o
    ut = np.linalg.solve(A, b)
    U = oracle.couette_profile(P.r, eta, Re_i, Re_o)
    w = oracle.diagnostics.trapezoid_weights(P.r)
    return np.sum(w * np.abs((ut - U) / U) * P.r)


@pytest.mark.parametrize("alpha", [0.0, 0.5])
def test_laminar_couette_error_order(alpha):
    # Sec. 5.1: global error E_u of the laminar profile falls as a power of n_r.
    # The paper's fit gives about -11; the stencils read here (shortened
    # symmetrically to 5 points at the walls) give the formal order 8.
    n = np.array([24, 32, 40])
    E = np.array([_laminar_error(k, alpha) for k in n])
    slope = np.polyfit(np.log(n), np.log(E), 1)[0]
    assert -9.0 < slope < -7.0, slope
    assert slope > paper_value("laminar_error_exponent")
    assert E[-1] < 1e-10


def test_couette_closed_form():
    # U = C1 r + C2/r satisfies the wall conditions of eq. nsBC
    eta, Re_i, Re_o = 0.5, 50.0, 200.0
    r_i, r_o = radii(eta)
    U = oracle.couette_profile(np.array([r_i, r_o]), eta, Re_i, Re_o)
    np.testing.assert_allclose(U, [Re_i, Re_o], rtol=1e-14)
