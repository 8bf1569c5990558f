"""Radial discretisation (Sec. 3.1 of the paper).

* Lengths are in units of the gap d = r_o - r_i, so r_i = eta/(1-eta) and
  r_o = 1/(1-eta) (Sec. 2, non-dimensionalisation).
* Nodes follow eq. nodeDist (Kosloff-Tal-Ezer map); alpha = 0 is taken as
  the Chebyshev limit alpha -> 0.  ``n_r`` counts all nodes j = 0..M
  including both walls, so M = n_r - 1.
* Radial derivatives are central finite differences with Fornberg weights
  computed on the actual (non-uniform) nodes.  Row i uses the nodes
  max(0, i-4) .. min(M, i+4): 9 points inside, shortened to 5 points at
  the walls so that the matrices stay banded with kl = ku = 4 (Sec. 3.1).
"""
import numpy as np

HALF = 4  # half-width of the 9-point stencil (n_s = 9)


def radii(eta):
    """Inner and outer radius in gap units."""
    return eta / (1.0 - eta), 1.0 / (1.0 - eta)


def nodes(n_r, eta, alpha):
    """Radial nodes r_j, j = 0..M (eq. nodeDist).

    -cos(pi j/M) is written as sin(pi (2j-M)/(2M)) so that the end points
    are exactly -1 and +1 and the map is odd about mid-gap.
    """
    M = n_r - 1
    j = np.arange(n_r, dtype=np.float64)
    x = np.sin(np.pi * (2.0 * j - M) / (2.0 * M))
    centre = (1.0 + eta) / (2.0 * (1.0 - eta))
    if alpha == 0.0:
        return centre + 0.5 * x
    return centre + np.arcsin(alpha * x) / (2.0 * np.arcsin(alpha))


def fornberg_weights(z, x, m):
    """Weights c[k, j] such that f^(k)(z) ~ sum_j c[k, j] f(x[j]), k = 0..m.

    Fornberg's recursive algorithm (B. Fornberg, Math. Comp. 51 (1988)),
    the reference the paper gives for its FD weights.  Exact for
    polynomials of degree < len(x).
    """
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    c = np.zeros((m + 1, n))
    c[0, 0] = 1.0
    prod_prev = 1.0
    dz_prev = x[0] - z
    for i in range(1, n):
        kmax = min(i, m)
        prod = 1.0
        dz_im1 = dz_prev
        dz_prev = x[i] - z
        for j in range(i):
            dx = x[i] - x[j]
            prod *= dx
            if j == i - 1:
                for k in range(kmax, 0, -1):
                    c[k, i] = prod_prev * (k * c[k - 1, i - 1] - dz_im1 * c[k, i - 1]) / prod
                c[0, i] = -prod_prev * dz_im1 * c[0, i - 1] / prod
            for k in range(kmax, 0, -1):
                c[k, j] = (dz_prev * c[k, j] - k * c[k - 1, j]) / dx
            c[0, j] = dz_prev * c[0, j] / dx
        prod_prev = prod
    return c


def stencil_range(i, n_r):
    """First and last node used by FD row i (stencils shortened at the walls)."""
    return max(0, i - HALF), min(n_r - 1, i + HALF)


def fd_matrices(r):
    """Dense first- and second-derivative matrices D1, D2 (banded, kl=ku=4)."""
    n_r = len(r)
    D1 = np.zeros((n_r, n_r))
    D2 = np.zeros((n_r, n_r))
    for i in range(n_r):
        lo, hi = stencil_range(i, n_r)
        w = fornberg_weights(r[i], r[lo:hi + 1], 2)
        D1[i, lo:hi + 1] = w[1]
        D2[i, lo:hi + 1] = w[2]
    return D1, D2


def couette_profile(r, eta, Re_i, Re_o):
    """Circular Couette flow U_theta = C1 r + C2 / r (Sec. 5.1)."""
    C1 = (Re_o - eta * Re_i) / (1.0 + eta)
    C2 = eta * (Re_i - eta * Re_o) / ((1.0 - eta) * (1.0 - eta ** 2))
    return C1 * r + C2 / r
