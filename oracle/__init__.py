"""FP64 CPU oracle for the Taylor-Couette projection step (test infrastructure).

This package is the plain, slow reference that the HIP path is checked
against.  It is test infrastructure only: the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the product path
(the C-ABI library and its Python binding) never does, and shares no code
with it.

Everything here is double precision and follows the paper (Shi, Rampp, Hof,
Avila, "A hybrid MPI-OpenMP parallel implementation for pseudospectral
simulations with application to Taylor-Couette flow") section by section:

* ``radial``     Sec. 3.1: node map (eq. nodeDist), Fornberg FD weights with
                 stencils shortened towards the walls.
* ``operators``  Sec. 3.1-3.2: mode-decoupled Helmholtz/Poisson operators
                 (eq. modalNSdecoup), their boundary rows, LAPACK banded LU
                 (DGBTRF/DGBTRS, the routines Sec. 4 names).
* ``nonlinear``  Sec. 3.2 step 1: pseudospectral nonlinear term with 3/2
                 dealiasing, rotational form omega x u and the paper's
                 convective form u.grad u.
* ``scheme``     Sec. 3.2 steps 1-6: AB2BD2 projection step (eqs. timeScheme,
                 pressure, vel, correction, update).
* ``diagnostics`` energies, divergence, wall slip (Sec. 5.3).
* ``adjoint``    tangent-linear and adjoint of one step (not in the paper).
"""
from .radial import radii, nodes, fornberg_weights, fd_matrices, couette_profile
from .operators import Problem
from .nonlinear import nonlinear_term, nonlinear_rot, nonlinear_conv
from . import scheme, diagnostics

__all__ = ["radii", "nodes", "fornberg_weights", "fd_matrices", "couette_profile",
           "Problem", "nonlinear_term", "nonlinear_rot", "nonlinear_conv", "scheme", "diagnostics"]
