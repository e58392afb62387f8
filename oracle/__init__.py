"""CPU oracle for the B-spline (IgA) Helmholtz solver: TEST INFRASTRUCTURE ONLY.

A plain, slow, float64/complex128 reimplementation, written from the paper
(Dwarka, Tielen, Moeller, Vuik: deflation + multigrid-approximated CSLP with
GMRES for isogeometric Helmholtz discretisations), of everything the GPU
library computes.  Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import it.  It shares no code with the HIP
library and imports nothing from it.

Modules
  bspline    knot vectors, Cox-de Boor basis, Gauss-Legendre element matrices,
             knot-insertion prolongation (section 2.3.1)
  helmholtz  stiffness / k^2-weighted mass, Dirichlet elimination, point
             source load (sections 2.1-2.3)
  solver     CSLP, multigrid V-cycle, (multilevel) deflation, FGMRES (section 3)
  cnn        the learned-smoother network in float64 (not from the paper:
             parity unpinned except by gradient checks and zero-weight cases)
"""
from . import bspline, helmholtz, solver  # noqa: F401
from .helmholtz import Problem  # noqa: F401
from .solver import Options, Solver  # noqa: F401
