"""Oracle for the block-structured multigrid Poisson path: TEST INFRASTRUCTURE.

A plain, slow, single-threaded CPU implementation (C++17, FP64, no FMA
contraction) that shares no code with the HIP library.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import, call, link or execute anything in this package.

Parity status per function (what pins it, see tests/test_oracle_*.py):
  chop / hierarchy       : worked chopping examples, coarsening invariants
  fill_boundary / bc     : numpy.pad (wrap / symmetric) on the global array
  gs                     : GS zeroes the residual of the updated colour
  residual / apply_op    : discrete sine eigenvectors (closed form), symmetry,
                           telescoping flux sum, beta==1 special case
  restrict / prolong     : reshape-mean, separable 1D interpolation, linear
                           reproduction, R(P(c)) identities on dyadic codes
  bottom                 : numpy.linalg.solve / lstsq on the assembled matrix
  solve (FP64 and mixed) : closed-form discrete solution, second-order error
                           convergence, dense 8^3 direct solve, contraction
"""
from . import pyoracle  # noqa: F401
