"""FP64 CPU oracle for the Gauss-Newton-Krylov registration hot path.

TEST INFRASTRUCTURE ONLY. This package is the plain, slow reference that the
GPU library is checked against. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the library never does, and the
two share no code (they share only the seeded input generators in ``synth``).

It follows Mang & Biros, "An inexact Newton-Krylov algorithm for constrained
diffeomorphic image registration" (arXiv 1408.6299), in the paper's order and
notation:

* ``spectral``  -- Fourier pseudospectral derivatives and the spectral
  operators A (first variation of the regulariser), K (elimination of the
  pressure, i.e. the Leray projection) and the preconditioner (beta A)^-1
  (Sections "Numerical Discretization", "Inversion: Regularization Operators",
  "Elimination of p and p~"; equations e:first-variation-H1/H2,
  e:eliminated-control).
* ``timebasis`` -- the Chebyshev expansion of v in time (e:expansion).
* ``transport`` -- RK2 (Heun) solves of the state equation, the adjoint
  equation and the incremental (Gauss-Newton) equations
  (e:first-order-forward, e:first-order-adjoint, e:gauss-newton).
* ``reduced``   -- objective, reduced gradient and GN Hessian matvec
  (e:first-order-control, e:eliminated-icontrol, Algorithm a:hessian-matvec).
* ``krylov``    -- PCG with the forcing sequence (e:termination-criterion-ksm),
  Armijo line search, the outer iteration (Algorithm a:outer-iteration),
  stopping rules (e:stopping-criteria) and beta continuation.
* ``defgrad``   -- the deformation gradient F and det F_1 (e:def-grad).

All floating point is FP64. Readings of passages where the paper is silent or
ambiguous are stated in each function's docstring.

Parity status: every function here is pinned by a test in
``tests/test_oracle_*.py`` against closed forms, brute force, invariants or
values printed in the paper. None is "parity unpinned".
"""
from . import spectral, timebasis, transport, reduced, krylov, defgrad  # noqa: F401
from .reduced import Problem  # noqa: F401
