"""FP64 CPU oracle for parareal matrix-function flows.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library (no kernels, headers, helpers, tables or pre/post-processing); the two
meet only through seeded inputs produced elsewhere.

The oracle is a plain, slow, obviously correct FP64 implementation of what the
GPU path computes, written from the paper (Chehab & Petcu, "Parallel Matrix
Function Evaluation via Initial value ODE modelling"):

* ``flows``      right-hand sides of the matrix ODEs (Sec. 1 and Sec. 2,
                 Example 1; steady-state modelling of Sec. 1 / Sec. 4)
* ``integrators`` classical RK4 fine propagator and forward-Euler coarse
                 propagator (Sec. 1 names explicit Euler and Runge-Kutta as the
                 time marching schemes)
* ``parareal``   the classical parareal algorithm (Sec. 2, Alg. 1)
* ``exact``      the targets f(A): LU inverse, eigen square root, and the
                 closed-form solutions of the three flows used as pins
* ``refine``     FP64 Newton-Schulz and full-Newton square-root refinement
* ``learned``    the learned coarse step family and its least-squares fit
* ``mlp``        the small MLP (forward, backward, Adam) in FP64

Every function works on either dense FP64 matrices (``MatrixAlgebra``) or on
the eigenvalues of a symmetric problem started from X0 = I
(``SpectralAlgebra``): with A = Q diag(lam) Q^T every iterate of every step
above is Q diag(x) Q^T where x runs the *same* discrete algorithm on lam.

Parity status per function is recorded in each module header.
"""

from .core import MatrixAlgebra, SpectralAlgebra, HOMOTOPY, STEADY_INV, SQRT, EXP, INV_LINEAR  # noqa: F401
from .core import KINDS, LINEAR_KINDS, INVERSE_KINDS  # noqa: F401
from . import flows, integrators, parareal, exact, refine, learned, mlp  # noqa: F401
