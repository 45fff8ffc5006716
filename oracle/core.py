"""Algebra back-ends for the oracle (test infrastructure only).

``MatrixAlgebra``: dense n x n FP64 matrices, products by numpy matmul.

``SpectralAlgebra``: a symmetric A = Q diag(lam) Q^T and an initial value that
is a function of A (here always X0 = I).  Every quantity the method forms from
such inputs (flow right-hand sides, RK4 stages, Euler steps, the parareal
correction, the learned polynomial step, Newton-Schulz and Newton refinement)
is a polynomial or rational function of A, so it equals Q diag(x) Q^T with x the
same expression evaluated on the eigenvalues.  The spectral algebra stores only
x (a length-n vector), multiplies elementwise, and its Frobenius norm is the
2-norm of x because Q is orthogonal.  ``to_matrix`` rebuilds the dense matrix.
"""

import numpy as np

# Flow kinds.  Numbering follows the C interface of the library under test so
# that test code can pass one value to both sides.
HOMOTOPY = 1    # dX/dt = X (I - A) X, X(0) = I, X(1) = A^{-1} (Sec. 2, Example 1)
STEADY_INV = 2  # dX/dt = X - X A X, stable steady state A^{-1}
SQRT = 3        # dX/dt = A - X^2, stable steady state A^{1/2} (A SPD)
EXP = 4         # dQ/dt = A Q, Q(0) = I, Q(1) = exp(A) (Sec. 2, Example 2)
INV_LINEAR = 5  # dX/dt = I - A X, stable steady state A^{-1} (Sec. 4, Example 5)
KINDS = (HOMOTOPY, STEADY_INV, SQRT, EXP, INV_LINEAR)
LINEAR_KINDS = (EXP, INV_LINEAR)
INVERSE_KINDS = (HOMOTOPY, STEADY_INV, INV_LINEAR)


class MatrixAlgebra:
    """Dense FP64 n x n matrices."""

    spectral = False

    def __init__(self, n):
        self.n = int(n)

    def eye(self):
        return np.eye(self.n)

    def mul(self, X, Y):
        return X @ Y

    def fro(self, X):
        return float(np.sqrt(np.sum(X * X)))

    def inner(self, X, Y):
        """Frobenius inner product <X, Y>_F = tr(Y^T X) (Sec. 3)."""
        return float(np.sum(X * Y))

    def solve(self, M, B):
        """M^{-1} B by LU with partial pivoting (LAPACK gesv)."""
        return np.linalg.solve(M, B)

    def trace(self, X):
        return float(np.trace(X))

    def to_matrix(self, X):
        return X


class SpectralAlgebra:
    """Functions of a symmetric A held as their eigenvalues in A's eigenbasis."""

    spectral = True

    def __init__(self, Q, lam):
        self.Q = np.asarray(Q, dtype=np.float64)
        self.lam = np.asarray(lam, dtype=np.float64)
        self.n = self.lam.shape[0]

    def eye(self):
        return np.ones(self.n)

    def mul(self, X, Y):
        return X * Y

    def fro(self, X):
        return float(np.sqrt(np.sum(X * X)))

    def inner(self, X, Y):
        return float(np.sum(X * Y))

    def solve(self, M, B):
        return B / M

    def trace(self, X):
        return float(np.sum(X))

    def to_matrix(self, x):
        return (self.Q * x) @ self.Q.T

    def entries(self, x, rows, cols):
        """Selected entries of Q diag(x) Q^T without forming the matrix."""
        rows = np.asarray(rows)
        cols = np.asarray(cols)
        return np.einsum("ij,j,ij->i", self.Q[rows], x, self.Q[cols])
