"""Adjoint of the linear solve (oracle side, FP64).

For L(x) with A x = b: lambda = A^{-T} dL/dx, dL/db = lambda and
dL/dA_ij = -lambda_i x_j on the sparsity pattern of A.  The transposed
system is solved with the transposed multifrontal sweeps over the same
factors (refined with A^T).  This is the plain definition; parity unpinned
beyond the dense and finite-difference checks in the tests.
"""
import numpy as np

from . import krylov, mf


def solve_and_adjoint(A, fac, b, dLdx, tol=1e-12, max_it=100):
    """Returns (x, lambda, dL/dval) with dL/dval aligned to A's CSR entries."""
    S = A.to_scipy()
    x, _, _ = krylov.refine(lambda v: S @ v, lambda v: mf.apply_inverse(fac, v), b, tol, max_it)
    g = dLdx(x)
    St = S.T.tocsr()
    lam, _, _ = krylov.refine(lambda v: St @ v, lambda v: mf.apply_inverse(fac, v, trans=True), g, tol, max_it)
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    dval = -lam[rows] * x[A.colind]
    return x, lam, dval
