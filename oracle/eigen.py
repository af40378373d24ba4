"""Oracle for the setup stage of MINRES-CG (TEST INFRASTRUCTURE ONLY: used by
tests, never by the product package): the k algebraically smallest
eigenpairs of a symmetric sparse matrix, i.e. the deflation data V-hat,
Lambda-hat of Section 2 (the paper obtains them with a sparse eigensolver,
Section 4).  This is their plain definition: assemble the dense matrix and
take a full symmetric eigendecomposition (a library routine as the one
step), in FP64.  For small matrices only."""
from __future__ import annotations

import numpy as np


def dense_from_csr(row_ptr, col, val, n):
    A = np.zeros((n, n))
    for i in range(n):
        for p in range(int(row_ptr[i]), int(row_ptr[i + 1])):
            A[i, int(col[p])] += float(val[p])
    return A


def lowest_eigenpairs(row_ptr, col, val, k):
    """(w, V): the k smallest eigenvalues, ascending, and orthonormal
    eigenvectors (n x k) of the symmetric matrix in CSR form."""
    n = len(row_ptr) - 1
    A = dense_from_csr(row_ptr, col, val, n)
    if not np.allclose(A, A.T, rtol=0, atol=1e-14 * max(1.0, np.abs(A).max())):
        raise ValueError("matrix is not symmetric")
    w, V = np.linalg.eigh(A)
    return w[:k], V[:, :k]
