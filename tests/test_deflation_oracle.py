"""Pins of the setup-stage oracle (the k smallest eigenpairs by a dense
symmetric eigendecomposition) against closed forms: the 1D and 2D Dirichlet
Laplacians have the sine modes with eigenvalues 2 - 2 cos(j pi / (m + 1))
(sums of two such values in 2D)."""
import numpy as np
import scipy.sparse as sp

from oracle import eigen as E


def lap1d(m):
    return sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1]).tocsr()


def csr_parts(A):
    A = A.tocsr()
    A.sort_indices()
    return A.indptr, A.indices, A.data, A.shape[0]


def test_1d_laplacian_closed_form():
    m, k = 40, 6
    rp, ci, va, n = csr_parts(lap1d(m))
    w, V = E.lowest_eigenpairs(rp, ci, va, k)
    j = np.arange(1, k + 1)
    assert np.allclose(w, 2 - 2 * np.cos(j * np.pi / (m + 1)), rtol=0, atol=1e-13)
    # eigenvectors are the sine modes up to sign
    x = np.arange(1, m + 1)
    for c in range(k):
        s = np.sin((c + 1) * np.pi * x / (m + 1))
        s /= np.linalg.norm(s)
        assert abs(abs(s @ V[:, c]) - 1.0) <= 1e-12


def test_2d_laplacian_shifted_closed_form():
    m, k = 12, 7
    L1 = lap1d(m)
    A = (sp.kron(sp.identity(m), L1) + sp.kron(L1, sp.identity(m))).tocsr()
    f = 2 - 2 * np.cos(np.arange(1, m + 1) * np.pi / (m + 1))
    ev = np.sort(np.add.outer(f, f).ravel())
    sigma = 0.5 * (ev[k - 1] + ev[k])
    rp, ci, va, n = csr_parts(A - sigma * sp.identity(m * m))
    w, V = E.lowest_eigenpairs(rp, ci, va, k)
    assert np.allclose(w, ev[:k] - sigma, rtol=0, atol=1e-12)
    assert np.all(w < 0)
    Ad = E.dense_from_csr(rp, ci, va, n)
    assert np.linalg.norm(Ad @ V - V * w) <= 1e-12
    assert np.linalg.norm(V.T @ V - np.eye(k)) <= 1e-12


def test_rejects_nonsymmetric():
    A = sp.csr_matrix(np.array([[1.0, 2.0], [0.0, 1.0]]))
    rp, ci, va, n = csr_parts(A)
    try:
        E.lowest_eigenpairs(rp, ci, va, 1)
    except ValueError:
        return
    raise AssertionError("non-symmetric matrix accepted")
