"""GPU setup stage (the k smallest eigenpairs, i.e. the deflation data) against
the oracle's dense eigendecomposition and the closed form of the 2D
Laplacian.  Bounds: every returned pair has ||A v - theta v|| <= tol g (g the
Gershgorin bound, checked here independently); then each Ritz value lies
within that residual of an eigenvalue, and within res^2 / gap of the wanted
one, and the sine of the angle between the computed and exact invariant
subspaces is at most res / gap (Davis-Kahan), gap = the distance from the
k-th to the (k+1)-th eigenvalue."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

from oracle import eigen as E
from paper_1805_12417_amd import solver as S
from paper_1805_12417_amd import workloads as W

pytestmark = pytest.mark.gpu


def dev_csr(A):
    A = A.tocsr()
    A.sort_indices()
    d = torch.device("cuda")
    return (torch.from_numpy(A.indptr.astype(np.int32)).to(d),
            torch.from_numpy(A.indices.astype(np.int32)).to(d),
            torch.from_numpy(A.data.astype(np.float64)).to(d))


def check_against_oracle(A, k, lam, V, st, tol):
    A = A.tocsr()
    A.sort_indices()
    Ad = A.toarray()
    g = np.abs(Ad).sum(axis=1).max()
    assert abs(st["bound"] - g) <= 1e-12 * g
    wo, Vo = E.lowest_eigenpairs(A.indptr, A.indices, A.data, k + 1)
    V = V.cpu().numpy()
    R = Ad @ V - V * lam
    res = np.linalg.norm(R, axis=0)
    assert st["converged"] == 1 and np.all(res <= tol * g * (1 + 1e-6)), res.max() / g
    assert np.linalg.norm(V.T @ V - np.eye(k)) <= 1e-10
    gap = wo[k] - wo[k - 1]
    assert np.all(np.abs(lam - wo[:k]) <= res + 1e-13 * g)
    assert np.all(np.abs(lam - wo[:k]) <= np.maximum(res ** 2 / gap, 1e-13 * g) * 1.01 + 1e-12 * g)
    # subspace angle: || (I - V V^T) Vo ||_2 <= ||R||_F / gap
    sin_t = np.linalg.norm(Vo[:, :k] - V @ (V.T @ Vo[:, :k]), 2)
    assert sin_t <= np.linalg.norm(R) / gap + 1e-10


@pytest.mark.parametrize("name,k", [("lap2d_64", 6), ("lap3d_small", 8), ("fe27_small", 10)])
def test_lowest_eigs_match_oracle(name, k):
    if name == "lap2d_64":
        w = W.shifted_laplace2d()
    elif name == "lap3d_small":
        w = W.shifted_laplace3d(dims=(12, 11, 10), k=k, seed=61)
    else:
        w = W.shifted_fe27(m=7, k=k, seed=62)
    A = sp.csr_matrix((w.val, w.col, w.row_ptr), shape=(w.n, w.n))
    lam, V, st = S.lowest_eigs(*dev_csr(A), k, tol=1e-11, seed=5)
    print(name, st)
    check_against_oracle(A, k, lam, V, st, 1e-11)
    assert st["negative"] == k and st["next_ritz"] > 0


def test_2d_laplacian_closed_form():
    """64 x 64 Dirichlet Laplacian shifted to 6 negative eigenvalues: the Ritz
    values equal the sine-mode eigenvalues f(i) + f(j) - sigma."""
    w = W.shifted_laplace2d()
    m = 64
    f = 2 - 2 * np.cos(np.arange(1, m + 1) * np.pi / (m + 1))
    ev = np.sort(np.add.outer(f, f).ravel()) - w.sigma
    A = sp.csr_matrix((w.val, w.col, w.row_ptr), shape=(w.n, w.n))
    lam, V, st = S.lowest_eigs(*dev_csr(A), 6, tol=1e-12, seed=9)
    assert np.all(np.abs(lam - ev[:6]) <= 1e-10), lam - ev[:6]
    assert abs(st["next_ritz"] - ev[6]) <= 1e-6


def test_gpu_deflation_drives_the_solver():
    """The solver created with the GPU-computed V-hat, Lambda-hat converges like
    with the workload's (setup-independent) ones."""
    w = W.shifted_laplace3d(dims=(23, 21, 19), k=20)
    A = sp.csr_matrix((w.val, w.col, w.row_ptr), shape=(w.n, w.n))
    rp, ci, va = dev_csr(A)
    lam, V, st = S.lowest_eigs(rp, ci, va, 20, tol=1e-10)
    assert st["converged"] == 1 and st["negative"] == 20
    b = torch.from_numpy(w.b).cuda()
    its = []
    for Vh, lh in ((V, torch.from_numpy(lam).cuda()),
                   (torch.from_numpy(np.ascontiguousarray(w.Vhat)).cuda(), torch.from_numpy(w.lam).cuda())):
        s = S.MinresCG(rp, ci, va, Vh, lh, precision=S.PREC_MIXED)
        x, sts = s.solve(b, s.preconditioner("jacobi"), rtol_out=1e-8, rtol_in=1e-4)
        r = np.linalg.norm(w.b - A @ x.cpu().numpy()) / np.linalg.norm(w.b)
        assert sts.status == 0 and r <= 1e-8
        its.append(sts.inner_its_total)
        s.close()
    assert abs(its[0] - its[1]) <= 0.05 * its[1] + 5, its


def test_block_sizes_and_invalid_arguments():
    w = W.shifted_laplace3d(dims=(12, 11, 10), k=4, seed=63)
    A = sp.csr_matrix((w.val, w.col, w.row_ptr), shape=(w.n, w.n))
    rp, ci, va = dev_csr(A)
    for block in (16, 32, 48, 64):
        lam, V, st = S.lowest_eigs(rp, ci, va, 4, block=block, tol=1e-10)
        check_against_oracle(A, 4, lam, V, st, 1e-10)
    with pytest.raises(S.MCGError):
        S.lowest_eigs(rp, ci, va, 0)
    with pytest.raises(S.MCGError):          # block above 64
        S.lowest_eigs(rp, ci, va, 4, block=80)
    with pytest.raises(S.MCGError):          # k above the block
        S.lowest_eigs(rp, ci, va, 20, block=16)
    tiny = sp.diags([1.0, -2.0, 3.0]).tocsr()
    with pytest.raises(S.MCGError):          # block larger than n
        S.lowest_eigs(*dev_csr(tiny), 1)
