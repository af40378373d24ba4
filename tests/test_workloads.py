"""Seeded input generators: structure and spectral placement of the shift."""
import numpy as np
import scipy.sparse as sp

from paper_1805_12417_amd import workloads as W


def test_laplace2d_closed_form_matches_dense_spectrum():
    w = W.shifted_laplace2d()
    assert (w.n, w.nnz, w.k) == (4096, 20224, 6)
    ev = np.linalg.eigvalsh(w.scipy().toarray())
    assert int((ev < 0).sum()) == 6
    assert np.allclose(np.sort(ev)[:6], np.sort(w.lam), atol=1e-12)
    assert abs(np.abs(ev).min() - w.meta["min_abs_eig"]) < 1e-12
    A = w.scipy()
    assert np.linalg.norm(A @ w.Vhat - w.Vhat * w.lam) < 1e-12
    assert np.linalg.norm(w.Vhat.T @ w.Vhat - np.eye(6)) < 1e-12


def test_laplace2d_literal_five_negatives_is_singular():
    """The 5th and 6th eigenvalues of the 64x64 Laplacian coincide."""
    w, _ = W.laplace2d_modes(64, 7)
    assert abs(w[4] - w[5]) < 1e-14 and w[5] < w[6]


def test_laplace3d_random_structure():
    rng = np.random.default_rng(0)
    A = W.laplace3d_random(5, 4, 3, rng)
    n = 60
    assert A.shape == (n, n) and abs(A - A.T).max() == 0
    # 7-point: nnz = n + 2 * (#interior edges)
    edges = 4 * 4 * 3 + 5 * 3 * 3 + 5 * 4 * 2
    assert A.nnz == n + 2 * edges
    # SPD and diagonally dominant (boundary edges add to the diagonal)
    assert np.linalg.eigvalsh(A.toarray()).min() > 0


def test_laplace3d_small_shift_places_exactly_k_negatives():
    w = W.shifted_laplace3d(m=12, k=7)
    ev = np.linalg.eigvalsh(w.scipy().toarray())
    assert int((ev < 0).sum()) == 7
    assert np.allclose(np.sort(ev)[:7], w.lam, atol=1e-9)
    assert np.linalg.norm(w.Vhat.T @ w.Vhat - np.eye(7)) < 1e-12


def test_fe27_structure_and_colouring():
    m = 5
    rp, ci, va, cptr = W.fe27_colored(m, np.random.default_rng(1))
    n = 3 * m ** 3
    A = sp.csr_matrix((va, ci, rp), shape=(n, n))
    assert A.nnz == 9 * (3 * m - 2) ** 3
    assert abs(A - A.T).max() < 1e-14
    assert np.linalg.eigvalsh(A.toarray()).min() > 0
    for i in range(n):
        assert np.all(np.diff(ci[rp[i]:rp[i + 1]]) > 0)
    # nodes of one colour are not coupled to other nodes of that colour
    node_colour = np.repeat(np.arange(8), np.diff(cptr))
    C = A.tocoo()
    same = node_colour[C.row // 3] == node_colour[C.col // 3]
    assert np.all((C.row // 3)[same] == (C.col // 3)[same])


def test_batch_sizes_log_uniform_range():
    sizes = W.batch_sizes()
    assert len(sizes) == 48
    ns = [a * b * c for (a, b, c), _ in sizes]
    assert min(ns) >= 1.5e4 and max(ns) <= 6e5
    assert all(2 <= k <= 40 for _, k in sizes)
