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


def test_brake_inner_level_inertia_and_pencil():
    """The stand-in for K_E - |gamma|^2 M (Section 3.1, eq. inner_level): M is
    SPD with ||M||_F << ||K_E||_F, exactly k eigenvalues of A are negative
    and, by Sylvester's law, exactly k generalized eigenvalues of the pencil
    (K_E, M) lie below |gamma|^2 (checked by a dense generalized
    eigensolver, independent of the generator's scaled problem); V_hat,
    lam_hat are A's negative eigenpairs."""
    import scipy.linalg as sla
    w = W.brake_inner_level(m=6, k=5)
    A = w.scipy().toarray()
    M = np.diag(w.meta["mass"])
    K = A + w.meta["gamma_abs2"] * M
    assert np.all(w.meta["mass"] > 0)
    assert np.linalg.norm(M) < 1e-2 * np.linalg.norm(K)
    assert np.linalg.eigvalsh(K).min() > 0
    ev = np.linalg.eigvalsh(A)
    assert int((ev < 0).sum()) == 5
    mu = sla.eigh(K, M, eigvals_only=True)
    assert int((mu < w.meta["gamma_abs2"]).sum()) == 5
    assert np.allclose(w.lam, ev[:5], rtol=1e-10)
    R = A @ w.Vhat - w.Vhat * w.lam
    assert np.linalg.norm(R) <= 1e-8 * np.abs(ev).max()


def test_brake_sweep_rhs_share_modulus():
    w = W.brake_inner_level(m=5, k=3)
    sw = W.brake_sweep_rhs(w, 4, 3)
    g = np.sqrt(w.meta["gamma_abs2"])
    assert len(sw) == 4
    for gamma, b in sw:
        assert abs(abs(gamma) - g) <= 1e-12 * g and gamma.real > 0 and gamma.imag > 0
        assert b.shape == (w.n,)
    assert len({round(gm.imag, 6) for gm, _ in sw}) == 4


def test_kkt_saddle_inertia_pattern_and_order():
    """[[K, B^T], [B, 0]] with K = the SPD 2D Laplacian and B of full row
    rank has exactly n_con negative eigenvalues (Sylvester's law on the
    block LDL^T); the zero block has no stored entries; with interleaving
    every constraint row sits just before the first unknown it couples
    (after any other constraint that couples it first)."""
    w = W.kkt_saddle(m=10, n_con=8, seed=3, coupling=10.0)
    A = w.scipy().toarray()
    assert np.array_equal(A, A.T)
    ev = np.linalg.eigvalsh(A)
    assert int((ev < 0).sum()) == 8 and w.k == 8
    assert np.allclose(w.lam, ev[:8], rtol=1e-10)
    assert np.linalg.norm(A @ w.Vhat - w.Vhat * w.lam) <= 1e-8 * np.abs(ev).max()
    S = w.scipy()
    diag_stored = np.zeros(w.n, bool)
    for i in range(w.n):
        diag_stored[i] = i in S.indices[S.indptr[i]:S.indptr[i + 1]]
    con = np.nonzero(~diag_stored)[0]               # the constraint rows
    assert con.size == 8
    for r in con:
        cols = S.indices[S.indptr[r]:S.indptr[r + 1]]
        nxt = r + 1
        while nxt in con:                           # constraints sharing that unknown
            nxt += 1
        assert cols.min() == nxt and np.all(np.isin(cols, con, invert=True))
    w2 = W.kkt_saddle(m=10, n_con=8, seed=3, coupling=10.0, interleave=False)
    assert np.allclose(np.sort(np.linalg.eigvalsh(w2.scipy().toarray())), ev, atol=1e-10)
