"""Pins of the FP64 reference of the learned preconditioner (CPU)."""
import numpy as np
import pytest
import torch

from oracle import learned as LR
from paper_1805_12417_amd import workloads as W


def tiny(m=3, k=2, seed=3):
    w = W.shifted_fe27(m=m, k=k, seed=seed)
    return w, LR.Graph(w.row_ptr, w.col, w.val, 3)


def test_graph_counts_match_the_27_point_structure():
    w, g = tiny(4)
    assert g.N == 64 and g.E == (3 * 4 - 2) ** 3 - 64
    assert np.all(np.diff(g.src) >= 0)
    # both directions, features transposed
    ek = {(int(a), int(b)): i for i, (a, b) in enumerate(zip(g.src, g.dst))}
    for (a, b), i in list(ek.items())[:50]:
        j = ek[(b, a)]
        assert np.allclose(g.fe[i].reshape(3, 3), g.fe[j].reshape(3, 3).T)


def test_C_is_lower_triangular_with_positive_diagonal_and_CCt_spd():
    w, g = tiny()
    theta = torch.from_numpy(LR.init_params(3, 0).astype(np.float64))
    rng = np.random.default_rng(1)
    theta = theta + 0.05 * torch.from_numpy(rng.standard_normal(theta.numel()))
    C = LR.assemble_C(theta, g).detach().numpy()
    # lower triangular with a positive diagonal: C is the Cholesky factor of
    # C C^T, which is therefore SPD
    assert np.allclose(C, np.tril(C))
    assert np.all(np.diag(C) > 0)
    sign, logdet = np.linalg.slogdet(C)
    assert sign > 0 and np.isfinite(logdet)
    x = rng.standard_normal((C.shape[0], 5))
    assert np.all(np.einsum("ij,ij->j", x, C @ (C.T @ x)) > 0)


def test_initial_network_is_close_to_jacobi():
    w, g = tiny()
    theta = torch.from_numpy(LR.init_params(3, 0).astype(np.float64))
    C = LR.assemble_C(theta, g).detach().numpy()
    S_inv = np.diag(1.0 / g.s)
    assert np.allclose(np.diag(C), np.diag(S_inv), rtol=0.2)
    off = C - np.diag(np.diag(C))
    assert np.abs(off).max() < 0.1 * np.abs(np.diag(C)).max()


def test_csr_values_match_dense_assembly():
    w, g = tiny()
    theta = torch.from_numpy(LR.init_params(3, 1).astype(np.float64))
    lp, lc, lv = LR.csr_C(theta, g, w.row_ptr, w.col)
    import scipy.sparse as sp
    Cs = sp.csr_matrix((lv, lc, lp), shape=(w.n, w.n)).toarray()
    C = LR.assemble_C(theta, g).detach().numpy()
    assert np.allclose(Cs, C, atol=1e-14)


def test_loss_gradient_matches_directional_finite_differences():
    """Autograd gradient of the loss against central differences along random
    directions (the loss is piecewise smooth: ReLU kinks are met with
    probability ~0 at this step size)."""
    w, g = tiny(m=3, k=2)
    rng = np.random.default_rng(2)
    theta = torch.from_numpy(LR.init_params(3, 2).astype(np.float64)
                             + 0.05 * rng.standard_normal(LR.n_params(3))).requires_grad_(True)
    Y = rng.standard_normal((w.n, 2)); Z = rng.standard_normal((w.n, 2))
    L = LR.loss(theta, g, Y, Z)
    L.backward()
    grad = theta.grad.detach()
    eps = 1e-6
    for _ in range(4):
        d = torch.from_numpy(rng.standard_normal(theta.numel()))
        with torch.no_grad():
            fd = (LR.loss(theta + eps * d, g, Y, Z) - LR.loss(theta - eps * d, g, Y, Z)) / (2 * eps)
        assert abs(float(fd) - float(grad @ d)) <= 2e-5 * abs(float(fd)) + 1e-8


def test_loss_is_zero_for_the_exact_pairs():
    """Loss vanishes when z = C C^T y for the network's own C."""
    w, g = tiny(m=3, k=2)
    theta = torch.from_numpy(LR.init_params(3, 4).astype(np.float64))
    C = LR.assemble_C(theta, g).detach().numpy()
    Y = np.random.default_rng(5).standard_normal((w.n, 3))
    Z = C @ (C.T @ Y)
    assert float(LR.loss(theta, g, Y, Z)) < 1e-28
