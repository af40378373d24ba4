"""Tiny dense constructions from Sections 1 and 2.1, in numpy (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).  These are used as
pins for the C oracle: they build the exact preconditioners for which the
paper states finite-termination results.

  * bunch_parlett(A): P A P^T = L D L^T with 1x1 / 2x2 pivots chosen by
    complete pivoting (Bunch & Parlett 1971, alpha = (1 + sqrt 17)/8), the
    factorization of eq. "pre".
  * abs_block_diag(D): the positive definite D~ of Section 1: a 1x1 block is
    replaced by its absolute value; a 2x2 block [[a, b], [b, c]] =
    Q diag(l1, l2) Q with Q = [[c, s], [s, -c]] is replaced by
    Q diag(|l1|, |l2|) Q.
  * bp_abs_preconditioner(A): M = P^T L D~ L^T P, for which M^{-1} A has only
    the eigenvalues +1 and -1 (so preconditioned MINRES stops after at most
    two iterations).
  * abs_matrix(A): |A| = V |Lambda| V^T from the full eigendecomposition.
  * smw_inverse(A, V, lam): A^{-1} - 2 V Lambda^{-1} V^T (Section 2.1), equal
    to M_mr^{-1} when V, lam are exact eigenpairs.
"""
from __future__ import annotations

import math

import numpy as np

ALPHA_BP = (1.0 + math.sqrt(17.0)) / 8.0


def bunch_parlett(A: np.ndarray):
    """Returns (perm, L, D, blocks): A[perm][:, perm] = L D L^T, L unit lower
    triangular (identity on 2x2 pivot blocks), D block diagonal, blocks a list
    of (start, size)."""
    A = np.array(A, dtype=np.float64)
    n = A.shape[0]
    perm = np.arange(n)
    L = np.eye(n)
    D = np.zeros((n, n))
    blocks = []
    S = A.copy()       # working (permuted, partially eliminated) matrix

    k = 0
    while k < n:
        R = np.abs(S[k:, k:])
        mu0 = R.max()
        if mu0 == 0.0:               # remaining block is zero: singular A
            blocks += [(i, 1) for i in range(k, n)]
            break
        diag = np.abs(np.diag(S)[k:])
        mu1 = diag.max()
        # L's already-computed columns 0..k-1 must follow the row swaps only
        if mu1 >= ALPHA_BP * mu0:
            i = k + int(np.argmax(diag))
            _swap_rows_only(L, k, i, S, perm)
            d = S[k, k]
            D[k, k] = d
            l = S[k + 1:, k] / d
            L[k + 1:, k] = l
            S[k + 1:, k + 1:] -= np.outer(l, l) * d
            S[k + 1:, k] = 0.0; S[k, k + 1:] = 0.0
            blocks.append((k, 1))
            k += 1
        else:
            off = R.copy()
            np.fill_diagonal(off, -1.0)
            i, j = np.unravel_index(int(np.argmax(off)), off.shape)
            i, j = sorted((k + i, k + j))
            _swap_rows_only(L, k, i, S, perm)
            _swap_rows_only(L, k + 1, j, S, perm)
            E = S[k:k + 2, k:k + 2].copy()
            D[k:k + 2, k:k + 2] = E
            Lb = S[k + 2:, k:k + 2] @ np.linalg.inv(E)
            L[k + 2:, k:k + 2] = Lb
            S[k + 2:, k + 2:] -= Lb @ E @ Lb.T
            S[k + 2:, k:k + 2] = 0.0; S[k:k + 2, k + 2:] = 0.0
            blocks.append((k, 2))
            k += 2
    return perm, L, D, blocks


def _swap_rows_only(L, i, j, S, perm):
    """Symmetric swap of positions i, j in the active matrix; in L only the
    already-computed columns (< i) are row-swapped (standard LDL^T pivoting)."""
    if i == j:
        return
    S[[i, j], :] = S[[j, i], :]
    S[:, [i, j]] = S[:, [j, i]]
    L[[i, j], :i] = L[[j, i], :i]
    perm[[i, j]] = perm[[j, i]]


def spectral_2x2(E: np.ndarray):
    """E = Q diag(l1, l2) Q with Q = [[c, s], [s, -c]], c^2 + s^2 = 1."""
    a, b, c_ = E[0, 0], E[0, 1], E[1, 1]
    mid = 0.5 * (a + c_)
    rad = math.hypot(0.5 * (a - c_), b)
    l1, l2 = mid + rad, mid - rad
    # eigenvector of l1: (b, l1 - a) or (l1 - c, b), whichever is better scaled
    v = np.array([b, l1 - a]) if abs(l1 - a) > abs(l1 - c_) else np.array([l1 - c_, b])
    nv = np.linalg.norm(v)
    if nv == 0.0:                      # E already diagonal
        v = np.array([1.0, 0.0]) if a >= c_ else np.array([0.0, 1.0])
        nv = 1.0
    cs, sn = v / nv
    Q = np.array([[cs, sn], [sn, -cs]])
    return Q, l1, l2


def abs_block_diag(D: np.ndarray, blocks) -> np.ndarray:
    Dt = np.zeros_like(D)
    for (s, size) in blocks:
        if size == 1:
            Dt[s, s] = abs(D[s, s])
        else:
            Q, l1, l2 = spectral_2x2(D[s:s + 2, s:s + 2])
            Dt[s:s + 2, s:s + 2] = Q @ np.diag([abs(l1), abs(l2)]) @ Q
    return Dt


def bp_abs_preconditioner(A: np.ndarray) -> np.ndarray:
    """M = P^T L D~ L^T P (Section 1)."""
    perm, L, D, blocks = bunch_parlett(A)
    Mp = L @ abs_block_diag(D, blocks) @ L.T
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    return Mp[np.ix_(inv, inv)]


def abs_matrix(A: np.ndarray) -> np.ndarray:
    w, V = np.linalg.eigh(A)
    return (V * np.abs(w)) @ V.T


def smw_inverse(A: np.ndarray, V: np.ndarray, lam: np.ndarray) -> np.ndarray:
    return np.linalg.inv(A) - 2.0 * (V / lam) @ V.T
