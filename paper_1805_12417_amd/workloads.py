"""Seeded synthetic workloads: sparse symmetric indefinite systems with few
negative eigenvalues, built by shifting an SPD operator (the construction the
paper uses for its SiO(sigma) instances, Section 3.2, table "UFmatrices").

This module is shared by the oracle and the GPU path.  It holds none of the
solver's arithmetic: it only produces inputs

    A (CSR, int32 row_ptr/col, float64 val), b, V_hat (n x k, column-major
    orthonormal approximate invariant subspace of the k negative
    eigenvalues), lam_hat (k negative eigenvalues),

which are the arguments of Algorithm "minres_cg" (MINRES-CG(A, b, x0,
Lambda_hat, V_hat)).  Computing V_hat / lam_hat is the paper's second setup
stage (Section 2, "three stages"); the paper uses MATLAB eigs for it, here a
dense or shift-invert Lanczos eigensolver (small n) or a Chebyshev-filtered
subspace iteration (large n) is used.

Every array is generated from numpy.random.default_rng(seed).  Readings of
unstated details:
  * 2D/3D Laplacians use Dirichlet boundaries with the boundary nodes
    eliminated; each boundary edge carries its own coefficient, added to the
    diagonal of the adjacent interior node.
  * "exp(N(0, 0.5))": 0.5 is the standard deviation of the normal.
  * A = A0 - sigma*I with sigma midway between the k-th and (k+1)-th smallest
    eigenvalue of the SPD A0, so A has exactly k negative eigenvalues.
  * For the 64x64 2D Laplacian the 5th and 6th eigenvalues coincide (modes
    (1,3) and (3,1)), so "midway between the 5th and 6th" would make A
    singular; k = 6 (sigma between the 6th and 7th) is used instead.
"""
from __future__ import annotations

import math
import sys
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


@dataclass
class Workload:
    """One system A x = b with its deflation data (all host numpy arrays)."""
    name: str
    row_ptr: np.ndarray      # int32 [n+1]
    col: np.ndarray          # int32 [nnz], sorted within each row
    val: np.ndarray          # float64 [nnz]
    b: np.ndarray            # float64 [n] or [n, nrhs] (column j = rhs j)
    Vhat: np.ndarray         # float64 [n, k], Fortran (column-major) order
    lam: np.ndarray          # float64 [k], all < 0
    sigma: float             # shift applied to the SPD A0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def k(self) -> int:
        return int(self.lam.shape[0])

    def scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))


def _csr_parts(A: sp.spmatrix):
    A = sp.csr_matrix(A)
    A.sum_duplicates()
    A.sort_indices()
    return (A.indptr.astype(np.int32), A.indices.astype(np.int32),
            np.ascontiguousarray(A.data, dtype=np.float64))


# --------------------------------------------------------------------------
# Operators
# --------------------------------------------------------------------------

def laplace2d(m: int) -> sp.csr_matrix:
    """5-point Dirichlet Laplacian on an m x m interior grid (diag 4, off -1).
    Node (i, j), i = x index, j = y index, has row i + m*j."""
    e = np.ones(m)
    T = sp.diags([-e[:-1], 2 * e, -e[:-1]], [-1, 0, 1])
    I = sp.identity(m)
    return sp.csr_matrix(sp.kron(I, T) + sp.kron(T, I))


def laplace2d_modes(m: int, count: int):
    """Closed-form lowest `count` eigenpairs of laplace2d(m).

    lambda_{pq} = f(p) + f(q), f(p) = 2 - 2 cos(p pi/(m+1)); eigenvector
    u(i, j) = (2/(m+1)) sin(p i pi/(m+1)) sin(q j pi/(m+1)), i, j = 1..m.
    Ties are broken by (p, q) so that the basis is deterministic."""
    h = math.pi / (m + 1)
    f = 2.0 - 2.0 * np.cos(np.arange(1, m + 1) * h)
    pairs = sorted(((f[p - 1] + f[q - 1], p, q) for p in range(1, m + 1)
                    for q in range(1, m + 1)), key=lambda t: (round(t[0], 14), t[1], t[2]))
    pairs = pairs[:count]
    idx = np.arange(1, m + 1)
    vals = np.array([t[0] for t in pairs])
    vecs = np.empty((m * m, count))
    for c, (_, p, q) in enumerate(pairs):
        sx = np.sin(p * idx * h)
        sy = np.sin(q * idx * h)
        # row = i + m*j: x fastest
        vecs[:, c] = (2.0 / (m + 1)) * np.outer(sy, sx).ravel()
    return vals, vecs


def laplace3d_random(mx: int, my: int, mz: int, rng: np.random.Generator,
                     sd: float = 0.5) -> sp.csr_matrix:
    """7-point Dirichlet operator sum_e c_e (e_i - e_j)(e_i - e_j)^T on an
    mx*my*mz grid with one coefficient c_e = exp(N(0, sd)) per edge,
    boundary edges included (they only add to the diagonal).
    Node (x, y, z) has row x + mx*(y + my*z)."""
    n = mx * my * mz
    cx = np.exp(sd * rng.standard_normal((mz, my, mx + 1)))
    cy = np.exp(sd * rng.standard_normal((mz, my + 1, mx)))
    cz = np.exp(sd * rng.standard_normal((mz + 1, my, mx)))
    diag = (cx[:, :, :-1] + cx[:, :, 1:] + cy[:, :-1, :] + cy[:, 1:, :]
            + cz[:-1, :, :] + cz[1:, :, :]).ravel()
    ids = np.arange(n).reshape(mz, my, mx)
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [diag]
    for a, b_, c in ((ids[:, :, :-1], ids[:, :, 1:], cx[:, :, 1:-1]),
                     (ids[:, :-1, :], ids[:, 1:, :], cy[:, 1:-1, :]),
                     (ids[:-1, :, :], ids[1:, :, :], cz[1:-1, :, :])):
        a = a.ravel(); b_ = b_.ravel(); c = c.ravel()
        rows += [a, b_]; cols += [b_, a]; vals += [-c, -c]
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return sp.csr_matrix(A)


def color8_node_order(m: int) -> np.ndarray:
    """new_index[node] for an m^3 node grid ordered by the 8-colour parity
    classes colour = (x%2) + 2(y%2) + 4(z%2), lexicographic (z, y, x) within a
    colour.  Nodes of one colour are never 27-point neighbours of each other."""
    z, y, x = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    colour = ((x % 2) + 2 * (y % 2) + 4 * (z % 2)).ravel()
    lin = (x + m * (y + m * z)).ravel()
    order = np.lexsort((lin, colour))          # nodes sorted by (colour, lin)
    new = np.empty(m ** 3, dtype=np.int64)
    new[order] = np.arange(m ** 3)
    return new


def fe27_colored(m: int, rng: np.random.Generator, dof: int = 3):
    """FE-elasticity-like SPD operator: 27-point node stencil on an m^3 grid,
    `dof` unknowns per node, A0 = sum_{pairs} (e_i - e_j)(e_i - e_j)^T (x) W_ij
    + sum_{missing neighbours} e_i e_i^T (x) W, W = G G^T/3 + 0.1 I with
    G ~ N(0,1)^{dof x dof} drawn per node pair / per missing neighbour.
    Nodes are numbered in the 8-colour order of color8_node_order; row of
    (node, d) is dof*node + d.  Returns (row_ptr, col, val, colour_ptr) where
    colour_ptr[c] is the first node of colour c (length 9)."""
    N = m ** 3
    newid = color8_node_order(m)
    grid = np.arange(N).reshape(m, m, m)   # [z, y, x] -> lin
    dirs = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
            if (dz, dy, dx) > (0, 0, 0)]
    assert len(dirs) == 13

    def spd_blocks(cnt):
        G = rng.standard_normal((cnt, dof, dof))
        return np.einsum("pij,pkj->pik", G, G) / 3.0 + 0.1 * np.eye(dof)

    I_list, J_list, B_list = [], [], []
    diag = np.zeros((N, dof, dof))
    for (dz, dy, dx) in dirs:
        zs = slice(max(0, -dz), m - max(0, dz))
        ys = slice(max(0, -dy), m - max(0, dy))
        xs = slice(max(0, -dx), m - max(0, dx))
        zt = slice(max(0, dz), m + min(0, dz))
        yt = slice(max(0, dy), m + min(0, dy))
        xt = slice(max(0, dx), m + min(0, dx))
        a = grid[zs, ys, xs].ravel()
        c = grid[zt, yt, xt].ravel()
        W = spd_blocks(a.size)
        np.add.at(diag, a, W)
        np.add.at(diag, c, W)
        I_list += [newid[a], newid[c]]
        J_list += [newid[c], newid[a]]
        B_list += [-W, -W]
    # anchoring: one W for every neighbour slot that falls outside the grid
    z, y, x = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    missing = np.zeros((m, m, m), dtype=np.int64)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if (dz, dy, dx) == (0, 0, 0):
                    continue
                out = ((z + dz < 0) | (z + dz >= m) | (y + dy < 0) | (y + dy >= m)
                       | (x + dx < 0) | (x + dx >= m))
                missing += out
    miss = missing.ravel()
    owners = np.repeat(np.arange(N), miss)
    if owners.size:
        np.add.at(diag, owners, spd_blocks(owners.size))
    inv = np.empty(N, dtype=np.int64)
    inv[newid] = np.arange(N)
    I_list.append(np.arange(N)); J_list.append(np.arange(N)); B_list.append(diag[inv])
    I = np.concatenate(I_list); J = np.concatenate(J_list)
    B = np.concatenate(B_list)
    del I_list, J_list, B_list
    order = np.lexsort((J, I))
    I = I[order]; J = J[order]; B = B[order]
    deg = np.bincount(I, minlength=N)
    start = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(deg, out=start[1:])
    # row (node I, d) holds dof*deg_I entries: blocks of the sorted pairs of I
    row_len = np.repeat(dof * deg, dof)
    row_ptr = np.zeros(N * dof + 1, dtype=np.int64)
    np.cumsum(row_len, out=row_ptr[1:])
    P = I.size
    pidx = np.arange(P) - start[I]                      # position of pair within node I
    base = (dof * dof) * start[I] + dof * pidx           # offset of (d=0, this pair, e=0)
    dd = np.arange(dof)
    pos = (base[:, None, None] + (dof * deg[I])[:, None, None] * dd[None, :, None]
           + dd[None, None, :])
    val = np.empty(P * dof * dof)
    val[pos.ravel()] = B.ravel()
    col = np.empty(P * dof * dof, dtype=np.int64)
    col[pos.ravel()] = (dof * J[:, None, None] + dd[None, None, :]
                        + 0 * dd[None, :, None]).ravel()
    del pos, B
    counts = np.bincount(((np.arange(m)[None, None, :] % 2) + 2 * (np.arange(m)[None, :, None] % 2)
                          + 4 * (np.arange(m)[:, None, None] % 2)).ravel(), minlength=8)
    colour_ptr = np.zeros(9, dtype=np.int64)
    np.cumsum(counts, out=colour_ptr[1:])
    assert row_ptr[-1] < 2 ** 31
    return (row_ptr.astype(np.int32), col.astype(np.int32), val, colour_ptr)


# --------------------------------------------------------------------------
# Second setup stage: lowest eigenpairs of the SPD A0
# --------------------------------------------------------------------------

def _gershgorin_upper(A: sp.csr_matrix) -> float:
    return float(np.max(np.asarray(abs(A).sum(axis=1)).ravel()))


def lowest_eigenpairs(A0: sp.csr_matrix, nev: int, seed: int, device: str = "cpu",
                      tol: float = 1e-10, verbose: bool = False):
    """nev smallest eigenpairs (ascending) of the SPD matrix A0.

    n <= 2500: dense eigh.  Else on the CPU: ARPACK shift-invert Lanczos about
    0 (sparse LU).  device="cuda": Chebyshev-filtered subspace iteration with
    Rayleigh-Ritz (Zhou, Saad, Tiago & Chelikowsky 2006) in torch, for sizes
    where a sparse LU is out of reach.  Eigen-residuals are <= tol*||A0||."""
    n = A0.shape[0]
    if n <= 2500 and device == "cpu":
        w, V = np.linalg.eigh(A0.toarray())
        return w[:nev], np.asfortranarray(V[:, :nev])
    if device == "cpu":
        rng = np.random.default_rng(seed + 7919)
        v0 = rng.standard_normal(n)
        w, V = spla.eigsh(A0.tocsc(), k=nev, sigma=0.0, which="LM", v0=v0, tol=0)
        order = np.argsort(w)
        w, V = w[order], V[:, order]
        # one Rayleigh-Ritz pass restores orthonormality to working precision
        Q, _ = np.linalg.qr(V)
        H = Q.T @ (A0 @ Q)
        w, S = np.linalg.eigh(0.5 * (H + H.T))
        return w, np.asfortranarray(Q @ S)
    return _chefsi_torch(A0, nev, seed, device, tol, verbose=verbose)


def _chefsi_torch(A0: sp.csr_matrix, nev: int, seed: int, device: str, tol: float,
                  degree: int = 48, max_outer: int = 400, verbose: bool = False):
    """Chebyshev-filtered subspace iteration (scaled three-term filter that
    damps [a, ub] and amplifies the wanted low end), Rayleigh-Ritz after each
    filter.  Runs an FP32 phase until the eigen-residuals reach ~1e-5 ub, then
    refines in FP64 to tol * ub.  Orthonormalisation is Cholesky-QR applied
    twice; Gram products are batched over row blocks."""
    import torch
    n = A0.shape[0]
    p = nev + max(8, nev // 2)
    dev = torch.device(device)
    ub = _gershgorin_upper(A0)

    def csr(dtype):
        return torch.sparse_csr_tensor(torch.from_numpy(A0.indptr.astype(np.int64)),
                                       torch.from_numpy(A0.indices.astype(np.int64)),
                                       torch.from_numpy(A0.data.astype(np.float64)),
                                       size=(n, n)).to(dtype).to(dev)

    nb = max(1, min(512, n // 2048))
    rows = -(-n // nb)

    def gram(X, Y):
        pad = nb * rows - n
        if pad:
            X = torch.nn.functional.pad(X, (0, 0, 0, pad)); Y = torch.nn.functional.pad(Y, (0, 0, 0, pad))
        Xb = X.reshape(nb, rows, X.shape[1])
        Yb = Y.reshape(nb, rows, Y.shape[1])
        return torch.bmm(Xb.transpose(1, 2), Yb).sum(0).to(torch.float64)

    def orth(X):
        for _ in range(2):
            G = gram(X, X)
            Rm, info = torch.linalg.cholesky_ex(G, upper=True)
            if int(info) != 0:
                Q, _ = torch.linalg.qr(X.to(torch.float64))
                return Q.to(X.dtype)
            X = X @ torch.linalg.inv(Rm).to(X.dtype)
        return X

    def rr(At, X):
        AX = At @ X
        H = gram(X, AX)
        theta, Q = torch.linalg.eigh(0.5 * (H + H.T))
        Qd = Q.to(X.dtype)
        return theta, X @ Qd, AX @ Qd

    rng = np.random.default_rng(seed + 7919)
    X = torch.from_numpy(rng.standard_normal((n, p))).to(dev)
    outer = 0
    for dtype, target in ((torch.float32, 1e-5), (torch.float64, tol)):
        At = csr(dtype)
        X = orth(X.to(dtype))
        theta, X, AX = rr(At, X)
        for _ in range(max_outer):
            outer += 1
            a = float(theta[-1]); a0 = float(theta[0])
            e = (ub - a) / 2.0; c = (ub + a) / 2.0
            s = e / (a0 - c); tau = 2.0 / s
            Y = At @ X
            Y.add_(X, alpha=-c).mul_(s / e)
            Xp = X
            for _d in range(2, degree + 1):
                s_new = 1.0 / (tau - s)
                Yn = At @ Y
                Yn.add_(Y, alpha=-c).mul_(2.0 * s_new / e).add_(Xp, alpha=-(s * s_new))
                Xp, Y, s = Y, Yn, s_new
            del Xp
            X = orth(Y)
            del Y
            theta, X, AX = rr(At, X)
            R = (AX[:, :nev] - X[:, :nev] * theta[:nev].to(X.dtype)).to(torch.float64)
            res = float(torch.linalg.vector_norm(R, dim=0).max())
            if verbose:
                print("chefsi %s outer %d res/ub %.2e" % (dtype, outer, res / ub), file=sys.stderr,
                      flush=True)
            if res <= target * ub:
                break
        del At
    w = theta[:nev].cpu().numpy()
    V = np.asfortranarray(X[:, :nev].cpu().numpy())
    del X, AX
    return w, V


def shift_to_k_negatives(A0: sp.csr_matrix, k: int, seed: int, device: str = "cpu",
                         verbose: bool = False):
    """A = A0 - sigma I with sigma = (lambda_k + lambda_{k+1})/2 of A0.
    Returns (A, sigma, Vhat, lam_hat, gap) with lam_hat = lambda_{1..k} - sigma."""
    w, V = lowest_eigenpairs(A0, k + 1, seed, device, verbose=verbose)
    sigma = 0.5 * (w[k - 1] + w[k])
    n = A0.shape[0]
    A = sp.csr_matrix(A0 - sigma * sp.identity(n, format="csr"))
    lam = w[:k] - sigma
    return A, float(sigma), np.asfortranarray(V[:, :k]), lam, float(w[k] - w[k - 1])


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

def shifted_laplace2d(seed: int = 1, m: int = 64, k: int = 6) -> Workload:
    """Plain method, FP64: 2D 5-point Laplacian on an m x m grid minus sigma*I,
    sigma midway between the k-th and (k+1)-th eigenvalue (closed form)."""
    A0 = laplace2d(m)
    w, V = laplace2d_modes(m, k + 1)
    sigma = 0.5 * (w[k - 1] + w[k])
    if not w[k] - w[k - 1] > 1e-12:
        raise ValueError("k-th and (k+1)-th eigenvalues coincide: A would be singular")
    A = sp.csr_matrix(A0 - sigma * sp.identity(m * m))
    rp, ci, va = _csr_parts(A)
    rng = np.random.default_rng(seed)
    b = rng.standard_normal(m * m)
    lam = w[:k] - sigma
    return Workload("laplace2d_%dx%d_k%d" % (m, m, k), rp, ci, va, b,
                    np.asfortranarray(V[:, :k]), lam, float(sigma),
                    dict(grid=(m, m), min_abs_eig=float(min(abs(w[k] - sigma), abs(w[k - 1] - sigma))),
                         max_eig=float(8.0 - sigma)))


def shifted_laplace3d(seed: int = 2, m: int = 128, k: int = 20, nrhs: int = 1,
            device: str = "cpu", dims=None, verbose: bool = False) -> Workload:
    """3D 7-point Laplacian with exp(N(0,0.5)) edge coefficients, shifted to
    k negative eigenvalues; b ~ N(0,1) (nrhs columns)."""
    mx, my, mz = dims if dims is not None else (m, m, m)
    rng = np.random.default_rng(seed)
    A0 = laplace3d_random(mx, my, mz, rng)
    b = rng.standard_normal((mx * my * mz, nrhs)) if nrhs > 1 else rng.standard_normal(mx * my * mz)
    A, sigma, V, lam, gap = shift_to_k_negatives(A0, k, seed, device, verbose)
    rp, ci, va = _csr_parts(A)
    return Workload("laplace3d_rand_%dx%dx%d_k%d" % (mx, my, mz, k), rp, ci, va,
                    np.asfortranarray(b), V, lam, sigma,
                    dict(grid=(mx, my, mz), min_abs_eig=gap / 2.0, max_eig=_gershgorin_upper(A)))


def shifted_fe27(seed: int = 3, m: int = 80, k: int = 30, device: str = "cpu",
            verbose: bool = False) -> Workload:
    """FE-elasticity-like 27-point, 3 dof/node, 8-colour node order, shifted
    to k negative eigenvalues; b ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    rp, ci, va, colour_ptr = fe27_colored(m, rng)
    n = rp.shape[0] - 1
    b = rng.standard_normal(n)
    A0 = sp.csr_matrix((va, ci, rp), shape=(n, n))
    A, sigma, V, lam, gap = shift_to_k_negatives(A0, k, seed, device, verbose)
    # the shift touches only the (present) diagonal: keep the pattern and order
    rp2, ci2, va2 = _csr_parts(A)
    assert rp2.shape == rp.shape and ci2.shape == ci.shape
    return Workload("fe27_%d^3x3_k%d" % (m, k), rp2, ci2, va2, b, V, lam, sigma,
                    dict(grid=(m, m, m), dof=3, colour_node_ptr=colour_ptr,
                         min_abs_eig=gap / 2.0, max_eig=_gershgorin_upper(A)))


def lowest_eigenpairs_indefinite(A: sp.csr_matrix, nev: int, seed: int, lower: float,
                                 device: str = "cpu", verbose: bool = False):
    """nev algebraically smallest eigenpairs of a symmetric indefinite A, given
    a lower bound `lower` on its spectrum.  n <= 2500: dense eigh; CPU:
    shift-invert Lanczos about `lower` (the eigenvalues closest to it are the
    smallest); device="cuda": the Chebyshev-filtered subspace iteration,
    which needs no definiteness."""
    n = A.shape[0]
    if n <= 2500 and device == "cpu":
        w, V = np.linalg.eigh(A.toarray())
        return w[:nev], np.asfortranarray(V[:, :nev])
    if device == "cpu":
        rng = np.random.default_rng(seed + 7919)
        w, V = spla.eigsh(A.tocsc(), k=nev, sigma=lower, which="LM",
                          v0=rng.standard_normal(n), tol=0)
        order = np.argsort(w)
        Q, _ = np.linalg.qr(V[:, order])
        H = Q.T @ (A @ Q)
        w, S = np.linalg.eigh(0.5 * (H + H.T))
        return w, np.asfortranarray(Q @ S)
    return _chefsi_torch(A, nev, seed, device, 1e-10, verbose=verbose)


def brake_inner_level(m: int = 16, k: int = 6, seed: int = 7, mass_scale: float = 1e-3,
                      device: str = "cpu", verbose: bool = False) -> Workload:
    """Synthetic stand-in for the inner-level system of the disk-brake pipeline
    (Section 3.1, eq. "inner_level"): A = K_E - |gamma|^2 M with K_E the
    FE-like SPD stiffness of fe27_colored (m^3 nodes x 3 dof) and M a lumped
    (diagonal) SPD mass matrix, one random mass per node (the same for its 3
    dof), scaled so that ||M||_F << ||K_E||_F as in the brake models.
    |gamma|^2 is placed midway between the k-th and (k+1)-th eigenvalue of the
    pencil (K_E, M) (computed on D^{-1/2} K_E D^{-1/2}, D = M), so that by
    Sylvester's law A has exactly k negative eigenvalues; V_hat, lam_hat are
    A's own k negative eigenpairs.  b is the right-hand side of the first
    sweep point (brake_sweep_rhs)."""
    rng = np.random.default_rng(seed)
    rp, ci, va, colour_ptr = fe27_colored(m, rng)
    n = rp.shape[0] - 1
    K = sp.csr_matrix((va, ci, rp), shape=(n, n))
    node_mass = rng.uniform(0.5, 1.5, n // 3)
    mass = mass_scale * float(np.mean(K.diagonal())) * np.repeat(node_mass, 3)
    Dm = sp.diags(1.0 / np.sqrt(mass))
    Ks = sp.csr_matrix(Dm @ K @ Dm)
    mu, _ = lowest_eigenpairs(Ks, k + 1, seed, device, verbose=verbose)
    g2 = 0.5 * (mu[k - 1] + mu[k])
    A = sp.csr_matrix(K - g2 * sp.diags(mass))
    rp2, ci2, va2 = _csr_parts(A)
    assert rp2.shape == rp.shape and ci2.shape == ci.shape
    lower = -g2 * float(mass.max()) * 1.05        # K_E >= 0, so A >= -|gamma|^2 max(M)
    w, V = lowest_eigenpairs_indefinite(A, k + 1, seed, lower, device, verbose)
    if not (w[k - 1] < 0.0 < w[k]):
        raise ValueError("inertia of K_E - |gamma|^2 M is not (k negative): %r" % (w[:k + 1],))
    w_all_hi = _gershgorin_upper(A)
    wl = Workload("brake_inner_%d^3x3_k%d" % (m, k), rp2, ci2, va2, np.zeros(n),
                  np.asfortranarray(V[:, :k]), w[:k], float(g2),
                  dict(grid=(m, m, m), dof=3, colour_node_ptr=colour_ptr, gamma_abs2=float(g2),
                       mass=mass, pencil_mu=mu, min_abs_eig=float(min(-w[k - 1], w[k])),
                       max_eig=w_all_hi))
    wl.b = brake_sweep_rhs(wl, 1, seed)[0][1]
    return wl


def brake_sweep_rhs(w: Workload, count: int, seed: int):
    """Right-hand sides of the inner-level systems for `count` shifts of the
    same modulus: gamma_j = |gamma| exp(i theta_j), theta_j spread over
    (0, pi/2) (Re and Im gamma > 0, the audible quadrant), b_j = -Im(gamma_j)
    v_j with v_j ~ N(0, I) from the seed.  Every system has the matrix of w
    (Section 3.1: the coefficient matrix depends on |gamma| only).  Returns
    [(gamma_j, b_j)]."""
    rng = np.random.default_rng(seed + 17)
    g = math.sqrt(w.meta["gamma_abs2"])
    out = []
    for j in range(count):
        th = (j + 1) * (math.pi / 2) / (count + 1)
        gamma = complex(g * math.cos(th), g * math.sin(th))
        out.append((gamma, -gamma.imag * rng.standard_normal(w.n)))
    return out


def kkt_saddle(m: int = 32, n_con: int = 16, seed: int = 9, per_row: int = 6,
               interleave: bool = True, coupling: float = 1.0, device: str = "cpu",
               verbose: bool = False) -> Workload:
    """Equality-constrained quadratic program, [[K, B^T], [B, 0]]: K the 2D
    Laplacian laplace2d(m) (SPD, m^2 unknowns), B n_con constraint rows, each
    coupling `per_row` random unknowns with N(0, coupling^2) weights (full row
    rank with probability one).  By Sylvester's law the matrix has exactly n_con
    negative eigenvalues; the (2, 2) block is zero and absent from the
    pattern, so a factorization without pivoting meets zero pivots there.
    This is the saddle-point structure of several of the paper's test
    matrices (Section 4); V_hat, lam_hat are its n_con negative
    eigenpairs, b ~ N(0, 1).  interleave: each constraint row is placed just
    before the first unknown it couples (the unknown order of mixed FE
    discretizations), so that a factorization in the given order meets the
    zero diagonal early; otherwise the constraints come last."""
    if n_con < 1 or n_con > 64 or per_row < 1:
        raise ValueError("n_con must be in 1..64 and per_row >= 1")
    rng = np.random.default_rng(seed)
    K = laplace2d(m)
    n1 = m * m
    rows, cols, vals = [], [], []
    for r in range(n_con):
        c = rng.choice(n1, size=per_row, replace=False)
        rows.append(np.full(per_row, r))
        cols.append(c)
        vals.append(coupling * rng.standard_normal(per_row))
    B = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n_con, n1))
    A = sp.bmat([[K, B.T], [B, None]], format="csr")
    n = n1 + n_con
    if interleave:
        first = np.asarray([B.indices[B.indptr[r]:B.indptr[r + 1]].min() for r in range(n_con)])
        key = np.concatenate([np.arange(n1, dtype=np.float64), first - 0.5])
        order = np.argsort(key, kind="stable")          # new position -> old index
        A = sp.csr_matrix(A[order][:, order])
    rp, ci, va = _csr_parts(A)
    lower = -float(np.max(np.asarray(abs(B).sum(axis=1)).ravel())) * 1.05 - 1.0
    w, V = lowest_eigenpairs_indefinite(sp.csr_matrix((va, ci, rp), shape=(n, n)), n_con + 1,
                                        seed, lower, device, verbose)
    if not (w[n_con - 1] < 0.0 < w[n_con]):
        raise ValueError("inertia of the KKT matrix is not (n_con negative): %r" % (w,))
    b = rng.standard_normal(n)
    Af = sp.csr_matrix((va, ci, rp), shape=(n, n))
    return Workload("kkt_lap2d_%d_c%d%s" % (m, n_con, "i" if interleave else ""), rp, ci, va, b,
                    np.asfortranarray(V[:, :n_con]), w[:n_con], 0.0,
                    dict(grid=(m, m), n_con=n_con, interleave=interleave, coupling=coupling,
                         min_abs_eig=float(min(-w[n_con - 1], w[n_con])),
                         max_eig=_gershgorin_upper(Af)))


def batch_sizes(count: int = 48, lo: float = 2e4, hi: float = 5e5, seed: int = 4000):
    """Uneven system sizes drawn log-uniform in [lo, hi] and k ~ U{2..40}."""
    rng = np.random.default_rng(seed)
    ns = np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))
    ks = rng.integers(2, 41, size=count)
    out = []
    for nn, kk in zip(ns, ks):
        mxy = max(2, int(round(nn ** (1.0 / 3.0))))
        mz = max(2, int(round(nn / (mxy * mxy))))
        out.append(((mxy, mxy, mz), int(kk)))
    return out
