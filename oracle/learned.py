"""FP64 CPU reference of the learned second-level preconditioner.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain PyTorch CPU ops
in float64; gradients come from autograd and are pinned by finite
differences in the tests.  The paper has no learned component: this network
is defined by this project (a message-passing net over the node graph of A
whose output C gives the SPD inner preconditioner M_cg^{-1} = C C^T); the
GPU kernels implement the same definition independently.

Definition (H = 32 hidden features, bs = unknowns per node, nodes I, J):
  S      = diag(sqrt|a_ii|),  At = S^-1 A S^-1
  x_I    = the bs(bs+1)/2 entries of the lower triangle of the diagonal block
           At_II (row-major order), f_IJ = the bs*bs entries of At_IJ, I != J
  h0_I   = W_in_n x_I,                e0_IJ = W_in_e f_IJ
  layer l = 0..3:
    m_IJ  = relu(W1_l [h_I; h_J; e_IJ] + b1_l)
    e_IJ <- e_IJ + m_IJ
    a_I   = sum_{J != I} m_IJ
    h_I  <- h_I + relu(W2_l [h_I; a_I] + b2_l)
  outputs (J < I):  Ct_IJ = EPS_OFF * reshape(W_oe e_IJ, bs x bs)
           node I:  o = W_od h_I + b_od (bs(bs+1)/2 values, lower triangle
                    row-major); diagonal entries softplus(o) + DIAG_FLOOR,
                    strictly lower entries EPS_OFF * o
  C      = S^-1 Ct (rows scaled), lower triangular on the pattern of lower(A)
Loss for pairs (y_b, z_b):  mean_b ||C C^T y_b - z_b||^2 / ||z_b||^2.
Parameter vector layout: see param_shapes().
"""
from __future__ import annotations

import numpy as np
import torch

H = 32
LAYERS = 4
EPS_OFF = 0.1
DIAG_FLOOR = 1e-3   # keeps C nonsingular when softplus underflows
# softplus(b) = 1 for the initial node bias on the diagonal outputs
SOFTPLUS_ONE = float(np.log(np.e - 1.0))


def param_shapes(bs: int):
    """Ordered (name, shape) of the flat parameter vector."""
    dn = bs * (bs + 1) // 2
    de = bs * bs
    out = [("W_in_n", (H, dn)), ("W_in_e", (H, de))]
    for l in range(LAYERS):
        out += [("W1_%d" % l, (H, 3 * H)), ("b1_%d" % l, (H,)),
                ("W2_%d" % l, (H, 2 * H)), ("b2_%d" % l, (H,))]
    out += [("W_oe", (de, H)), ("W_od", (dn, H)), ("b_od", (dn,))]
    return out


def n_params(bs: int) -> int:
    return int(sum(np.prod(s) for _, s in param_shapes(bs)))


def unpack(theta: torch.Tensor, bs: int):
    p, off = {}, 0
    for name, shp in param_shapes(bs):
        cnt = int(np.prod(shp))
        p[name] = theta[off:off + cnt].reshape(shp)
        off += cnt
    return p


def init_params(bs: int, seed: int) -> np.ndarray:
    """Seeded initialisation (float32 values): Glorot-like weights scaled by
    1/2, zero biases, diagonal output bias softplus^-1(1), so that at start
    C~ is close to the identity (a Jacobi preconditioner)."""
    rng = np.random.default_rng(seed)
    chunks = []
    dn = bs * (bs + 1) // 2
    diag_idx = [a * (a + 1) // 2 + a for a in range(bs)]
    for name, shp in param_shapes(bs):
        if name.startswith("b"):
            v = np.zeros(shp)
            if name == "b_od":
                v[diag_idx] = SOFTPLUS_ONE
        else:
            fan_in = shp[1]
            v = rng.standard_normal(shp) * 0.5 / np.sqrt(fan_in)
            if name in ("W_oe", "W_od"):
                v *= 0.02
        chunks.append(v.ravel())
    return np.concatenate(chunks).astype(np.float32)


class Graph:
    """Node graph of a block-structured sparse A (both directions stored).
    Built from the CSR of A on the host; the same definition is used by the
    GPU path (which builds its own)."""

    def __init__(self, row_ptr, col, val, bs: int):
        row_ptr = np.asarray(row_ptr); col = np.asarray(col); val = np.asarray(val, np.float64)
        n = row_ptr.size - 1
        assert n % bs == 0
        self.n, self.bs, self.N = n, bs, n // bs
        rows = np.repeat(np.arange(n), np.diff(row_ptr))
        diag = np.zeros(n)
        dmask = rows == col
        diag[rows[dmask]] = val[dmask]
        self.s = np.sqrt(np.abs(diag))
        at = val / (self.s[rows] * self.s[col])
        I = rows // bs; J = col // bs; a = rows % bs; b = col % bs
        N = self.N
        key = I * N + J
        # node features: lower triangle of the diagonal blocks, row-major
        self.xn = np.zeros((N, bs * (bs + 1) // 2))
        m = (I == J) & (b <= a)
        self.xn[I[m], a[m] * (a[m] + 1) // 2 + b[m]] = at[m]
        # edges I != J, sorted by (I, J)
        off = I != J
        ukeys = np.unique(key[off])
        self.src = (ukeys // N).astype(np.int64)
        self.dst = (ukeys % N).astype(np.int64)
        self.E = ukeys.size
        eidx = np.searchsorted(ukeys, key[off])
        self.fe = np.zeros((self.E, bs * bs))
        self.fe[eidx, a[off] * bs + b[off]] = at[off]


def forward(theta: torch.Tensor, g: Graph):
    """Returns (Ct_off [E, bs, bs] for all edges (used only where J < I),
    Ct_diag [N, bs, bs] lower triangular)."""
    bs = g.bs
    p = unpack(theta, bs)
    xn = torch.from_numpy(g.xn)
    fe = torch.from_numpy(g.fe)
    src = torch.from_numpy(g.src); dst = torch.from_numpy(g.dst)
    h = xn @ p["W_in_n"].T
    e = fe @ p["W_in_e"].T
    for l in range(LAYERS):
        X = torch.cat([h[src], h[dst], e], dim=1)
        m = torch.relu(X @ p["W1_%d" % l].T + p["b1_%d" % l])
        e = e + m
        agg = torch.zeros_like(h).index_add(0, src, m)
        Xn = torch.cat([h, agg], dim=1)
        h = h + torch.relu(Xn @ p["W2_%d" % l].T + p["b2_%d" % l])
    ct_off = EPS_OFF * (e @ p["W_oe"].T).reshape(g.E, bs, bs)
    o = h @ p["W_od"].T + p["b_od"]
    ct_diag = torch.zeros(g.N, bs, bs, dtype=theta.dtype)
    for a in range(bs):
        for b in range(a + 1):
            v = o[:, a * (a + 1) // 2 + b]
            ct_diag[:, a, b] = (torch.nn.functional.softplus(v) + DIAG_FLOOR) if a == b \
                else EPS_OFF * v
    return ct_off, ct_diag


def assemble_C(theta: torch.Tensor, g: Graph):
    """Dense C (n x n) for tiny graphs: C = S^-1 Ct, lower triangular."""
    ct_off, ct_diag = forward(theta, g)
    bs, n = g.bs, g.n
    C = torch.zeros(n, n, dtype=theta.dtype)
    for e in range(g.E):
        I, J = int(g.src[e]), int(g.dst[e])
        if J < I:
            C[I * bs:(I + 1) * bs, J * bs:(J + 1) * bs] = ct_off[e]
    for I in range(g.N):
        C[I * bs:(I + 1) * bs, I * bs:(I + 1) * bs] = ct_diag[I]
    s = torch.from_numpy(g.s)
    return C / s[:, None]


def csr_C(theta: torch.Tensor, g: Graph, row_ptr, col):
    """Values of C on the lower pattern of A (CSR order), float64 numpy."""
    ct_off, ct_diag = forward(theta, g)
    ct_off = ct_off.detach().numpy(); ct_diag = ct_diag.detach().numpy()
    bs = g.bs
    row_ptr = np.asarray(row_ptr); col = np.asarray(col)
    n = g.n
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    low = col <= rows
    r, c = rows[low], col[low]
    I, J, a, b = r // bs, c // bs, r % bs, c % bs
    key = I * g.N + J
    ekeys = g.src * g.N + g.dst
    vals = np.empty(r.size)
    d = I == J
    vals[d] = ct_diag[I[d], a[d], b[d]]
    eidx = np.searchsorted(ekeys, key[~d])
    vals[~d] = ct_off[eidx, a[~d], b[~d]]
    vals /= g.s[r]
    lp = np.zeros(n + 1, np.int64)
    np.add.at(lp, r + 1, 1)
    return np.cumsum(lp).astype(np.int32), c.astype(np.int32), vals


def loss(theta: torch.Tensor, g: Graph, Y: np.ndarray, Z: np.ndarray):
    """mean_b ||C C^T y_b - z_b||^2 / ||z_b||^2 with dense C (tiny graphs)."""
    C = assemble_C(theta, g)
    Yt = torch.from_numpy(Y); Zt = torch.from_numpy(Z)
    Zh = C @ (C.T @ Yt)
    return (((Zh - Zt) ** 2).sum(0) / (Zt ** 2).sum(0)).mean()
