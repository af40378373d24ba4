"""Learned second-level preconditioner M_cg^{-1} = C C^T (include/mcg_learned.h).

A message-passing network over the node graph of A outputs a lower-triangular
C with a positive diagonal on the pattern of lower(A); the inner CG of
MINRES-CG (Section 2, the CG on M_mr) then uses C C^T, which is SPD for any
weights.  Inference, loss, backward and Adam all run in the library's HIP
kernels; this module only marshals arguments, draws the initial weights and
the training pairs, and drives the training loop.

Training pairs (y, z) satisfy z = M_mr^{-1} y:
  * "solver": the right-hand sides y that MINRES hands to the inner solves
    of the solver's own solves (random b), and the inner CG's results z
    (minres_cg_solve_record): the (residual, inner-CG solution) pairs;
  * "cg": y ~ N(0, I), z = the inner CG solution (the solver's own PCG with
    the incomplete LDL^T(0) preconditioner, tight tolerance);
  * "mx": z ~ N(0, I), y = M_mr z (the solver's M_mr apply): the pair an
    exact inner solve would give, weighting all of M_mr's spectrum evenly.
"""
from __future__ import annotations

import ctypes as C
import math
import sys
import time

import numpy as np
import torch

from . import _native as N
from .solver import MinresCG, Preconditioner, _check, _dev, _ptr, _stream

HIDDEN = 32
LAYERS = 4


def param_layout(bs: int):
    """(name, shape) of the flat parameter vector, in the header's order."""
    dn, de = bs * (bs + 1) // 2, bs * bs
    out = [("W_in_n", (HIDDEN, dn)), ("W_in_e", (HIDDEN, de))]
    for l in range(LAYERS):
        out += [("W1_%d" % l, (HIDDEN, 3 * HIDDEN)), ("b1_%d" % l, (HIDDEN,)),
                ("W2_%d" % l, (HIDDEN, 2 * HIDDEN)), ("b2_%d" % l, (HIDDEN,))]
    out += [("W_oe", (de, HIDDEN)), ("W_od", (dn, HIDDEN)), ("b_od", (dn,))]
    return out


def initial_params(bs: int, seed: int = 0) -> np.ndarray:
    """Seeded starting weights: scaled Glorot-normal matrices, zero biases,
    small output heads and a diagonal output bias of softplus^{-1}(1), so the
    initial C is close to diag(|a_ii|)^{-1/2} (a Jacobi preconditioner)."""
    rng = np.random.default_rng(seed)
    chunks = []
    for name, shp in param_layout(bs):
        if len(shp) == 1:
            v = np.zeros(shp)
            if name == "b_od":
                for a in range(bs):
                    v[a * (a + 3) // 2] = math.log(math.e - 1.0)
        else:
            v = rng.standard_normal(shp) * (0.5 / math.sqrt(shp[1]))
            if name in ("W_oe", "W_od"):
                v *= 0.02
        chunks.append(v.ravel())
    return np.concatenate(chunks).astype(np.float32)


class LearnedFactor:
    """Network state and C for one matrix A (device CSR, FP64 values)."""

    def __init__(self, row_ptr, col, val, block_size: int = 1, theta=None, seed: int = 0,
                 stream=None):
        _dev(row_ptr, torch.int32, "row_ptr"); _dev(col, torch.int32, "col")
        _dev(val, torch.float64, "val")
        self.n = row_ptr.numel() - 1
        self.bs = int(block_size)
        self.device = row_ptr.device
        self._A = N.CSR(self.n, col.numel(), row_ptr.data_ptr(), col.data_ptr(), val.data_ptr())
        self.h = C.c_void_p()
        _check(N.lib().mcg_learned_create(C.byref(self.h), C.byref(self._A), self.bs,
                                          _stream(stream)), "mcg_learned_create")
        self.num_params = int(N.lib().mcg_learned_num_params(self.h))
        nodes, edges, nnzc = C.c_int64(), C.c_int64(), C.c_int64()
        _check(N.lib().mcg_learned_sizes(self.h, C.byref(nodes), C.byref(edges), C.byref(nnzc)),
               "mcg_learned_sizes")
        self.nodes, self.edges, self.nnz_c = nodes.value, edges.value, nnzc.value
        if theta is None:
            theta = initial_params(self.bs, seed)
        self.set_params(theta, stream)
        self.grad = torch.zeros(self.num_params, dtype=torch.float32, device=self.device)

    # -- parameters --------------------------------------------------------
    def set_params(self, theta, stream=None):
        t = torch.as_tensor(np.asarray(theta, np.float32) if not isinstance(theta, torch.Tensor)
                            else theta, dtype=torch.float32).to(self.device).contiguous()
        if t.numel() != self.num_params:
            raise ValueError("expected %d parameters, got %d" % (self.num_params, t.numel()))
        _check(N.lib().mcg_learned_set_params(self.h, _ptr(t), _stream(stream)),
               "mcg_learned_set_params")
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()

    def params(self, stream=None) -> torch.Tensor:
        t = torch.empty(self.num_params, dtype=torch.float32, device=self.device)
        _check(N.lib().mcg_learned_get_params(self.h, _ptr(t), _stream(stream)),
               "mcg_learned_get_params")
        return t

    # -- inference -----------------------------------------------------------
    def forward(self, stream=None):
        """Runs the network; returns C as (row_ptr, col, val) device tensors."""
        _check(N.lib().mcg_learned_forward(self.h, _stream(stream)), "mcg_learned_forward")
        rp = torch.empty(self.n + 1, dtype=torch.int32, device=self.device)
        ci = torch.empty(self.nnz_c, dtype=torch.int32, device=self.device)
        cv = torch.empty(self.nnz_c, dtype=torch.float64, device=self.device)
        _check(N.lib().mcg_learned_factor_copy(self.h, _ptr(rp), _ptr(ci), _ptr(cv),
                                               _stream(stream)), "mcg_learned_factor_copy")
        return rp, ci, cv

    def forward_ms(self) -> float:
        return float(N.lib().mcg_learned_forward_ms(self.h))

    def preconditioner(self, solver: MinresCG, smw: bool = False, stream=None) -> Preconditioner:
        """Inner preconditioner C C^T for `solver` from a fresh forward pass."""
        return solver.preconditioner("cct", smw=smw, C_csr=self.forward(stream), stream=stream)

    # -- training ------------------------------------------------------------
    def loss_grad(self, Y: torch.Tensor, Z: torch.Tensor, stream=None):
        """Loss and gradient for pairs given as n x nb row-interleaved FP32
        tensors (nb a power of two <= 32)."""
        _dev(Y, torch.float32, "Y"); _dev(Z, torch.float32, "Z")
        if Y.dim() != 2 or Y.shape != Z.shape or Y.shape[0] != self.n:
            raise ValueError("Y and Z must both be n x nb")
        loss = C.c_double()
        _check(N.lib().mcg_learned_loss_grad(self.h, _ptr(Y), _ptr(Z), int(Y.shape[1]),
                                             C.byref(loss), _ptr(self.grad), _stream(stream)),
               "mcg_learned_loss_grad")
        return float(loss.value), self.grad

    def close(self):
        if self.h:
            N.lib().mcg_learned_free(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_pairs(solver: MinresCG, count: int, kind: str, seed: int, pc: Preconditioner = None,
               rtol: float = 1e-6):
    """Training pairs (Y, Z) as n x count FP32 tensors, z = M_mr^{-1} y
    (see the module docstring for the two kinds)."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    n = solver.n
    Y = torch.empty(n, count, dtype=torch.float32, device="cuda")
    Z = torch.empty_like(Y)
    for j in range(count):
        v = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
        if kind == "mx":
            y, z = solver.mmr_apply(v), v
        elif kind == "cg":
            if pc is None:
                raise ValueError("kind 'cg' needs the inner CG's preconditioner")
            z, rc, _ = solver.pcg(v, pc, rtol=rtol)
            if rc != N.OK:
                raise RuntimeError("inner CG did not converge while making pairs (%d)" % rc)
            y = v
        else:
            raise ValueError("kind must be 'mx' or 'cg'")
        Y[:, j] = y.float()
        Z[:, j] = z.float()
    return Y, Z


def make_solver_pairs(solver: MinresCG, pc: Preconditioner, count: int, seed: int,
                      rtol_out: float = 1e-8, rtol_in: float = 1e-4):
    """`count` (residual, inner-CG solution) pairs from the solver's own
    solves of A x = b, b ~ N(0, I): each solve contributes every inner solve
    MINRES runs (its right-hand side and the inner CG's result).  Returns
    (Y, Z) as n x count FP32 tensors and the number of solves."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    n = solver.n
    Y = torch.empty(n, count, dtype=torch.float32, device="cuda")
    Z = torch.empty_like(Y)
    have, solves = 0, 0
    while have < count:
        b = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
        _, st, Yr, Zr = solver.solve_record(b, pc, count - have, rtol_out=rtol_out,
                                            rtol_in=rtol_in)
        solves += 1
        k = Yr.shape[1]
        if k == 0:
            raise RuntimeError("a solve recorded no inner solve (status %s)" % st.status_name)
        Y[:, have:have + k] = Yr.float()
        Z[:, have:have + k] = Zr.float()
        have += k
    return Y, Z, solves


class Adam:
    """Adam state (FP32 theta and moments on the device) shared by the
    handles of all training matrices; the update runs in the library."""

    def __init__(self, theta: torch.Tensor, lr=2e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.theta = theta.detach().clone().float().contiguous()
        self.m1 = torch.zeros_like(self.theta)
        self.m2 = torch.zeros_like(self.theta)
        self.lr, self.beta1, self.beta2, self.eps = lr, beta1, beta2, eps
        self.step = 0

    def update(self, grad: torch.Tensor, lr=None, stream=None):
        _dev(grad, torch.float32, "grad")
        self.step += 1
        _check(N.lib().mcg_learned_adam(self.theta.numel(), _ptr(self.theta), _ptr(grad),
                                        _ptr(self.m1), _ptr(self.m2),
                                        self.lr if lr is None else lr, self.beta1, self.beta2,
                                        self.eps, self.step, _stream(stream)),
               "mcg_learned_adam")


def train(factors, pairs, steps: int, nb: int = 16, lr: float = 2e-3, seed: int = 0,
          log_every: int = 0, lr_final_frac: float = 0.1, theta=None):
    """Adam on the loss over several matrices sharing one parameter vector.
    `factors` are LearnedFactor handles (one per matrix) and `pairs` the
    matching (Y, Z) pools (n x count FP32); step t draws nb random pairs of
    matrix t mod len(factors).  The learning rate decays by a cosine to
    lr * lr_final_frac.  Returns (theta, loss history)."""
    rng = np.random.default_rng(seed)
    opt = Adam(factors[0].params() if theta is None else
               torch.as_tensor(theta, dtype=torch.float32, device=factors[0].device), lr=lr)
    hist = []
    t0 = time.perf_counter()
    for step in range(steps):
        i = step % len(factors)
        f = factors[i]
        Y, Z = pairs[i]
        cols = torch.from_numpy(rng.choice(Y.shape[1], size=nb, replace=Y.shape[1] < nb)).to(
            Y.device)
        Yb = Y.index_select(1, cols).contiguous()
        Zb = Z.index_select(1, cols).contiguous()
        f.set_params(opt.theta)
        loss, grad = f.loss_grad(Yb, Zb)
        frac = lr_final_frac + (1 - lr_final_frac) * 0.5 * (1 + math.cos(math.pi * step / steps))
        opt.update(grad, lr=lr * frac)
        hist.append(loss)
        if log_every and (step % log_every == 0 or step == steps - 1):
            print("train step %d/%d loss %.4e (%.1fs)" % (step, steps, loss,
                                                        time.perf_counter() - t0),
                  file=sys.stderr, flush=True)
    for f in factors:
        f.set_params(opt.theta)
    return opt.theta.clone(), hist


def fit(workloads, block_size: int, pairs_per_matrix: int = 256, steps: int = 600, nb: int = 16,
        lr: float = 3e-3, seed: int = 0, log=None, pairs_kind: str = "mx"):
    """Trains one parameter vector on a family of matrices (workloads.Workload
    objects with their deflation data), then `steps` Adam steps.  Pairs
    (pairs_kind): "mx", y = M_mr z, z ~ N(0, I) from each matrix's own M_mr
    apply; "solver", the (residual, inner-CG solution) pairs of the solver's
    own solves (FP64, Jacobi second level, rtol_in 1e-4).  Returns (theta,
    loss history, seconds)."""
    from .solver import from_workload
    t0 = time.perf_counter()
    solvers, factors, pairs = [], [], []
    try:
        for i, w in enumerate(workloads):
            s, _ = from_workload(w, precision=N.PREC_FP64)
            solvers.append(s)
            dev = torch.device("cuda")
            factors.append(LearnedFactor(torch.from_numpy(w.row_ptr).to(dev),
                                         torch.from_numpy(w.col).to(dev),
                                         torch.from_numpy(w.val).to(dev), block_size=block_size,
                                         theta=initial_params(block_size, seed)))
            if pairs_kind == "solver":
                pc = s.preconditioner("jacobi")
                Y, Z, _ = make_solver_pairs(s, pc, pairs_per_matrix, seed=seed * 1000 + i)
                pc.close()
                pairs.append((Y, Z))
            else:
                pairs.append(make_pairs(s, pairs_per_matrix, "mx", seed=seed * 1000 + i))
        theta, hist = train(factors, pairs, steps=steps, nb=nb, lr=lr, seed=seed,
                            log_every=(steps // 4 if log else 0))
        torch.cuda.synchronize()
    finally:
        for f in factors:
            f.close()
        for s in solvers:
            s.close()
    dt = time.perf_counter() - t0
    if log:
        log("learned: trained on %d matrices, %d steps, loss %.3e -> %.3e, %.1fs" % (
            len(workloads), steps, float(np.mean(hist[:10])), float(np.mean(hist[-50:])), dt))
    return theta, hist, dt
