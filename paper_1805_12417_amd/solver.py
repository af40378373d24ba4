"""Python front end of the MINRES-CG HIP library.

Torch tensors provide device memory and the stream; the arrays go to the C
ABI as raw pointers and every computation happens in the library's kernels.
There is no fallback: without the built library or a GPU the calls raise.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _native as N
from ._native import (PC_CCT, PC_ILDL0, PC_ILDLP, PC_JACOBI, PC_NONE, PC_SMW,  # noqa: F401
                      PREC_FP64, PREC_MIXED)


class MCGError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s failed: %s (%d)" % (what, N.strerror(code), code))
        self.code = code


def _check(code, what):
    if code < 0:
        raise MCGError(code, what)
    return code


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


@dataclass
class SolveStats:
    status: int
    outer_its: int
    inner_its_total: int
    final_relres: float
    bnorm: float
    inner_its: np.ndarray
    relres: np.ndarray
    phibar: np.ndarray

    @property
    def status_name(self):
        return N.STATUS_NAMES.get(self.status, str(self.status))


class Preconditioner:
    """Second-level preconditioner M_cg (owned by the library)."""

    def __init__(self, solver: "MinresCG", kind: int, params=None, stream=None):
        self.solver = solver
        self.kind = kind
        self.h = C.c_void_p()
        self._keep = params
        p = C.c_void_p(0)
        if isinstance(params, (N.CSR, N.IldlpParams)):
            p = C.cast(C.pointer(params), C.c_void_p)
        elif isinstance(params, float):
            self._pivtol = C.c_double(params)
            p = C.cast(C.pointer(self._pivtol), C.c_void_p)
        _check(N.lib().minres_cg_precond_create(C.byref(self.h), solver.h, kind, p, _stream(stream)),
               "minres_cg_precond_create")

    def apply(self, g: torch.Tensor, precision: int = PREC_FP64, out=None, stream=None):
        dt = torch.float64 if precision == PREC_FP64 else torch.float32
        _dev(g, dt, "g")
        t = out if out is not None else torch.empty_like(g)
        _check(N.lib().mcg_precond_apply(self.h, precision, _ptr(g), _ptr(t), _stream(stream)),
               "mcg_precond_apply")
        return t

    def ildlp_factor(self):
        """The pivoted incomplete factor P A P^T ~ L D L^T (host copies):
        dict of perm, bsize, dd, doff, l_ptr, l_col, l_val."""
        nz = C.c_int64(0)
        vp0 = C.c_void_p(0)
        _check(N.lib().mcg_ildlp_factor_get(self.h, vp0, vp0, vp0, vp0, vp0, vp0, vp0,
                                            C.byref(nz)), "mcg_ildlp_factor_get")
        n, m = self.solver.n, nz.value
        out = {"perm": np.zeros(n, np.int32), "bsize": np.zeros(n, np.int32),
               "dd": np.zeros(n), "doff": np.zeros(n), "l_ptr": np.zeros(n + 1, np.int32),
               "l_col": np.zeros(max(m, 1), np.int32), "l_val": np.zeros(max(m, 1))}
        ptr = {k: v.ctypes.data_as(C.c_void_p) for k, v in out.items()}
        _check(N.lib().mcg_ildlp_factor_get(self.h, ptr["perm"], ptr["bsize"], ptr["dd"],
                                            ptr["doff"], ptr["l_ptr"], ptr["l_col"],
                                            ptr["l_val"], C.byref(nz)), "mcg_ildlp_factor_get")
        out["l_col"], out["l_val"] = out["l_col"][:m], out["l_val"][:m]
        return out

    def close(self):
        if self.h:
            N.lib().minres_cg_precond_free(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MinresCG:
    """Solver for A x = b, A sparse symmetric indefinite with k negative
    eigenvalues whose eigenvectors Vhat (n x k) and eigenvalues lam (< 0) are
    given (Algorithm "minres_cg": MINRES-CG(A, b, x0, Lambda_hat, V_hat)).

    row_ptr, col: int32 CUDA tensors; val: float64; Vhat: float64 (n, k);
    lam: float64 (k,).  precision: PREC_FP64 or PREC_MIXED (FP32 inner CG)."""

    def __init__(self, row_ptr, col, val, Vhat=None, lam=None, precision=PREC_FP64,
                 lanes=0, autotune=False, stag_window=10, keep_best=True, block_size=1,
                 chunk=0, profile=False, mmr_form=0, spmv_format=0, eager=False, xcd_order=0,
                 stream=None):
        _dev(row_ptr, torch.int32, "row_ptr")
        _dev(col, torch.int32, "col")
        _dev(val, torch.float64, "val")
        self.n = row_ptr.numel() - 1
        self.nnz = col.numel()
        if Vhat is not None and Vhat.numel() > 0:
            if Vhat.dim() != 2 or Vhat.shape[0] != self.n:
                raise ValueError("Vhat must have shape (n, k)")
            Vt = _dev(Vhat.t().contiguous(), torch.float64, "Vhat")  # column-major storage
            lam = _dev(lam, torch.float64, "lam")
            self.k = Vhat.shape[1]
        else:
            Vt, lam, self.k = None, None, 0
        self.precision = precision
        opt = N.Options()
        N.lib().minres_cg_default_options(C.byref(opt))
        opt.precision = precision
        opt.spmv_lanes = lanes
        opt.autotune = 1 if autotune else 0
        opt.stag_window = stag_window
        opt.keep_best = 1 if keep_best else 0
        opt.block_size = block_size
        opt.chunk = chunk
        opt.profile = int(profile) if profile else 0   # True/1: M_mr apply, 2: A p
        opt.mmr_form = mmr_form
        opt.spmv_format = spmv_format
        opt.xcd_order = xcd_order
        opt.eager = 1 if eager else 0
        A = N.CSR(self.n, self.nnz, row_ptr.data_ptr(), col.data_ptr(), val.data_ptr())
        self.h = C.c_void_p()
        _check(N.lib().minres_cg_create(C.byref(self.h), C.byref(A), self.k, _ptr(Vt), _ptr(lam),
                                        C.byref(opt), _stream(stream)), "minres_cg_create")
        self.device = row_ptr.device

    # -- second-level preconditioners ------------------------------------
    def preconditioner(self, kind: str = "jacobi", smw: bool = False, pivtol=None, C_csr=None,
                       fill=3.0, drop=1e-3, sweeps=0, stream=None) -> Preconditioner:
        """kind: "none", "jacobi", "ildl0" (pivtol), "ildlp" (fill, drop:
        ILDL^T(fill, drop) with 1x1 / 2x2 pivoting; sweeps > 0: Jacobi
        sweeps instead of the triangular solves) or "cct" (C_csr)."""
        kinds = {"none": PC_NONE, "jacobi": PC_JACOBI, "ildl0": PC_ILDL0, "ildlp": PC_ILDLP,
                 "cct": PC_CCT}
        code = kinds[kind] | (PC_SMW if smw else 0)
        params = None
        if kind == "ildl0" and pivtol is not None:
            params = float(pivtol)
        if kind == "ildlp":
            params = N.IldlpParams(float(fill), float(drop), int(sweeps))
        if kind == "cct":
            rp, ci, cv = C_csr
            _dev(rp, torch.int32, "C.row_ptr"); _dev(ci, torch.int32, "C.col")
            _dev(cv, torch.float64, "C.val")
            params = N.CSR(rp.numel() - 1, ci.numel(), rp.data_ptr(), ci.data_ptr(), cv.data_ptr())
        return Preconditioner(self, code, params, stream)

    # -- the solve ---------------------------------------------------------
    def solve(self, b, pc: Preconditioner, x0=None, rtol_out=1e-8, rtol_in=1e-3, maxit_out=200,
              maxit_inner_total=10 ** 8, hist_cap=None, stream=None):
        """b: (n,) or (nrhs, n) float64 CUDA tensor (row j = right-hand side
        j, solved one after the other).  Returns (x, SolveStats) for a 1-D b,
        (x, [SolveStats per right-hand side]) for a 2-D b."""
        _dev(b, torch.float64, "b")
        multi = b.dim() == 2
        if b.shape[-1] != self.n or b.dim() not in (1, 2) or (multi and b.shape[0] < 1):
            raise ValueError("b must have shape (n,) or (nrhs, n)")
        b = b.contiguous()
        nrhs = b.shape[0] if multi else 1
        x = torch.zeros_like(b) if x0 is None else _dev(x0, torch.float64, "x0").clone()
        if x.shape != b.shape:
            raise ValueError("x0 must have the shape of b")
        cap = (maxit_out + 2) if hist_cap is None else hist_cap
        hist = [(np.zeros(cap, np.int64), np.full(cap, np.nan), np.full(cap, np.nan))
                for _ in range(nrhs)]
        sts = (N.Stats * nrhs)()
        for j, (inner, rel, phb) in enumerate(hist):
            sts[j].hist_cap = cap
            sts[j].inner_its = inner.ctypes.data_as(C.POINTER(C.c_int64))
            sts[j].relres = rel.ctypes.data_as(C.POINTER(C.c_double))
            sts[j].phibar = phb.ctypes.data_as(C.POINTER(C.c_double))
        rc = N.lib().minres_cg_solve(self.h, pc.h, _ptr(b), _ptr(x), nrhs, rtol_out, rtol_in,
                                     maxit_out, int(maxit_inner_total), sts, _stream(stream))
        _check(rc, "minres_cg_solve")
        out = []
        for j, (inner, rel, phb) in enumerate(hist):
            st = sts[j]
            k = st.outer_its
            out.append(SolveStats(int(st.status), int(k), int(st.inner_its_total),
                                  float(st.final_relres), float(st.bnorm), inner[:k + 1].copy(),
                                  rel[:k + 1].copy(), phb[:k + 1].copy()))
        return x, (out if multi else out[0])

    def solve_record(self, b, pc: Preconditioner, cap, x0=None, rtol_out=1e-8, rtol_in=1e-3,
                     maxit_out=200, maxit_inner_total=10 ** 8, stream=None):
        """solve() that also returns the first `cap` inner solves' right-hand
        sides Y and results Z (float64 tensors (n, count)): the solver's own
        (residual, inner-CG solution) pairs."""
        _dev(b, torch.float64, "b")
        if b.numel() != self.n:
            raise ValueError("b has the wrong length")
        x = torch.zeros_like(b) if x0 is None else _dev(x0, torch.float64, "x0").clone()
        Yt = torch.empty((max(cap, 1), self.n), dtype=torch.float64, device=b.device)
        Zt = torch.empty_like(Yt)
        cnt = C.c_int32(0)
        st = N.Stats()
        st.hist_cap = 0
        rc = N.lib().minres_cg_solve_record(self.h, pc.h, _ptr(b), _ptr(x), rtol_out, rtol_in,
                                            maxit_out, int(maxit_inner_total), _ptr(Yt), _ptr(Zt),
                                            int(cap), C.byref(cnt), C.byref(st), _stream(stream))
        _check(rc, "minres_cg_solve_record")
        k = cnt.value
        stats = SolveStats(int(st.status), int(st.outer_its), int(st.inner_its_total),
                           float(st.final_relres), float(st.bnorm), np.zeros(0, np.int64),
                           np.zeros(0), np.zeros(0))
        return x, stats, Yt[:k].t(), Zt[:k].t()

    # -- single steps --------------------------------------------------------
    def _vec(self, v, precision, name):
        dt = torch.float64 if precision == PREC_FP64 else torch.float32
        return _dev(v, dt, name)

    def spmv(self, x, precision=PREC_FP64, out=None, stream=None):
        self._vec(x, precision, "x")
        y = out if out is not None else torch.empty_like(x)
        _check(N.lib().mcg_spmv(self.h, precision, _ptr(x), _ptr(y), _stream(stream)), "mcg_spmv")
        return y

    def mmr_apply(self, u, precision=PREC_FP64, out=None, stream=None):
        self._vec(u, precision, "u")
        q = out if out is not None else torch.empty_like(u)
        _check(N.lib().mcg_mmr_apply(self.h, precision, _ptr(u), _ptr(q), _stream(stream)),
               "mcg_mmr_apply")
        return q

    def pcg(self, y, pc: Preconditioner, rtol=1e-3, maxit=None, stream=None):
        _dev(y, torch.float64, "y")
        z = torch.empty_like(y)
        its = C.c_int64(0)
        rc = N.lib().mcg_pcg_solve(self.h, pc.h, _ptr(y), _ptr(z), rtol,
                                   int(maxit if maxit is not None else self.n), C.byref(its),
                                   _stream(stream))
        _check(rc, "mcg_pcg_solve")
        return z, int(rc), int(its.value)

    @property
    def lanes(self):
        """Lanes per CSR row used by the SpMV kernels."""
        return int(N.lib().minres_cg_spmv_lanes(self.h))

    @property
    def block_csr(self):
        """Block size of the block CSR copy of A used by the inner SpMVs (0: CSR)."""
        return int(N.lib().minres_cg_block_csr(self.h))

    @property
    def sliced_ell(self):
        """Column bits (16 or 32) of the sliced ELL copy of A used by the inner
        products, 0 when there is none."""
        return int(N.lib().minres_cg_sliced_ell(self.h))

    @property
    def sliced_blocks(self):
        """Block size of the sliced block copy of A (0: none)."""
        return int(N.lib().minres_cg_sliced_blocks(self.h))

    @property
    def xcd_sections(self):
        """Sections of the sliced block SpMV's XCD slice order (0: the
        launch's round-robin order, -1: no sliced block copy)."""
        return int(N.lib().minres_cg_xcd_sections(self.h))

    @property
    def mmr_split(self):
        """True if the Jacobi iteration's M_mr apply runs as SpMV + rank-k pass."""
        return bool(N.lib().minres_cg_mmr_split(self.h))

    def kernel_time(self, reset=False):
        """(total ms, launches) of the M_mr-apply kernel inside solves
        (requires profile=True)."""
        ms, n = C.c_double(0), C.c_int64(0)
        _check(N.lib().minres_cg_kernel_time(self.h, C.byref(ms), C.byref(n), 1 if reset else 0),
               "minres_cg_kernel_time")
        return ms.value, n.value

    def close(self):
        if self.h:
            N.lib().minres_cg_free(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lowest_eigs(row_ptr, col, val, k, block=0, degree=0, max_outer=0, tol=0.0, seed=0,
                stream=None):
    """The k smallest eigenpairs of the symmetric matrix (row_ptr, col, val)
    (int32 / int32 / float64 CUDA tensors) on the GPU: the deflation data the
    solver takes.  Returns (lam: numpy (k,), Vhat: float64 CUDA tensor (n, k)
    with orthonormal columns, stats dict)."""
    _dev(row_ptr, torch.int32, "row_ptr")
    _dev(col, torch.int32, "col")
    _dev(val, torch.float64, "val")
    n = row_ptr.numel() - 1
    A = N.CSR(n, col.numel(), row_ptr.data_ptr(), col.data_ptr(), val.data_ptr())
    opt = N.EigOptions()
    N.lib().minres_cg_eig_default_options(C.byref(opt))
    opt.block, opt.degree, opt.max_outer, opt.tol, opt.seed = block, degree, max_outer, tol, seed
    Vt = torch.empty((k, n), dtype=torch.float64, device=row_ptr.device)  # column-major n x k
    lam = np.zeros(k)
    st = N.EigStats()
    _check(N.lib().minres_cg_lowest_eigs(C.byref(A), int(k), C.byref(opt), C.c_void_p(Vt.data_ptr()),
                                         lam.ctypes.data_as(C.c_void_p), C.byref(st),
                                         _stream(stream)), "minres_cg_lowest_eigs")
    stats = {f: getattr(st, f) for f, _ in N.EigStats._fields_}
    return lam, Vt.t(), stats


def mmr_apply_noalloc(row_ptr, col, val, Vhat, lam, u, out=None, stream=None):
    """q = A u + 2 Vhat (|lam| o (Vhat^T u)) in FP64 straight from the caller's
    CUDA tensors (row_ptr, col int32; val, Vhat (n, k), lam, u float64), with
    no handle and no device allocation in the library (a fixed workspace
    array of the library is used; calls that overlap on one GPU race)."""
    _dev(row_ptr, torch.int32, "row_ptr"); _dev(col, torch.int32, "col")
    _dev(val, torch.float64, "val"); _dev(u, torch.float64, "u")
    n = row_ptr.numel() - 1
    if u.numel() != n:
        raise ValueError("u has the wrong length")
    if Vhat is not None and Vhat.numel() > 0:
        if Vhat.dim() != 2 or Vhat.shape[0] != n:
            raise ValueError("Vhat must have shape (n, k)")
        Vt = _dev(Vhat.t().contiguous(), torch.float64, "Vhat")   # column-major storage
        _dev(lam, torch.float64, "lam")
        k = Vhat.shape[1]
    else:
        Vt, lam, k = None, None, 0
    q = out if out is not None else torch.empty_like(u)
    A = N.CSR(n, col.numel(), row_ptr.data_ptr(), col.data_ptr(), val.data_ptr())
    _check(N.lib().mcg_mmr_apply_noalloc(C.byref(A), k, _ptr(Vt), _ptr(lam), _ptr(u), _ptr(q),
                                         _stream(stream)), "mcg_mmr_apply_noalloc")
    return q


def from_workload(w, precision=PREC_FP64, device="cuda", **kw):
    """MinresCG for a workloads.Workload, plus the device copy of b."""
    dev = torch.device(device)
    rp = torch.from_numpy(w.row_ptr).to(dev)
    ci = torch.from_numpy(w.col).to(dev)
    va = torch.from_numpy(w.val).to(dev)
    V = torch.from_numpy(np.ascontiguousarray(w.Vhat)).to(dev) if w.k else None
    lam = torch.from_numpy(w.lam).to(dev) if w.k else None
    kw.setdefault("block_size", int(w.meta.get("dof", 1)))
    s = MinresCG(rp, ci, va, V, lam, precision=precision, **kw)
    b = torch.from_numpy(np.ascontiguousarray(w.b)).to(dev)
    return s, b


@dataclass
class BatchStats:
    status: np.ndarray      # (nsys, nrhs)
    outer_its: np.ndarray
    inner_its: np.ndarray
    relres: np.ndarray


class BatchSystem:
    """A batch's single-system handle (not owned: the batch frees it)."""

    def __init__(self, h, n, batch):
        self.h, self.n, self._batch = h, n, batch

    preconditioner = None  # set below to MinresCG.preconditioner


class BatchedMinresCG:
    """Many independent systems with nrhs (1..8) right-hand sides each,
    solved by one persistent kernel launch (Jacobi inner preconditioner).

    systems: list of (row_ptr, col, val, Vhat, lam) CUDA tensors as for
    MinresCG (Vhat (n, k) or None)."""

    def __init__(self, systems, nrhs, precision=PREC_MIXED, stag_window=10, keep_best=True,
                 stream=None):
        self.nsys = len(systems)
        self.nrhs = nrhs
        self.ns = []
        csrs = (N.CSR * self.nsys)()
        ks = (C.c_int32 * self.nsys)()
        vps = (C.c_void_p * self.nsys)()
        lps = (C.c_void_p * self.nsys)()
        keep = []
        for i, (rp, ci, va, V, lam) in enumerate(systems):
            _dev(rp, torch.int32, "row_ptr"); _dev(ci, torch.int32, "col")
            _dev(va, torch.float64, "val")
            n = rp.numel() - 1
            self.ns.append(n)
            csrs[i] = N.CSR(n, ci.numel(), rp.data_ptr(), ci.data_ptr(), va.data_ptr())
            if V is not None and V.numel():
                Vt = _dev(V.t().contiguous(), torch.float64, "Vhat")
                _dev(lam, torch.float64, "lam")
                keep += [Vt, lam]
                ks[i] = V.shape[1]
                vps[i] = Vt.data_ptr()
                lps[i] = lam.data_ptr()
            else:
                ks[i] = 0
        opt = N.Options()
        N.lib().minres_cg_default_options(C.byref(opt))
        opt.precision = precision
        opt.stag_window = stag_window
        opt.keep_best = 1 if keep_best else 0
        self.h = C.c_void_p()
        _check(N.lib().minres_cg_batch_create(C.byref(self.h), self.nsys, csrs, ks, vps, lps,
                                              nrhs, C.byref(opt), _stream(stream)),
               "minres_cg_batch_create")

    def system(self, i):
        """System i's single-system handle (owned by the batch), on which
        second-level preconditioners of any kind are created for
        solve(..., streams=s, pcs=[...])."""
        h = C.c_void_p()
        _check(N.lib().minres_cg_batch_system(self.h, int(i), C.byref(h)), "minres_cg_batch_system")
        return BatchSystem(h, self.ns[i], self)

    def info(self):
        nb = C.c_int32(0)
        teams = (C.c_int32 * self.nsys)()
        _check(N.lib().minres_cg_batch_info(self.h, C.byref(nb), teams), "minres_cg_batch_info")
        return nb.value, list(teams)

    def profile(self):
        """Timing of the last persistent solve per system: team start and end
        (seconds on the GPU wall clock), inner iterations the team ran, the
        seconds its first workgroup spent in the inner iteration's phases
        (phase_s[:, 0..5]: SpMM + rank-k work, its reduction; z / r update,
        its reduction; direction update, its barrier), and the index of its
        k-bucket launch."""
        n = self.nsys
        t0, t1, its = (np.zeros(n, np.int64) for _ in range(3))
        ph = np.zeros((n, 6), np.int64)
        grp = np.zeros(n, np.int32)
        hz = C.c_double(0.0)
        _check(N.lib().minres_cg_batch_profile(
            self.h, t0.ctypes.data_as(C.c_void_p), t1.ctypes.data_as(C.c_void_p),
            its.ctypes.data_as(C.c_void_p), ph.ctypes.data_as(C.c_void_p),
            grp.ctypes.data_as(C.c_void_p), C.byref(hz)), "minres_cg_batch_profile")
        return {"t_begin": t0 / hz.value, "t_end": t1 / hz.value, "team_iters": its,
                "phase_s": ph / hz.value, "group": grp, "clock_hz": hz.value}

    def rebalance(self, weights):
        """Re-plan the persistent launches' teams in proportion to
        weights[i] x (nnz + (k + 1) n) -- typically each system's inner
        iteration count from an earlier solve, e.g.
        ``stats.inner_its.max(axis=1)``."""
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1))
        if w.shape[0] != self.nsys:
            raise ValueError("one weight per system")
        _check(N.lib().minres_cg_batch_rebalance(self.h, w.ctypes.data_as(C.POINTER(C.c_double))),
               "minres_cg_batch_rebalance")

    def rebalance_measured(self):
        """Re-plan the persistent launches' teams in proportion to the
        block-time (team span x team size) each system took in the last
        persistent solve."""
        _check(N.lib().minres_cg_batch_rebalance_measured(self.h),
               "minres_cg_batch_rebalance_measured")

    def solve(self, Bs, Xs=None, rtol_out=1e-8, rtol_in=1e-4, maxit_out=200, maxit_inner=10 ** 7,
              use_graph=False, streams=0, pcs=None, stream=None):
        """Bs[i]: (nrhs, n_i) float64 CUDA tensors (row j = right-hand side j).
        streams = 0: one persistent launch for the whole batch (optionally
        replayed from a HIP graph); streams = s >= 1: the systems solved one
        by one with the single-system kernels on s concurrent HIP streams.
        Returns (list of X tensors (nrhs, n_i), BatchStats, worst status)."""
        if len(Bs) != self.nsys:
            raise ValueError("one right-hand-side block per system")
        if Xs is None:
            Xs = [torch.zeros_like(b) for b in Bs]
        bp = (C.c_void_p * self.nsys)()
        xp = (C.c_void_p * self.nsys)()
        for i, (b, x) in enumerate(zip(Bs, Xs)):
            _dev(b, torch.float64, "B"); _dev(x, torch.float64, "X")
            if tuple(b.shape) != (self.nrhs, self.ns[i]) or b.shape != x.shape:
                raise ValueError("B[%d] must have shape (nrhs, n)" % i)
            bp[i] = b.data_ptr()
            xp[i] = x.data_ptr()
        m = self.nsys * self.nrhs
        st_ = np.zeros(m, np.int32); oi = np.zeros(m, np.int32)
        ii = np.zeros(m, np.int64); rr = np.zeros(m)
        st = N.BatchStats(st_.ctypes.data_as(C.POINTER(C.c_int32)),
                          oi.ctypes.data_as(C.POINTER(C.c_int32)),
                          ii.ctypes.data_as(C.POINTER(C.c_int64)),
                          rr.ctypes.data_as(C.POINTER(C.c_double)))
        if pcs is not None and not streams:
            raise ValueError("per-system preconditioners apply to the stream mode only")
        if streams:
            if use_graph:
                raise ValueError("use_graph applies to the persistent launch only")
            if pcs is not None:
                if len(pcs) != self.nsys:
                    raise ValueError("one preconditioner (or None) per system")
                pp = (C.c_void_p * self.nsys)(*[(pc.h.value if pc is not None else None)
                                                for pc in pcs])
                rc = N.lib().minres_cg_batch_solve_streams_pc(
                    self.h, pp, bp, xp, rtol_out, rtol_in, maxit_out, int(maxit_inner),
                    int(streams), C.byref(st), _stream(stream))
                _check(rc, "minres_cg_batch_solve_streams_pc")
            else:
                rc = N.lib().minres_cg_batch_solve_streams(self.h, bp, xp, rtol_out, rtol_in,
                                                           maxit_out, int(maxit_inner),
                                                           int(streams), C.byref(st),
                                                           _stream(stream))
                _check(rc, "minres_cg_batch_solve_streams")
        else:
            rc = N.lib().minres_cg_batch_solve(self.h, bp, xp, rtol_out, rtol_in, maxit_out,
                                               int(maxit_inner), 1 if use_graph else 0,
                                               C.byref(st), _stream(stream))
            _check(rc, "minres_cg_batch_solve")
        shp = (self.nsys, self.nrhs)
        return Xs, BatchStats(st_.reshape(shp), oi.reshape(shp), ii.reshape(shp),
                              rr.reshape(shp)), rc

    def close(self):
        if self.h:
            N.lib().minres_cg_batch_free(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


BatchSystem.preconditioner = MinresCG.preconditioner
