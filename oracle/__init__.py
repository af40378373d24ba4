"""Oracle for MINRES-CG: plain, slow, obviously-correct FP64 CPU reference.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this
module; only the tests, the smoke check and the benchmark's CPU-baseline leg
use it.  It shares no code with the HIP library.

  * mcg_oracle.c (loaded through ctypes): SpMV, the M_mr apply, incomplete
    LDL^T(0), the inner PCG and the outer preconditioned MINRES, following
    Section 2 and Algorithm "minres_cg" step by step.
  * dense.py (numpy): tiny dense constructions of Section 1 used as pins
    (Bunch-Parlett LDL^T with the 2x2 "absolute value", |A|, the
    Sherman-Morrison-Woodbury inverse of Section 2.1).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mcg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, MAXIT, STAGNATION, BREAKDOWN, NOT_SPD, EINVAL = 0, 1, 2, 3, 4, -1
PC_NONE, PC_JACOBI, PC_ILDL0, PC_DENSE, PC_CCT, PC_ILDLP = 0, 1, 2, 3, 4, 5
OUT_PCG, OUT_DENSE, OUT_NONE = 0, 1, 2


def build() -> str:
    """Compile the oracle (plain gcc, -O2, OpenMP)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None

_d = C.POINTER(C.c_double)
_i32 = C.POINTER(C.c_int32)
_i64 = C.POINTER(C.c_int64)


class _Problem(C.Structure):
    _fields_ = [("n", C.c_int32), ("row_ptr", _i32), ("col", _i32), ("val", _d),
                ("k", C.c_int32), ("Vhat", _d), ("lam", _d)]


class _ILDLP(C.Structure):
    _fields_ = [("n", C.c_int32), ("perm", _i32), ("bsize", _i32), ("dd", _d), ("doff", _d),
                ("l_ptr", _i32), ("l_col", _i32), ("l_val", _d), ("nnz_l", C.c_int64)]


class _InnerPC(C.Structure):
    _fields_ = [("kind", C.c_int32), ("diag", _d), ("l_ptr", _i32), ("l_col", _i32),
                ("l_val", _d), ("d", _d), ("dense", _d), ("c_ptr", _i32), ("c_col", _i32),
                ("c_val", _d), ("smw", C.c_int32), ("ildlp", C.POINTER(_ILDLP)),
                ("ildlp_sweeps", C.c_int32)]


class _Opts(C.Structure):
    _fields_ = [("outer_kind", C.c_int32), ("dense", _d), ("rtol_out", C.c_double),
                ("rtol_in", C.c_double), ("maxit_out", C.c_int32), ("maxit_in", C.c_int64),
                ("maxit_in_total", C.c_int64), ("stag_window", C.c_int32),
                ("keep_best", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [("status", C.c_int32), ("outer_its", C.c_int32), ("inner_its_total", C.c_int64),
                ("final_relres", C.c_double), ("hist_cap", C.c_int32), ("inner_its", _i64),
                ("relres", _d), ("phibar", _d)]


def load(path: str):
    """Load and type a compiled oracle library (the default one, or a copy
    built elsewhere, e.g. by the mutation tests)."""
    L = C.CDLL(path)
    L.orc_spmv.argtypes = [C.c_int32, _i32, _i32, _d, _d, _d]
    L.orc_mmr_apply.argtypes = [C.c_int32, _i32, _i32, _d, C.c_int32, _d, _d, _d, _d]
    L.orc_ildl0_nnz_lower.argtypes = [C.c_int32, _i32, _i32]
    L.orc_ildl0_nnz_lower.restype = C.c_int64
    L.orc_ildl0_factor.argtypes = [C.c_int32, _i32, _i32, _d, C.c_double, _i32, _i32, _d, _d]
    L.orc_ildl0_factor.restype = C.c_int32
    L.orc_ildl0_solve.argtypes = [C.c_int32, _i32, _i32, _d, _d, _d, _d]
    L.orc_precond_apply.argtypes = [C.POINTER(_Problem), C.POINTER(_InnerPC), _d, _d]
    L.orc_ildlp_factor.argtypes = [C.c_int32, _i32, _i32, _d, C.c_double, C.c_double]
    L.orc_ildlp_factor.restype = C.POINTER(_ILDLP)
    L.orc_ildlp_free.argtypes = [C.POINTER(_ILDLP)]
    L.orc_ildlp_free.restype = None
    L.orc_ildlp_solve.argtypes = [C.POINTER(_ILDLP), _d, _d]
    L.orc_ildlp_solve_sweeps.argtypes = [C.POINTER(_ILDLP), C.c_int32, _d, _d]
    L.orc_ildlp_solve_sweeps.restype = None
    L.orc_pcg.argtypes = [C.POINTER(_Problem), C.POINTER(_InnerPC), _d, _d, C.c_double,
                          C.c_int64, _i64, _d]
    L.orc_pcg.restype = C.c_int32
    L.orc_minres_cg.argtypes = [C.POINTER(_Problem), C.POINTER(_InnerPC), C.POINTER(_Opts),
                                _d, _d, C.POINTER(_Stats)]
    L.orc_minres_cg.restype = C.c_int32
    L.orc_num_threads.restype = C.c_int32
    L.orc_set_num_threads.argtypes = [C.c_int32]
    L.orc_set_num_threads.restype = None
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = load(_LIB)
    return _lib


class use_library:
    """Context manager: route every oracle call through another build."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = _lib
        _lib = load(self.path)
        return _lib

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def _p(a, ct):
    return a.ctypes.data_as(ct) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32a(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(t: int) -> None:
    """OpenMP threads of later oracle calls (for timing; results do not
    depend on it)."""
    lib().orc_set_num_threads(int(t))


# ---------------------------------------------------------------------------
# building blocks
# ---------------------------------------------------------------------------

def spmv(row_ptr, col, val, x):
    """y = A x (CSR, FP64)."""
    row_ptr, col, val, x = _i32a(row_ptr), _i32a(col), _f64(val), _f64(x)
    n = row_ptr.size - 1
    y = np.empty(n)
    lib().orc_spmv(n, _p(row_ptr, _i32), _p(col, _i32), _p(val, _d), _p(x, _d), _p(y, _d))
    return y


def mmr_apply(row_ptr, col, val, Vhat, lam, u):
    """q = A u + 2 Vhat (|lam| * (Vhat^T u)) (Section 2)."""
    row_ptr, col, val, u = _i32a(row_ptr), _i32a(col), _f64(val), _f64(u)
    V = np.asfortranarray(Vhat, dtype=np.float64)
    lam = _f64(lam)
    n = row_ptr.size - 1
    q = np.empty(n)
    lib().orc_mmr_apply(n, _p(row_ptr, _i32), _p(col, _i32), _p(val, _d), lam.size,
                        V.ctypes.data_as(_d), _p(lam, _d), _p(u, _d), _p(q, _d))
    return q


def ildl0_factor(row_ptr, col, val, pivtol=1e-8):
    """Incomplete LDL^T(0) of A: returns (l_ptr, l_col, l_val, d, n_modified_pivots)."""
    row_ptr, col, val = _i32a(row_ptr), _i32a(col), _f64(val)
    n = row_ptr.size - 1
    L = lib()
    nl = L.orc_ildl0_nnz_lower(n, _p(row_ptr, _i32), _p(col, _i32))
    lp = np.empty(n + 1, np.int32); lc = np.empty(nl, np.int32)
    lv = np.empty(nl); d = np.empty(n)
    mod = L.orc_ildl0_factor(n, _p(row_ptr, _i32), _p(col, _i32), _p(val, _d), pivtol,
                             _p(lp, _i32), _p(lc, _i32), _p(lv, _d), _p(d, _d))
    if mod < 0:
        raise ValueError("ildl0: missing diagonal entry")
    return lp, lc, lv, d, int(mod)


def ildl0_solve(factor, g):
    lp, lc, lv, d = factor[:4]
    g = _f64(g)
    t = np.empty_like(g)
    lib().orc_ildl0_solve(g.size, _p(lp, _i32), _p(lc, _i32), _p(lv, _d), _p(d, _d),
                          _p(g, _d), _p(t, _d))
    return t


class ILDLP:
    """Incomplete LDL^T with 1x1 / 2x2 symmetric pivoting, fill factor and drop
    tolerance (mcg_oracle.c, orc_ildlp_factor): P A P^T ~ L D L^T.  Arrays
    (copies): perm (logical -> original), bsize, dd, doff, L (logical CSR,
    strictly lower)."""

    def __init__(self, row_ptr, col, val, fill=3.0, drop=1e-3):
        rp, ci, va = _i32a(row_ptr), _i32a(col), _f64(val)
        self.n = rp.size - 1
        self._lib = lib()
        ptr = self._lib.orc_ildlp_factor(self.n, _p(rp, _i32), _p(ci, _i32), _p(va, _d),
                                         float(fill), float(drop))
        if not ptr:
            raise MemoryError("orc_ildlp_factor failed")
        self.ptr = ptr
        F = ptr.contents
        n, nnz = self.n, int(F.nnz_l)
        self.perm = np.ctypeslib.as_array(F.perm, (n,)).copy()
        self.bsize = np.ctypeslib.as_array(F.bsize, (n,)).copy()
        self.dd = np.ctypeslib.as_array(F.dd, (n,)).copy()
        self.doff = np.ctypeslib.as_array(F.doff, (n,)).copy()
        self.l_ptr = np.ctypeslib.as_array(F.l_ptr, (n + 1,)).copy()
        self.l_col = np.ctypeslib.as_array(F.l_col, (max(nnz, 1),))[:nnz].copy()
        self.l_val = np.ctypeslib.as_array(F.l_val, (max(nnz, 1),))[:nnz].copy()

    def D(self):
        """Block diagonal D as a dense matrix (small n only)."""
        Dm = np.diag(self.dd)
        for k in np.nonzero(self.bsize == 2)[0]:
            Dm[k, k + 1] = Dm[k + 1, k] = self.doff[k]
        return Dm

    def L(self):
        """Unit lower triangular L as a dense matrix (small n only)."""
        import scipy.sparse as sp
        return sp.csr_matrix((self.l_val, self.l_col, self.l_ptr),
                             shape=(self.n, self.n)).toarray() + np.eye(self.n)

    def solve(self, g, sweeps=0):
        """P^T L^{-T} D^{-1} L^{-1} P g; sweeps > 0: each triangular solve
        replaced by that many Jacobi sweeps (orc_ildlp_solve_sweeps)."""
        g = _f64(g)
        t = np.empty_like(g)
        if sweeps > 0:
            self._lib.orc_ildlp_solve_sweeps(self.ptr, int(sweeps), _p(g, _d), _p(t, _d))
        else:
            self._lib.orc_ildlp_solve(self.ptr, _p(g, _d), _p(t, _d))
        return t

    def __del__(self):
        try:
            if getattr(self, "ptr", None):
                self._lib.orc_ildlp_free(self.ptr)
                self.ptr = None
        except Exception:
            pass


# ---------------------------------------------------------------------------
# solvers
# ---------------------------------------------------------------------------

class Problem:
    """Holds the arrays alive for the C structs."""

    def __init__(self, row_ptr, col, val, Vhat=None, lam=None):
        self.row_ptr, self.col, self.val = _i32a(row_ptr), _i32a(col), _f64(val)
        self.n = self.row_ptr.size - 1
        if Vhat is None or lam is None or np.size(lam) == 0:
            self.V = np.zeros((self.n, 0), order="F"); self.lam = np.zeros(0)
        else:
            self.V = np.asfortranarray(Vhat, dtype=np.float64); self.lam = _f64(lam)
        self.c = _Problem(self.n, _p(self.row_ptr, _i32), _p(self.col, _i32), _p(self.val, _d),
                          self.lam.size, self.V.ctypes.data_as(_d) if self.lam.size else None,
                          _p(self.lam, _d) if self.lam.size else None)

    def diag(self):
        out = np.zeros(self.n)
        for i in range(self.n):
            s, e = self.row_ptr[i], self.row_ptr[i + 1]
            hit = np.nonzero(self.col[s:e] == i)[0]
            if hit.size:
                out[i] = self.val[s + hit[0]]
        return out


class InnerPC:
    """Inner (CG) preconditioner M_cg description.

    kind: PC_NONE | PC_JACOBI (diag) | PC_ILDL0 (factor tuple) |
          PC_DENSE (dense Minv) | PC_CCT (C as (ptr, col, val)) |
          PC_ILDLP (an ILDLP factor; sweeps > 0: Jacobi sweeps instead of
          the triangular solves); smw=True
          adds -2 Vhat Lambda^{-1} Vhat^T (MINRES-CG*, Section 2.1)."""

    def __init__(self, kind, problem: Problem | None = None, diag=None, factor=None,
                 dense=None, C_csr=None, smw=False, sweeps=0):
        self.kind = kind
        self.keep = []
        c = _InnerPC()
        c.kind = kind
        c.smw = 1 if smw else 0
        if kind == PC_JACOBI:
            dg = _f64(diag if diag is not None else problem.diag())
            if np.any(dg == 0):
                raise ValueError("Jacobi: zero diagonal")
            self.keep.append(dg); c.diag = _p(dg, _d)
        elif kind == PC_ILDL0:
            f = factor if factor is not None else ildl0_factor(problem.row_ptr, problem.col, problem.val)
            self.keep.append(f)
            c.l_ptr, c.l_col, c.l_val, c.d = _p(f[0], _i32), _p(f[1], _i32), _p(f[2], _d), _p(f[3], _d)
        elif kind == PC_DENSE:
            M = np.ascontiguousarray(dense, dtype=np.float64)
            self.keep.append(M); c.dense = _p(M, _d)
        elif kind == PC_ILDLP:
            f = factor if factor is not None else ILDLP(problem.row_ptr, problem.col, problem.val)
            self.keep.append(f)
            c.ildlp = f.ptr
            c.ildlp_sweeps = int(sweeps)
        elif kind == PC_CCT:
            cp, cc, cv = _i32a(C_csr[0]), _i32a(C_csr[1]), _f64(C_csr[2])
            self.keep += [cp, cc, cv]
            c.c_ptr, c.c_col, c.c_val = _p(cp, _i32), _p(cc, _i32), _p(cv, _d)
        self.c = c


def precond_apply(problem: Problem, pc: InnerPC, g):
    """t = M_cg^{-1} g, the second-level apply on its own."""
    g = _f64(g)
    t = np.empty_like(g)
    lib().orc_precond_apply(C.byref(problem.c), C.byref(pc.c), _p(g, _d), _p(t, _d))
    return t


def pcg(problem: Problem, pc: InnerPC, y, rtol, maxit=None):
    """Inner PCG on M_mr z = y from z0 = 0. Returns (z, status, its, relres)."""
    y = _f64(y)
    z = np.empty_like(y)
    its = C.c_int64(0); rr = C.c_double(0)
    st = lib().orc_pcg(C.byref(problem.c), C.byref(pc.c), _p(y, _d), _p(z, _d), rtol,
                       int(maxit if maxit is not None else problem.n), C.byref(its), C.byref(rr))
    return z, int(st), int(its.value), float(rr.value)


def minres_cg(problem: Problem, pc: InnerPC | None, b, x0=None, rtol_out=1e-8, rtol_in=1e-3,
              maxit_out=200, maxit_in=None, maxit_in_total=10 ** 7, stag_window=10,
              outer_kind=OUT_PCG, outer_dense=None, keep_best=True):
    """Outer preconditioned MINRES with the inner PCG preconditioner.
    Returns dict(x, status, outer_its, inner_its_total, inner_its, relres,
    phibar, final_relres)."""
    b = _f64(b)
    x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
    cap = maxit_out + 2
    inner = np.zeros(cap, np.int64); rel = np.full(cap, np.nan); phb = np.full(cap, np.nan)
    st = _Stats(0, 0, 0, 0.0, cap, _p(inner, _i64), _p(rel, _d), _p(phb, _d))
    o = _Opts()
    o.outer_kind = outer_kind
    dense = None
    if outer_kind == OUT_DENSE:
        dense = np.ascontiguousarray(outer_dense, dtype=np.float64)
        o.dense = _p(dense, _d)
    o.rtol_out, o.rtol_in = rtol_out, rtol_in
    o.maxit_out = maxit_out
    o.maxit_in = int(maxit_in if maxit_in is not None else problem.n)
    o.maxit_in_total = int(maxit_in_total)
    o.stag_window = stag_window
    o.keep_best = 1 if keep_best else 0
    if pc is None:
        pc = InnerPC(PC_NONE)
    status = lib().orc_minres_cg(C.byref(problem.c), C.byref(pc.c), C.byref(o), _p(b, _d),
                                 _p(x, _d), C.byref(st))
    k = st.outer_its
    return dict(x=x, status=int(status), outer_its=int(k), inner_its_total=int(st.inner_its_total),
                inner_its=inner[:k + 1].copy(), relres=rel[:k + 1].copy(), phibar=phb[:k + 1].copy(),
                final_relres=float(st.final_relres))
