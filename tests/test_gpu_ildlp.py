"""GPU parity of the pivoted incomplete LDL^T(fill, drop) second level
(Section 4's ILDL^T with 1x1 / 2x2 Bunch-Kaufman pivots), through the C ABI,
against the oracle's own factorization, apply and solves.

The factorization decides integers (the pivot sequence, the block sizes,
which entries are kept): those must agree exactly.  Its floating point values
agree to rounding (the two implementations take the same steps in the same
order; the compilers may contract differently)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1805_12417_amd import solver as S
from paper_1805_12417_amd import workloads as W

pytestmark = pytest.mark.gpu

_CACHE = {}


def workload(name):
    if name not in _CACHE:
        _CACHE[name] = {
            "kkt32": lambda: W.kkt_saddle(m=32, n_con=16, seed=9, coupling=10.0),
            "kkt128": lambda: W.kkt_saddle(m=128, n_con=32, seed=10, coupling=10.0),
            "kkt128b": lambda: W.kkt_saddle(m=128, n_con=32, seed=10, interleave=False),
            "fe6": lambda: W.shifted_fe27(m=6, k=8),
            "lap2d": lambda: W.shifted_laplace2d(m=40, k=6),
            "edge": tile_edge_pairs,
        }[name]()
    return _CACHE[name]


def tile_edge_pairs(n=700, pairs=(255, 511, 600)):
    """Tridiagonal (4, -1) with saddle pairs [[0, 5], [5, 0]] at rows (i, i+1):
    each is a 2x2 Bunch-Kaufman pivot (no interchange) and one negative
    eigenvalue; rows 255/256 and 511/512 straddle the sweep kernels'
    256-row tiles."""
    A = np.diag(np.full(n, 4.0)) + np.diag(np.full(n - 1, -1.0), 1) + np.diag(np.full(n - 1, -1.0), -1)
    for i in pairs:
        A[i, i] = A[i + 1, i + 1] = 0.0
        A[i, i + 1] = A[i + 1, i] = 5.0
    rp = np.zeros(n + 1, np.int32)
    ci, va = [], []
    for i in range(n):
        nz = np.nonzero(A[i])[0]
        ci += list(nz)
        va += list(A[i, nz])
        rp[i + 1] = len(ci)
    w, V = np.linalg.eigh(A)
    neg = w < 0
    b = np.random.default_rng(5).standard_normal(n)
    return W.Workload("tile_edge", rp, np.asarray(ci, np.int32), np.asarray(va), b,
                      np.asfortranarray(V[:, neg]), w[neg], 0.0,
                      dict(min_abs_eig=float(np.min(np.abs(w)))))


def tiny(kind):
    """Degenerate systems: one 2x2 pivot, a diagonal matrix (L empty), 1 x 1."""
    if kind == "swap":
        A = np.array([[0.0, 1.0], [1.0, 0.0]])
    elif kind == "diag":
        A = np.diag([3.0, -2.0, 5.0, -1.0, 4.0])
    else:
        A = np.array([[-2.0]])
    n = A.shape[0]
    rp = np.zeros(n + 1, np.int32)
    ci, va = [], []
    for i in range(n):
        nz = np.nonzero(A[i])[0]
        ci += list(nz)
        va += list(A[i, nz])
        rp[i + 1] = len(ci)
    w, V = np.linalg.eigh(A)
    neg = w < 0
    return W.Workload("tiny_" + kind, rp, np.asarray(ci, np.int32), np.asarray(va), np.ones(n),
                      np.asfortranarray(V[:, neg]), w[neg], 0.0, dict(min_abs_eig=1.0))


def check_factor(w, fill, drop, precision=S.PREC_FP64):
    s, _ = S.from_workload(w, precision=precision)
    pc = s.preconditioner("ildlp", fill=fill, drop=drop)
    g = pc.ildlp_factor()
    F = O.ILDLP(w.row_ptr, w.col, w.val, fill=fill, drop=drop)
    assert np.array_equal(g["perm"], F.perm)
    assert np.array_equal(g["bsize"], F.bsize)
    assert np.array_equal(g["l_ptr"], F.l_ptr)
    assert np.array_equal(g["l_col"], F.l_col)
    scale_d = np.abs(F.dd).max()
    assert np.allclose(g["dd"], F.dd, rtol=1e-12, atol=1e-14 * scale_d)
    assert np.allclose(g["doff"], F.doff, rtol=1e-12, atol=1e-14 * scale_d)
    assert np.allclose(g["l_val"], F.l_val, rtol=1e-11, atol=1e-13 * max(1.0, np.abs(F.l_val).max(initial=0)))
    return s, pc, F


@pytest.mark.parametrize("name,fill,drop", [("kkt32", 3.0, 1e-3), ("kkt32", 1.0, 1e-2),
                                            ("kkt32", 0.0, 0.0), ("kkt128", 3.0, 1e-3),
                                            ("kkt128b", 5.0, 1e-4), ("fe6", 3.0, 1e-3),
                                            ("fe6", 1.0, 1e-1), ("lap2d", 2.0, 1e-2)])
def test_ildlp_factor_matches_oracle(name, fill, drop):
    w = workload(name)
    _, _, F = check_factor(w, fill, drop)
    if name.startswith("kkt") and name != "kkt128b":
        assert int((F.bsize == 2).sum()) == w.meta["n_con"]     # the family's 2x2 pivots


@pytest.mark.parametrize("kind", ["swap", "diag", "one"])
def test_ildlp_degenerate_sizes(kind):
    w = tiny(kind)
    s, pc, F = check_factor(w, 3.0, 1e-3)
    g = np.arange(1.0, w.n + 1)
    t = pc.apply(torch.from_numpy(g).cuda()).cpu().numpy()
    A = w.scipy().toarray()
    assert np.allclose(t, np.linalg.solve(A, g), rtol=1e-13, atol=1e-14)  # exact factor here


@pytest.mark.parametrize("name,fill,drop", [("kkt128", 3.0, 1e-3), ("kkt128", 1.0, 1e-2),
                                            ("fe6", 3.0, 1e-3), ("lap2d", 2.0, 1e-2)])
def test_ildlp_apply_matches_oracle(name, fill, drop):
    w = workload(name)
    s, pc, F = check_factor(w, fill, drop)
    rng = np.random.default_rng(5)
    for _ in range(2):
        g = rng.standard_normal(w.n)
        ref = F.solve(g)
        t = pc.apply(torch.from_numpy(g).cuda()).cpu().numpy()
        assert np.linalg.norm(t - ref) <= 1e-11 * np.linalg.norm(ref)
    # mixed precision: the same factor read in FP32
    sm, _ = S.from_workload(w, precision=S.PREC_MIXED)
    pm = sm.preconditioner("ildlp", fill=fill, drop=drop)
    g = rng.standard_normal(w.n)
    ref = F.solve(g)
    t = pm.apply(torch.from_numpy(g).float().cuda(), S.PREC_MIXED).cpu().double().numpy()
    # FP32 triangular sweeps: error grows with the factor's condition
    bound = 1e-5 * np.linalg.norm(ref) * max(1.0, np.abs(F.l_val).max(initial=0))
    assert np.linalg.norm(t - ref) <= bound


@pytest.mark.parametrize("name,precision,smw", [("kkt128", S.PREC_FP64, False),
                                                ("kkt128", S.PREC_MIXED, False),
                                                ("kkt128", S.PREC_FP64, True),
                                                ("fe6", S.PREC_FP64, False)])
def test_solve_with_ildlp_matches_oracle(name, precision, smw):
    w = workload(name)
    fill, drop = 3.0, 1e-3
    s, b = S.from_workload(w, precision=precision)
    pc = s.preconditioner("ildlp", smw=smw, fill=fill, drop=drop)
    x, st = s.solve(b, pc, rtol_out=1e-8, rtol_in=1e-3)
    P = O.Problem(w.row_ptr, w.col, w.val, w.Vhat, w.lam)
    F = O.ILDLP(w.row_ptr, w.col, w.val, fill=fill, drop=drop)
    ro = O.minres_cg(P, O.InnerPC(O.PC_ILDLP, factor=F, smw=smw), w.b, rtol_out=1e-8,
                     rtol_in=1e-3)
    print("%s prec=%d smw=%d: gpu %d/%d its, oracle %d/%d" % (
        name, precision, smw, st.outer_its, st.inner_its_total, ro["outer_its"],
        ro["inner_its_total"]), flush=True)
    assert st.status == 0 and ro["status"] == 0
    xg = x.cpu().numpy()
    rg = np.linalg.norm(w.b - O.spmv(w.row_ptr, w.col, w.val, xg)) / np.linalg.norm(w.b)
    assert rg <= 1e-8
    bound = max(1e-6 * np.linalg.norm(ro["x"]),
                (rg + ro["final_relres"]) * np.linalg.norm(w.b) / w.meta["min_abs_eig"])
    assert np.linalg.norm(xg - ro["x"]) <= bound
    if precision == S.PREC_FP64:
        assert abs(st.inner_its_total - ro["inner_its_total"]) <= 0.05 * ro["inner_its_total"] + 4


@pytest.mark.parametrize("name,sweeps", [("kkt128", 1), ("kkt128", 2), ("kkt128", 3),
                                         ("fe6", 3), ("kkt32", 64), ("edge", 1), ("edge", 2),
                                         ("edge", 3)])
def test_ildlp_sweeps_apply_matches_oracle(name, sweeps):
    w = workload(name)
    fill, drop = 3.0, 1e-3
    F = O.ILDLP(w.row_ptr, w.col, w.val, fill=fill, drop=drop)
    if name == "edge":  # 2x2 blocks across the 256-row tile edges
        assert F.bsize[255] == 2 and F.bsize[511] == 2 and F.bsize[600] == 2
        assert np.array_equal(F.perm, np.arange(w.n))
    rng = np.random.default_rng(sweeps)
    for prec, tol in ((S.PREC_FP64, 1e-12), (S.PREC_MIXED, 1e-5)):
        s, _ = S.from_workload(w, precision=prec)
        pc = s.preconditioner("ildlp", fill=fill, drop=drop, sweeps=sweeps)
        g = rng.standard_normal(w.n)
        ref = F.solve(g, sweeps=sweeps)
        gt = torch.from_numpy(g).cuda()
        gd = gt if prec == S.PREC_FP64 else gt.float()
        t = pc.apply(gd, prec).cpu().double().numpy()
        assert np.linalg.norm(t - ref) <= tol * np.linalg.norm(ref) * max(1, sweeps)
        # in place (g and t the same array) gives the same result
        gi = gd.clone()
        pc.apply(gi, prec, out=gi)
        assert np.array_equal(gi.cpu().double().numpy(), t)


@pytest.mark.parametrize("precision", [S.PREC_FP64, S.PREC_MIXED])
def test_solve_with_ildlp_sweeps_matches_oracle(precision):
    w = workload("kkt128")
    fill, drop, sw = 3.0, 1e-3, 3
    s, b = S.from_workload(w, precision=precision)
    x, st = s.solve(b, s.preconditioner("ildlp", fill=fill, drop=drop, sweeps=sw),
                    rtol_out=1e-8, rtol_in=1e-3)
    P = O.Problem(w.row_ptr, w.col, w.val, w.Vhat, w.lam)
    F = O.ILDLP(w.row_ptr, w.col, w.val, fill=fill, drop=drop)
    ro = O.minres_cg(P, O.InnerPC(O.PC_ILDLP, factor=F, sweeps=sw), w.b, rtol_out=1e-8,
                     rtol_in=1e-3)
    print("sweeps=%d prec=%d: gpu %d/%d its, oracle %d/%d" % (
        sw, precision, st.outer_its, st.inner_its_total, ro["outer_its"],
        ro["inner_its_total"]), flush=True)
    assert st.status == 0 and ro["status"] == 0
    xg = x.cpu().numpy()
    rg = np.linalg.norm(w.b - O.spmv(w.row_ptr, w.col, w.val, xg)) / np.linalg.norm(w.b)
    assert rg <= 1e-8
    bound = max(1e-6 * np.linalg.norm(ro["x"]),
                (rg + ro["final_relres"]) * np.linalg.norm(w.b) / w.meta["min_abs_eig"])
    assert np.linalg.norm(xg - ro["x"]) <= bound
    if precision == S.PREC_FP64:
        assert abs(st.inner_its_total - ro["inner_its_total"]) <= 0.05 * ro["inner_its_total"] + 4


def test_ildlp_beats_no_preconditioner_on_the_saddle_family():
    """On [[K, B^T], [B, 0]] neither Jacobi (zero diagonal) nor the unpivoted
    ILDL^T(0) has a pivot in the constraint rows; the pivoted factor does, and
    cuts the inner iterations against M_cg = I."""
    w = workload("kkt128")
    s, b = S.from_workload(w)
    with pytest.raises(S.MCGError):
        s.preconditioner("jacobi")
    _, st_p = s.solve(b, s.preconditioner("ildlp"), rtol_out=1e-8, rtol_in=1e-3)
    _, st_n = s.solve(b, s.preconditioner("none"), rtol_out=1e-8, rtol_in=1e-3)
    print("inner its: ildlp %d, none %d" % (st_p.inner_its_total, st_n.inner_its_total),
          flush=True)
    assert st_p.status == 0 and st_n.status == 0
    assert st_p.inner_its_total * 3 < st_n.inner_its_total


def test_ildlp_rejects_bad_parameters():
    w = workload("kkt32")
    s, _ = S.from_workload(w)
    for fill, drop, sw in ((-1.0, 1e-3, 0), (3.0, -1e-3, 0), (float("nan"), 1e-3, 0),
                           (3.0, float("inf"), 0), (3.0, 1e-3, -1), (3.0, 1e-3, 65)):
        with pytest.raises(S.MCGError) as e:
            s.preconditioner("ildlp", fill=fill, drop=drop, sweeps=sw)
        assert e.value.code == S.N.EINVAL
    pj = s.preconditioner("none")
    with pytest.raises(S.MCGError):
        pj.ildlp_factor()
