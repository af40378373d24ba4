"""GPU parity: every step of the hot path, called through the C ABI, against
the FP64 CPU oracle on the same seeded inputs.

Sizes span several 256-row tiles and include ragged tails.  Tolerances:
  * SpMV / M_mr apply / Jacobi (FP64): |gpu - oracle| <= 8 eps (|A||x|)_i per row
    (both sum the same products in different orders);
  * FP32 steps: the oracle is run on the FP32-rounded inputs and the bound
    uses FP32 epsilon times the row length;
  * whole solves: both true relative residuals (recomputed by the oracle's
    FP64 SpMV) <= rtol, and ||x_gpu - x_oracle|| <= max(1e-6 ||x_oracle||,
    (||r_gpu|| + ||r_oracle||) / min|lambda(A)|), the second term being the
    bound any two solutions with these residuals obey.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1805_12417_amd import solver as S
from paper_1805_12417_amd import workloads as W

pytestmark = pytest.mark.gpu

EPS64 = np.finfo(np.float64).eps
EPS32 = np.finfo(np.float32).eps


def cfg(name):
    if name == "cfg1":
        return W.shifted_laplace2d()
    if name == "cfg2s":      # 3D random-coefficient Laplacian, ragged tail (9177 rows)
        return W.shifted_laplace3d(dims=(23, 21, 19), k=20)
    if name == "cfg3s":      # FE-like 27-point, 3 dof (3*7^3 = 1029 rows)
        return W.shifted_fe27(m=7, k=10)
    if name == "cfg3m":      # 20^3 nodes: 125 slices of 64 block rows
        return W.shifted_fe27(m=20, k=6)
    raise KeyError(name)


_CACHE = {}


def workload(name):
    if name not in _CACHE:
        _CACHE[name] = cfg(name)
    return _CACHE[name]


def gpu_solver(w, precision=S.PREC_FP64, **kw):
    return S.from_workload(w, precision=precision, **kw)


def absAx(w, x):
    return O.spmv(w.row_ptr, w.col, np.abs(w.val), np.abs(x))


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


@pytest.mark.parametrize("name", ["cfg1", "cfg2s", "cfg3s", "cfg3m"])
def test_spmv_fp64(name):
    w = workload(name)
    # cfg3m: x fits in one XCD's L2, so the automatic choice keeps the
    # launch's order; xcd_order = 2 forces the section order the line model
    # picks: 8 colour sections of 15-16 slices, split unevenly over the XCDs
    s, _ = gpu_solver(w, xcd_order=2) if name == "cfg3m" else gpu_solver(w)
    if name == "cfg3m":
        assert s.sliced_blocks == 3 and s.xcd_sections == 8
        assert gpu_solver(w)[0].xcd_sections == 0
    x = np.random.default_rng(1).standard_normal(w.n)
    y = s.spmv(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = O.spmv(w.row_ptr, w.col, w.val, x)
    assert np.all(np.abs(y - ref) <= 8 * EPS64 * absAx(w, x) + 1e-300)


@pytest.mark.parametrize("name", ["cfg2s", "cfg3s", "cfg3m"])
def test_spmv_fp32(name):
    w = workload(name)
    s, _ = gpu_solver(w, S.PREC_MIXED, **({"xcd_order": 2} if name == "cfg3m" else {}))
    if name == "cfg3m":
        assert s.xcd_sections == 8
        assert gpu_solver(w, S.PREC_MIXED, xcd_order=1)[0].xcd_sections == 0
    x = np.random.default_rng(2).standard_normal(w.n)
    y = s.spmv(torch.from_numpy(x).float().cuda(), S.PREC_MIXED).cpu().numpy().astype(np.float64)
    ref = O.spmv(w.row_ptr, w.col, f32(w.val), f32(x))
    rowlen = np.diff(w.row_ptr)
    bound = 2 * rowlen * EPS32 * O.spmv(w.row_ptr, w.col, np.abs(f32(w.val)), np.abs(f32(x)))
    assert np.all(np.abs(y - ref) <= bound)


@pytest.mark.parametrize("name", ["cfg1", "cfg2s", "cfg3s"])
def test_mmr_apply_fp64(name):
    w = workload(name)
    s, _ = gpu_solver(w)
    u = np.random.default_rng(3).standard_normal(w.n)
    q = s.mmr_apply(torch.from_numpy(u).cuda()).cpu().numpy()
    ref = O.mmr_apply(w.row_ptr, w.col, w.val, w.Vhat, w.lam, u)
    scale = absAx(w, u) + 2 * np.abs(w.Vhat) @ (np.abs(w.lam) * np.abs(w.Vhat.T @ u)) \
        + np.abs(w.Vhat) @ (np.abs(w.lam) * (np.abs(w.Vhat).T @ np.abs(u)))
    assert np.all(np.abs(q - ref) <= 64 * EPS64 * scale)


def test_mmr_apply_fp32():
    w = workload("cfg2s")
    s, _ = gpu_solver(w, S.PREC_MIXED)
    u = np.random.default_rng(4).standard_normal(w.n)
    q = s.mmr_apply(torch.from_numpy(u).float().cuda(), S.PREC_MIXED).cpu().numpy()
    ref = O.mmr_apply(w.row_ptr, w.col, f32(w.val), f32(w.Vhat), w.lam, f32(u))
    scale = absAx(w, u) + 2 * np.abs(w.Vhat) @ (np.abs(w.lam) * (np.abs(w.Vhat).T @ np.abs(u)))
    assert np.linalg.norm(q - ref) <= 64 * EPS32 * np.linalg.norm(scale)
    assert np.all(np.abs(q - ref) <= 4096 * EPS32 * scale)


def test_jacobi_apply_and_identity():
    w = workload("cfg2s")
    s, _ = gpu_solver(w)
    g = np.random.default_rng(5).standard_normal(w.n)
    t = s.preconditioner("jacobi").apply(torch.from_numpy(g).cuda()).cpu().numpy()
    assert np.allclose(t, g / O.Problem(w.row_ptr, w.col, w.val).diag(), rtol=2 * EPS64, atol=0)
    t0 = s.preconditioner("none").apply(torch.from_numpy(g).cuda()).cpu().numpy()
    assert np.array_equal(t0, g)


def test_smw_preconditioner_apply():
    """MINRES-CG* second-level preconditioner: diag(A)^{-1} - 2 V Lambda^{-1} V^T."""
    w = workload("cfg2s")
    s, _ = gpu_solver(w)
    g = np.random.default_rng(6).standard_normal(w.n)
    t = s.preconditioner("jacobi", smw=True).apply(torch.from_numpy(g).cuda()).cpu().numpy()
    d = O.Problem(w.row_ptr, w.col, w.val).diag()
    ref = g / d - 2.0 * w.Vhat @ ((w.Vhat.T @ g) / w.lam)
    assert np.allclose(t, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("name,precision", [("cfg1", S.PREC_FP64), ("cfg2s", S.PREC_FP64),
                                            ("cfg2s", S.PREC_MIXED), ("cfg3s", S.PREC_FP64)])
def test_inner_pcg_matches_oracle(name, precision):
    w = workload(name)
    s, _ = gpu_solver(w, precision)
    pc = s.preconditioner("jacobi")
    P = O.Problem(w.row_ptr, w.col, w.val, w.Vhat, w.lam)
    y = np.random.default_rng(7).standard_normal(w.n)
    rtol = 1e-10 if precision == S.PREC_FP64 else 1e-4
    z, st, its = s.pcg(torch.from_numpy(y).cuda(), pc, rtol=rtol)
    z = z.cpu().numpy()
    zo, sto, itso, _ = O.pcg(P, O.InnerPC(O.PC_JACOBI, P), y, rtol)
    assert st == 0 and sto == 0
    res = np.linalg.norm(y - O.mmr_apply(w.row_ptr, w.col, w.val, w.Vhat, w.lam, z))
    if precision == S.PREC_FP64:
        assert abs(its - itso) <= 2
        assert res <= 1.01 * rtol * np.linalg.norm(y)
    else:
        # the FP32 recurrence residual meets rtol; the FP64 one may sit above it
        assert abs(its - itso) <= max(3, itso // 10)
        assert res <= 10 * rtol * np.linalg.norm(y)


def _true_relres(w, x, b=None):
    b = w.b if b is None else b
    return np.linalg.norm(b - O.spmv(w.row_ptr, w.col, w.val, x)) / np.linalg.norm(b)


def _check_solution(w, xg, xo, rtol, b=None):
    rg, ro = _true_relres(w, xg, b), _true_relres(w, xo, b)
    assert rg <= rtol and ro <= rtol
    bn = np.linalg.norm(w.b if b is None else b)
    bound = max(1e-6 * np.linalg.norm(xo), (rg + ro) * bn / w.meta["min_abs_eig"])
    assert np.linalg.norm(xg - xo) <= bound


@pytest.mark.parametrize("name,precision,rtol,rtol_in", [
    ("cfg1", S.PREC_FP64, 1e-10, 1e-4),
    ("cfg1", S.PREC_MIXED, 1e-10, 1e-4),
    ("cfg2s", S.PREC_FP64, 1e-8, 1e-3),
    ("cfg2s", S.PREC_MIXED, 1e-8, 1e-3),
    ("cfg3s", S.PREC_FP64, 1e-8, 1e-3),
])
def test_minres_cg_solve_matches_oracle(name, precision, rtol, rtol_in):
    w = workload(name)
    s, b = gpu_solver(w, precision)
    pc = s.preconditioner("jacobi")
    x, st = s.solve(b, pc, rtol_out=rtol, rtol_in=rtol_in)
    xg = x.cpu().numpy()
    P = O.Problem(w.row_ptr, w.col, w.val, w.Vhat, w.lam)
    ro = O.minres_cg(P, O.InnerPC(O.PC_JACOBI, P), w.b, rtol_out=rtol, rtol_in=rtol_in)
    assert st.status == 0 and ro["status"] == 0
    _check_solution(w, xg, ro["x"], rtol)
    assert abs(st.final_relres - _true_relres(w, xg)) <= 1e-3 * st.final_relres + 1e-15
    if precision == S.PREC_FP64:
        assert abs(st.outer_its - ro["outer_its"]) <= 1
    assert np.all(np.diff(st.phibar[~np.isnan(st.phibar)]) <= 1e-12 * st.phibar[0])


def test_minres_cg_star_solve():
    w = workload("cfg2s")
    s, b = gpu_solver(w)
    x, st = s.solve(b, s.preconditioner("jacobi", smw=True), rtol_out=1e-8, rtol_in=1e-3)
    P = O.Problem(w.row_ptr, w.col, w.val, w.Vhat, w.lam)
    ro = O.minres_cg(P, O.InnerPC(O.PC_JACOBI, P, smw=True), w.b, rtol_out=1e-8, rtol_in=1e-3)
    assert st.status == 0 and ro["status"] == 0
    _check_solution(w, x.cpu().numpy(), ro["x"], 1e-8)
    assert abs(st.inner_its_total - ro["inner_its_total"]) <= 0.1 * ro["inner_its_total"] + 4


@pytest.mark.parametrize("precision", [S.PREC_FP64, S.PREC_MIXED])
def test_multi_rhs_solve_equals_single_solves(precision):
    """nrhs right-hand sides in one minres_cg_solve call: each column is the
    single-column solve, bitwise (same handle, same kernels), every column
    against its own oracle solve; nrhs = 0 is rejected."""
    w = workload("cfg2s")
    s, b = gpu_solver(w, precision)
    pc = s.preconditioner("jacobi")
    rng = np.random.default_rng(31)
    Bh = np.stack([w.b, rng.standard_normal(w.n), np.zeros(w.n)])
    Bd = torch.from_numpy(Bh).cuda()
    X, sts = s.solve(Bd, pc, rtol_out=1e-8, rtol_in=1e-3)
    assert len(sts) == 3 and X.shape == Bd.shape
    P = O.Problem(w.row_ptr, w.col, w.val, w.Vhat, w.lam)
    for j in range(3):
        x1, st1 = s.solve(Bd[j].contiguous(), pc, rtol_out=1e-8, rtol_in=1e-3)
        assert torch.equal(X[j], x1)
        assert sts[j].status == st1.status == 0
        assert sts[j].inner_its_total == st1.inner_its_total
        if j < 2:
            ro = O.minres_cg(P, O.InnerPC(O.PC_JACOBI, P), Bh[j], rtol_out=1e-8, rtol_in=1e-3)
            _check_solution(w, X[j].cpu().numpy(), ro["x"], 1e-8, b=Bh[j])
    assert torch.count_nonzero(X[2]) == 0
    L = S.N.lib()
    assert L.minres_cg_solve(s.h, pc.h, Bd.data_ptr(), X.data_ptr(), 0, 1e-8, 1e-3, 10, 100,
                             None, None) == S.N.EINVAL


def test_deterministic_bitwise():
    w = workload("cfg2s")
    s, b = gpu_solver(w, S.PREC_MIXED)
    pc = s.preconditioner("jacobi")
    x1, st1 = s.solve(b, pc, rtol_out=1e-8)
    x2, st2 = s.solve(b, pc, rtol_out=1e-8)
    assert torch.equal(x1, x2) and st1.inner_its_total == st2.inner_its_total


def test_zero_rhs_and_exact_initial_guess():
    w = workload("cfg2s")
    s, b = gpu_solver(w)
    pc = s.preconditioner("jacobi")
    x, st = s.solve(torch.zeros_like(b), pc, x0=torch.ones_like(b))
    assert st.status == 0 and torch.count_nonzero(x) == 0
    xo = O.minres_cg(O.Problem(w.row_ptr, w.col, w.val, w.Vhat, w.lam),
                     O.InnerPC(O.PC_JACOBI, O.Problem(w.row_ptr, w.col, w.val)), w.b,
                     rtol_out=1e-12)["x"]
    x, st = s.solve(b, pc, x0=torch.from_numpy(xo).cuda(), rtol_out=1e-8)
    assert st.status == 0 and st.outer_its == 0


def test_spd_without_deflation_k0():
    """k = 0: M_mr = A (SPD), the method is MINRES preconditioned by CG."""
    rng = np.random.default_rng(9)
    import scipy.sparse as sp
    A = W.laplace3d_random(13, 11, 7, rng)
    A.sort_indices()
    wk = W.Workload("spd", A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.copy(),
                    rng.standard_normal(A.shape[0]), np.zeros((A.shape[0], 0), order="F"),
                    np.zeros(0), 0.0, {"min_abs_eig": float(np.linalg.eigvalsh(A.toarray()).min())})
    s, b = gpu_solver(wk)
    x, st = s.solve(b, s.preconditioner("jacobi"), rtol_out=1e-10)
    assert st.status == 0
    xs = np.linalg.solve(A.toarray(), wk.b)
    assert np.linalg.norm(x.cpu().numpy() - xs) <= 1e-6 * np.linalg.norm(xs)


def test_status_maxit_and_not_spd():
    w = workload("cfg2s")
    s, b = gpu_solver(w)
    x, st = s.solve(b, s.preconditioner("jacobi"), rtol_out=1e-12, maxit_out=1)
    assert st.status == 1 and st.outer_its == 1
    x, st = s.solve(b, s.preconditioner("jacobi"), rtol_out=1e-12, maxit_inner_total=50)
    assert st.status == 1
    # drop one negative eigenvector: M_mr indefinite
    s2 = S.MinresCG(torch.from_numpy(w.row_ptr).cuda(), torch.from_numpy(w.col).cuda(),
                    torch.from_numpy(w.val).cuda(), torch.from_numpy(np.ascontiguousarray(w.Vhat[:, 1:])).cuda(),
                    torch.from_numpy(w.lam[1:]).cuda())
    x, st = s2.solve(b, s2.preconditioner("jacobi"), rtol_out=1e-10, rtol_in=1e-10)
    P = O.Problem(w.row_ptr, w.col, w.val, w.Vhat[:, 1:], w.lam[1:])
    ro = O.minres_cg(P, O.InnerPC(O.PC_JACOBI, P), w.b, rtol_out=1e-10, rtol_in=1e-10)
    assert st.status == 4 and ro["status"] == 4


def test_invalid_inputs_are_rejected():
    w = workload("cfg1")
    dev = torch.device("cuda")
    rp = torch.from_numpy(w.row_ptr).to(dev); va = torch.from_numpy(w.val).to(dev)
    bad_col = w.col.copy(); bad_col[[1, 2]] = bad_col[[2, 1]]       # unsorted row
    with pytest.raises(S.MCGError):
        S.MinresCG(rp, torch.from_numpy(bad_col).to(dev), va)
    with pytest.raises(S.MCGError):                                  # lam >= 0
        S.MinresCG(rp, torch.from_numpy(w.col).to(dev), va,
                   torch.from_numpy(np.ascontiguousarray(w.Vhat)).to(dev),
                   torch.from_numpy(-w.lam).to(dev))
    for opt in ({"xcd_order": 3}, {"xcd_order": -1}, {"mmr_form": 3}):   # option out of range
        with pytest.raises(S.MCGError):
            gpu_solver(w, **opt)
    s, b = gpu_solver(w)
    bn = b.clone(); bn[5] = float("nan")
    with pytest.raises(S.MCGError):
        s.solve(bn, s.preconditioner("jacobi"))


def test_autotuned_lanes_give_the_same_products(tmp_path, monkeypatch):
    monkeypatch.setenv("MCG_TUNE_CACHE", str(tmp_path / "tune.json"))
    w = workload("cfg3s")
    s, _ = gpu_solver(w, S.PREC_MIXED, autotune=True)
    assert s.lanes in (1, 2, 4, 8, 16, 32, 64)
    assert (tmp_path / "tune.json").exists()
    s2, _ = gpu_solver(w, S.PREC_MIXED, autotune=True)      # from the cache
    assert s2.lanes == s.lanes
    x = np.random.default_rng(8).standard_normal(w.n)
    y = s.spmv(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = O.spmv(w.row_ptr, w.col, w.val, x)
    assert np.all(np.abs(y - ref) <= 8 * EPS64 * absAx(w, x) + 1e-300)
    for L in (1, 2, 4, 16, 64):
        sl, _ = gpu_solver(w, lanes=L)
        assert sl.lanes == L
        yl = sl.spmv(torch.from_numpy(x).cuda()).cpu().numpy()
        assert np.all(np.abs(yl - ref) <= 8 * EPS64 * absAx(w, x) + 1e-300)


@pytest.mark.parametrize("precision", [S.PREC_FP64, S.PREC_MIXED])
def test_split_and_fused_mmr_give_the_same_solve(precision, tmp_path, monkeypatch):
    """Both forms of the Jacobi iteration's M_mr apply (one fused kernel, or
    SpMV + streaming rank-k pass) solve to the oracle's accuracy."""
    monkeypatch.setenv("MCG_TUNE_CACHE", str(tmp_path / "t.json"))
    w = workload("cfg2s")
    s, b = gpu_solver(w, precision, autotune=True)
    x1, st1 = s.solve(b, s.preconditioner("jacobi"), rtol_out=1e-8, rtol_in=1e-3)
    assert st1.status == 0 and _true_relres(w, x1.cpu().numpy()) <= 1e-8
    for L in (1, 4):
        for form in (1, 2):
            s2, _ = gpu_solver(w, precision, lanes=L, mmr_form=form)
            assert s2.mmr_split == (form == 2)
            x2, st2 = s2.solve(b, s2.preconditioner("jacobi"), rtol_out=1e-8, rtol_in=1e-3)
            assert st2.status == 0 and _true_relres(w, x2.cpu().numpy()) <= 1e-8
            if precision == S.PREC_FP64:
                assert abs(st2.inner_its_total - st1.inner_its_total) <= 0.05 * st1.inner_its_total


def test_block_csr_is_used_only_for_dense_blocks():
    """FE-like 3-dof matrices get the block CSR copy (the cfg3s SpMV, M_mr and
    solve tests above then run through it); a scalar Laplacian asked for
    2 x 2 blocks has sparse blocks and stays in CSR, with the same products."""
    s3, _ = gpu_solver(workload("cfg3s"), S.PREC_MIXED)
    assert s3.block_csr == 3
    w2 = W.shifted_laplace3d(dims=(24, 21, 19), k=4)  # n even, so blocks of 2 are possible
    s2, _ = gpu_solver(w2, block_size=2)
    assert s2.block_csr == 0
    x = np.random.default_rng(5).standard_normal(w2.n)
    y = s2.spmv(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = O.spmv(w2.row_ptr, w2.col, w2.val, x)
    assert np.all(np.abs(y - ref) <= 8 * EPS64 * absAx(w2, x) + 1e-300)


# -- storage formats of A for the inner products ---------------------------------

def permuted(w, seed):
    """P A P^T x = P b with P a random permutation: the same spectrum and
    deflation space (rows of Vhat permuted), but column offsets up to n."""
    import scipy.sparse as sp
    perm = np.random.default_rng(seed).permutation(w.n)
    A = sp.csr_matrix((w.val, w.col, w.row_ptr), shape=(w.n, w.n))[perm][:, perm].tocsr()
    A.sort_indices()
    return W.Workload(w.name + "_perm", A.indptr.astype(np.int32), A.indices.astype(np.int32),
                      A.data.copy(), w.b[perm].copy(), np.asfortranarray(w.Vhat[perm]),
                      w.lam.copy(), w.sigma, dict(w.meta))


def check_products(w, s):
    x = np.random.default_rng(31).standard_normal(w.n)
    y = s.spmv(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = O.spmv(w.row_ptr, w.col, w.val, x)
    assert np.all(np.abs(y - ref) <= 8 * EPS64 * absAx(w, x) + 1e-300)
    if s.precision == S.PREC_MIXED:
        y32 = s.spmv(torch.from_numpy(x).float().cuda(), S.PREC_MIXED).cpu().numpy()
        ref32 = O.spmv(w.row_ptr, w.col, f32(w.val), f32(x))
        bound = 2 * np.diff(w.row_ptr) * EPS32 * O.spmv(w.row_ptr, w.col, np.abs(f32(w.val)),
                                                         np.abs(f32(x)))
        assert np.all(np.abs(y32.astype(np.float64) - ref32) <= bound)
    q = s.mmr_apply(torch.from_numpy(x).cuda()).cpu().numpy()
    refq = O.mmr_apply(w.row_ptr, w.col, w.val, w.Vhat, w.lam, x)
    scale = absAx(w, x) + 2 * np.abs(w.Vhat) @ (np.abs(w.lam) * (np.abs(w.Vhat).T @ np.abs(x)))
    assert np.all(np.abs(q - refq) <= 64 * EPS64 * scale)


@pytest.mark.parametrize("fmt,bits", [(0, 16), (2, 32), (1, 0)])
@pytest.mark.parametrize("name", ["cfg1", "cfg2s"])
def test_storage_formats_give_the_same_products(name, fmt, bits):
    """Automatic choice on stencil matrices: sliced ELL with 16-bit column
    offsets; forced 32-bit columns; CSR only.  The ragged last slice (cfg2s:
    9177 rows) is covered."""
    w = workload(name)
    s, _ = gpu_solver(w, S.PREC_MIXED, spmv_format=fmt)
    assert s.sliced_ell == bits and s.block_csr == 0
    check_products(w, s)


def test_sliced_ell_with_wide_offsets_uses_32_bit_columns():
    """Rows in random order: offsets exceed 16 bits, slices mix row lengths;
    products and a mixed-precision solve through the 32-bit sliced copy."""
    w = permuted(W.shifted_laplace3d(dims=(40, 30, 30), k=6, seed=33), 34)
    s, b = gpu_solver(w, S.PREC_MIXED)
    assert s.sliced_ell == 32
    check_products(w, s)
    x, st = s.solve(b, s.preconditioner("jacobi"), rtol_out=1e-8, rtol_in=1e-4)
    assert st.status == 0 and _true_relres(w, x.cpu().numpy()) <= 1e-8


@pytest.mark.parametrize("name,pcname", [("cfg2s", "jacobi"), ("cfg2s", "ildl0"),
                                         ("cfg3s", "jacobi"), ("cfg3s", "ildl0")])
def test_sliced_ell_and_csr_solves_agree(name, pcname):
    """FP64 solves with A in its automatic storage (sliced ELL for the scalar
    Laplacian, sliced 3 x 3 blocks for the FE-like matrix) and in CSR: same
    iterations (to the rounding of different summation orders) and both to
    the tolerance."""
    w = workload(name)
    out = []
    for fmt in (0, 1):
        s, b = gpu_solver(w, S.PREC_FP64, spmv_format=fmt)
        if name == "cfg2s":
            assert (s.sliced_ell > 0) == (fmt == 0)
        else:
            assert s.block_csr == (3 if fmt == 0 else 0) and s.sliced_ell == 0
        x, st = s.solve(b, s.preconditioner(pcname), rtol_out=1e-8, rtol_in=1e-3)
        assert st.status == 0 and _true_relres(w, x.cpu().numpy()) <= 1e-8
        out.append(st)
    assert out[0].outer_its == out[1].outer_its
    assert abs(out[0].inner_its_total - out[1].inner_its_total) <= 0.02 * out[1].inner_its_total + 2


@pytest.mark.parametrize("fmt,bits", [(0, 16), (2, 32)])
@pytest.mark.parametrize("form", [1, 2])
def test_sliced_ell_fused_and_split_forms(form, fmt, bits):
    """Both M_mr forms over the sliced copy (16-bit and forced 32-bit columns):
    products against the oracle and mixed-precision solves to the tolerance."""
    w = workload("cfg2s")
    s, b = gpu_solver(w, S.PREC_MIXED, spmv_format=fmt, mmr_form=form)
    assert s.sliced_ell == bits and s.mmr_split == (form == 2)
    check_products(w, s)
    for pcname in ("jacobi", "ildl0"):
        x, st = s.solve(b, s.preconditioner(pcname), rtol_out=1e-8, rtol_in=1e-4)
        assert st.status == 0 and _true_relres(w, x.cpu().numpy()) <= 1e-8, pcname


def test_solve_ignores_stale_workspace_contents():
    """Workspace memory handed back by a freed NaN-filled buffer: the MINRES
    direction vectors start from zero, so the solve is unaffected (the first
    two direction updates scale the older directions by zero)."""
    w = workload("cfg2s")
    junk = torch.full((1 << 27,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    del junk
    torch.cuda.empty_cache()
    s, b = gpu_solver(w, S.PREC_MIXED)
    x, st = s.solve(b, s.preconditioner("jacobi"), rtol_out=1e-8, rtol_in=1e-4)
    assert st.status == 0 and _true_relres(w, x.cpu().numpy()) <= 1e-8


# -- degenerate sizes and structures ------------------------------------------------

def small_system(n, kind, seed):
    """Tiny indefinite systems with exact deflation data: 'diag' (A diagonal,
    V-hat = unit vectors of its negative entries) and 'tridiag' (a shifted
    1D Laplacian; dense eigendecomposition)."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    if kind == "diag":
        d = rng.uniform(0.5, 2.0, n)
        d[rng.choice(n, size=max(1, min(n // 5, 40)), replace=False)] *= -1.0
        A = sp.diags(d).tocsr()
        neg = np.flatnonzero(d < 0)
        V = np.zeros((n, neg.size))
        V[neg, np.arange(neg.size)] = 1.0
        lam = d[neg]
    else:
        A0 = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1])
        ev = np.linalg.eigvalsh(A0.toarray())
        k = min(3, n - 1)
        A = (A0 - 0.5 * (ev[k - 1] + ev[k]) * sp.identity(n)).tocsr()
        w, U = np.linalg.eigh(A.toarray())
        V, lam = U[:, :k], w[:k]
    A.sort_indices()
    return A, np.asfortranarray(V), lam, rng.standard_normal(n)


@pytest.mark.parametrize("n,kind", [(1, "diag"), (65, "diag"), (1000, "diag"), (3, "tridiag"),
                                    (130, "tridiag")])
@pytest.mark.parametrize("precision", [S.PREC_FP64, S.PREC_MIXED])
def test_degenerate_sizes_solve_exactly(n, kind, precision):
    """One row, a slice plus one row, diagonal matrices (rows of length 1,
    M_mr = |A| exactly, Jacobi = A itself: an indefinite second-level
    preconditioner) and short tridiagonals: the solution matches the direct
    solve to the residual bound."""
    A, V, lam, b = small_system(n, kind, 40 + n)
    dev = torch.device("cuda")
    s = S.MinresCG(torch.from_numpy(A.indptr.astype(np.int32)).to(dev),
                   torch.from_numpy(A.indices.astype(np.int32)).to(dev),
                   torch.from_numpy(A.data.copy()).to(dev),
                   torch.from_numpy(np.ascontiguousarray(V)).to(dev) if V.shape[1] else None,
                   torch.from_numpy(lam).to(dev) if V.shape[1] else None, precision=precision)
    x, st = s.solve(torch.from_numpy(b).to(dev), s.preconditioner("jacobi"), rtol_out=1e-10,
                    rtol_in=1e-6)
    assert st.status == 0
    xs = np.linalg.solve(A.toarray(), b)
    smin = np.abs(np.linalg.eigvalsh(A.toarray())).min()
    r = np.linalg.norm(b - A @ x.cpu().numpy())
    assert r <= 1e-10 * np.linalg.norm(b) * (1 + 1e-6)
    assert np.linalg.norm(x.cpu().numpy() - xs) <= r / smin * (1 + 1e-6) + 1e-14
    s.close()


@pytest.mark.parametrize("name,precision,pcname", [("cfg2s", S.PREC_MIXED, "jacobi"),
                                                   ("cfg2s", S.PREC_FP64, "ildl0"),
                                                   ("cfg2s", S.PREC_MIXED, "smw"),
                                                   ("cfg3s", S.PREC_MIXED, "jacobi"),
                                                   ("cfg1", S.PREC_FP64, "jacobi")])
def test_graph_replay_matches_eager(name, precision, pcname):
    """Inner iterations replayed from the captured 32-iteration HIP graph give
    bitwise the eager launches' results, solve after solve (different
    right-hand sides, eager work in between)."""
    w = workload(name)
    sg, b = gpu_solver(w, precision)
    se, _ = gpu_solver(w, precision, eager=True)
    kw = dict(smw=True) if pcname == "smw" else {}
    pk = "jacobi" if pcname == "smw" else pcname
    pg, pe = sg.preconditioner(pk, **kw), se.preconditioner(pk, **kw)
    for rep in range(3):
        bb = b * (1.0 + 0.25 * rep) + rep
        torch.cuda.synchronize()
        xg, stg = sg.solve(bb, pg, rtol_out=1e-8, rtol_in=1e-4)
        xe, ste = se.solve(bb, pe, rtol_out=1e-8, rtol_in=1e-4)
        assert stg.status == 0 and ste.status == 0
        assert stg.inner_its_total == ste.inner_its_total, rep
        assert torch.equal(xg, xe), rep
        _ = (xg * 2).sum()      # eager torch work between replays


def test_zero_inner_budget_returns_x0_like_the_oracle():
    """No inner iteration allowed: MAXIT, x = x0, nothing read from a stale z."""
    w = workload("cfg2s")
    s, b = gpu_solver(w)
    pc = s.preconditioner("jacobi")
    x0 = torch.from_numpy(np.random.default_rng(5).standard_normal(w.n)).cuda()
    x, st = s.solve(b, pc, x0=x0, maxit_inner_total=0)
    P = O.Problem(w.row_ptr, w.col, w.val, w.Vhat, w.lam)
    ro = O.minres_cg(P, O.InnerPC(O.PC_JACOBI, P), w.b, x0=x0.cpu().numpy(), maxit_in_total=0)
    assert st.status == ro["status"] == O.MAXIT
    assert st.outer_its == 0 and st.inner_its_total == 0
    assert torch.equal(x, x0)
    z, rc, its = s.pcg(b, pc, rtol=1e-6, maxit=0)
    assert rc == O.MAXIT and its == 0 and torch.count_nonzero(z) == 0


def test_ildl0_rejects_an_exactly_zero_pivot():
    """[[0, 1], [1, 0]] with the zero diagonal stored: pivtol = 0 leaves d = 0."""
    dev = torch.device("cuda")
    rp = torch.tensor([0, 2, 4], dtype=torch.int32, device=dev)
    ci = torch.tensor([0, 1, 0, 1], dtype=torch.int32, device=dev)
    va = torch.tensor([0.0, 1.0, 1.0, 0.0], dtype=torch.float64, device=dev)
    s = S.MinresCG(rp, ci, va)
    with pytest.raises(S.MCGError):
        s.preconditioner("ildl0", pivtol=0.0)
    pc = s.preconditioner("ildl0", pivtol=1e-8)     # floored pivots: usable
    t = pc.apply(torch.ones(2, dtype=torch.float64, device=dev))
    assert torch.isfinite(t).all()


def test_stagnation_and_best_iterate_match_the_oracle():
    """Loose inner solves (rtol_in 0.5) stall MINRES on this system (the
    paper's double-dagger mark); both sides report STAGNATION and return the
    iterate with the smallest true residual."""
    w = W.shifted_laplace2d(m=16, k=4)
    s, b = gpu_solver(w)
    x, st = s.solve(b, s.preconditioner("jacobi"), rtol_out=1e-12, rtol_in=0.5, maxit_out=300)
    P = O.Problem(w.row_ptr, w.col, w.val, w.Vhat, w.lam)
    ro = O.minres_cg(P, O.InnerPC(O.PC_JACOBI, P), w.b, rtol_out=1e-12, rtol_in=0.5,
                     maxit_out=300, stag_window=10)
    assert st.status == ro["status"] == O.STAGNATION
    rg = _true_relres(w, x.cpu().numpy())
    hist = st.relres[~np.isnan(st.relres)]
    assert abs(rg - hist.min()) <= 1e-10 * rg
    assert abs(rg - st.final_relres) <= 1e-10 * rg
    assert abs(rg - ro["final_relres"]) <= 0.2 * ro["final_relres"]
