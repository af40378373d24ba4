"""The allocation-free M_mr apply (mcg_mmr_apply_noalloc) against the
handle-based mcg_mmr_apply, through the C ABI: two calls in a row, the
second on a smaller system (the library's fixed workspace keeps the first
call's contents), then replays of a captured graph of the call with eager
work in between.  Bar: the FP64 M_mr apply's, |q - q_ref| <= 1e-12 ||q_ref||
norm-wise and per entry (both sum the same products in different orders)."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_1805_12417_amd import _native as N
from paper_1805_12417_amd import solver as S
from paper_1805_12417_amd import workloads as W

pytestmark = pytest.mark.gpu


def dev_parts(w):
    d = torch.device("cuda")
    return (torch.from_numpy(w.row_ptr).to(d), torch.from_numpy(w.col).to(d),
            torch.from_numpy(w.val).to(d), torch.from_numpy(np.ascontiguousarray(w.Vhat)).to(d),
            torch.from_numpy(w.lam).to(d))


def check(q, ref):
    q, ref = q.cpu().numpy(), ref.cpu().numpy()
    scale = np.abs(ref).max()
    assert np.linalg.norm(q - ref) <= 1e-12 * np.linalg.norm(ref)
    assert np.all(np.abs(q - ref) <= 1e-12 * scale)


def test_noalloc_mmr_apply_matches_handle_apply_twice_then_smaller():
    big = W.shifted_laplace3d(dims=(23, 21, 19), k=20)       # 9,177 rows, k = 20
    small = W.shifted_laplace2d(m=24, k=6)                    # 576 rows, k = 6
    for w, seed in ((big, 1), (small, 2)):
        rp, ci, va, V, lam = dev_parts(w)
        u = torch.from_numpy(np.random.default_rng(seed).standard_normal(w.n)).cuda()
        q = S.mmr_apply_noalloc(rp, ci, va, V, lam, u)
        s = S.MinresCG(rp, ci, va, V, lam)
        ref = s.mmr_apply(u)
        torch.cuda.synchronize()
        check(q, ref)
        s.close()


def test_noalloc_mmr_apply_k0_and_invalid_k():
    w = W.shifted_laplace2d(m=16, k=3)
    rp, ci, va, V, lam = dev_parts(w)
    u = torch.from_numpy(np.random.default_rng(3).standard_normal(w.n)).cuda()
    q = S.mmr_apply_noalloc(rp, ci, va, None, None, u)
    ref = S.MinresCG(rp, ci, va).spmv(u)
    torch.cuda.synchronize()
    check(q, ref)
    A = N.CSR(w.n, w.nnz, rp.data_ptr(), ci.data_ptr(), va.data_ptr())
    rc = N.lib().mcg_mmr_apply_noalloc(C.byref(A), 65, C.c_void_p(V.data_ptr()),
                                       C.c_void_p(lam.data_ptr()), C.c_void_p(u.data_ptr()),
                                       C.c_void_p(q.data_ptr()), None)
    assert rc == N.EINVAL


def test_noalloc_mmr_apply_replays_from_a_captured_graph():
    """Captured once, replayed three times with eager calls on other inputs
    in between: every replay equals the eager result."""
    w = W.shifted_laplace3d(dims=(17, 16, 15), k=9)
    other = W.shifted_laplace2d(m=20, k=4)
    rp, ci, va, V, lam = dev_parts(w)
    orp, oci, ova, oV, olam = dev_parts(other)
    Vt = V.t().contiguous()
    u = torch.from_numpy(np.random.default_rng(4).standard_normal(w.n)).cuda()
    ou = torch.from_numpy(np.random.default_rng(5).standard_normal(other.n)).cuda()
    q = torch.empty_like(u)
    ref = S.mmr_apply_noalloc(rp, ci, va, V, lam, u)      # eager (also the first use)
    torch.cuda.synchronize()
    A = N.CSR(w.n, w.nnz, rp.data_ptr(), ci.data_ptr(), va.data_ptr())
    side = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        rc = N.lib().mcg_mmr_apply_noalloc(C.byref(A), w.k, C.c_void_p(Vt.data_ptr()),
                                           C.c_void_p(lam.data_ptr()), C.c_void_p(u.data_ptr()),
                                           C.c_void_p(q.data_ptr()),
                                           C.c_void_p(side.cuda_stream))
    assert rc == 0
    for rep in range(3):
        q.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        check(q, ref)
        S.mmr_apply_noalloc(orp, oci, ova, oV, olam, ou)   # eager work on the same scratch
        torch.cuda.synchronize()
