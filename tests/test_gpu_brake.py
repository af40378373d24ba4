"""The disk-brake inner-level systems (Section 3.1, eq. inner_level): a sweep
of shifts gamma of one modulus shares the matrix K_E - |gamma|^2 M, so the
deflation data (V_hat, Lambda_hat) and the second-level preconditioner are
built once and reused for every right-hand side -gamma_i v.  One solver
handle and one preconditioner serve the whole sweep on the GPU; every solve
is checked against its own FP64 oracle solve (same inputs): FP64 true
relative residual <= rtol for both, and the solutions within max(1e-6 ||x_o||,
(r + r_o) ||b|| / min|lambda(A)|)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1805_12417_amd import solver as S
from paper_1805_12417_amd import workloads as W

pytestmark = pytest.mark.gpu


def run_sweep(w, count, precision, pcname, rtol=1e-8, rtol_in=1e-4):
    P = O.Problem(w.row_ptr, w.col, w.val, w.Vhat, w.lam)
    pco = O.InnerPC(O.PC_ILDL0 if pcname == "ildl0" else O.PC_JACOBI, P)
    s, _ = S.from_workload(w, precision=precision)
    pc = s.preconditioner(pcname)                      # built once for the sweep
    nb = []
    for gamma, b in W.brake_sweep_rhs(w, count, 11):
        x, st = s.solve(torch.from_numpy(b).cuda(), pc, rtol_out=rtol, rtol_in=rtol_in)
        ro = O.minres_cg(P, pco, b, rtol_out=rtol, rtol_in=rtol_in)
        xg = x.cpu().numpy()
        rg = np.linalg.norm(b - O.spmv(w.row_ptr, w.col, w.val, xg)) / np.linalg.norm(b)
        assert st.status == 0 and ro["status"] == 0, (gamma, st.status_name)
        assert rg <= rtol and ro["final_relres"] <= rtol
        bound = max(1e-6 * np.linalg.norm(ro["x"]),
                    (rg + ro["final_relres"]) * np.linalg.norm(b) / w.meta["min_abs_eig"])
        err = np.linalg.norm(xg - ro["x"])
        print("gamma %s: outer %d inner %d (oracle %d / %d) |x - x_o|/|x_o| = %.2e" % (
            gamma, st.outer_its, st.inner_its_total, ro["outer_its"], ro["inner_its_total"],
            err / np.linalg.norm(ro["x"])))
        assert err <= bound
        nb.append(st.inner_its_total)
    pc.close()
    s.close()
    return nb


@pytest.mark.parametrize("precision,pcname", [(S.PREC_FP64, "ildl0"), (S.PREC_MIXED, "ildl0"),
                                              (S.PREC_MIXED, "jacobi")])
def test_brake_sweep_small(precision, pcname):
    w = W.brake_inner_level(m=8, k=6)              # 1,536 unknowns
    run_sweep(w, 4, precision, pcname)


def test_brake_sweep_medium():
    """12,288 unknowns, 10 negative eigenvalues, deflation data from the
    generator's GPU eigensolver."""
    w = W.brake_inner_level(m=16, k=10, device="cuda")
    run_sweep(w, 3, S.PREC_MIXED, "ildl0")
