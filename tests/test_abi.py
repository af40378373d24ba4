"""C ABI: the library loads without a GPU, exports every function that the
headers under include/ declare, and answers the host-only queries."""
import ctypes as C
import glob
import json
import os
import re

import pytest

from paper_1805_12417_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def declared_functions():
    text = "\n".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n.startswith(("minres_cg_", "mcg_"))))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("minres_cg_create", "minres_cg_solve", "minres_cg_free", "minres_cg_precond_create",
                 "mcg_spmv", "mcg_mmr_apply", "mcg_precond_apply", "mcg_pcg_solve",
                 "mcg_learned_create", "mcg_learned_forward", "mcg_learned_loss_grad",
                 "mcg_learned_adam", "mcg_learned_factor"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = N.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_storage_matches_paper_table():
    """Table "storage": MINRES-CG keeps 11 + k vectors besides A, M and b."""
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "storage_table.json")))
    L = N.lib()
    paper, total = C.c_int32(), C.c_int32()
    for k in (0, 6, 20, 30, 64):
        assert L.minres_cg_workspace_vectors(k, N.PREC_FP64, N.PC_JACOBI, C.byref(paper),
                                             C.byref(total)) == 0
        assert paper.value == golden["MINRES-CG"]["constant"] + golden["MINRES-CG"]["per_k"] * k
        assert total.value >= paper.value
    assert L.minres_cg_workspace_vectors(65, 0, 1, C.byref(paper), C.byref(total)) == N.EINVAL


def test_default_options_and_strings():
    L = N.lib()
    o = N.Options()
    L.minres_cg_default_options(C.byref(o))
    assert (o.precision, o.stag_window, o.keep_best, o.block_size) == (0, 10, 1, 1)
    assert N.strerror(0) == "converged"
    assert "invalid" in N.strerror(-1)
    assert b"gfx950" in L.minres_cg_version()


def test_null_arguments_are_rejected_without_a_gpu():
    L = N.lib()
    h = C.c_void_p()
    assert L.minres_cg_create(None, None, 0, None, None, None, None) == N.EINVAL
    A = N.CSR(0, 0, None, None, None)
    assert L.minres_cg_create(C.byref(h), C.byref(A), 0, None, None, None, None) == N.EINVAL
    assert L.minres_cg_solve(None, None, None, None, 1, 1e-8, 1e-3, 10, 100, None, None) == N.EINVAL
