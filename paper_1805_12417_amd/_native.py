"""ctypes binding of libminrescg.so (declarations in include/minres_cg.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Importing this module raises if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libminrescg.so")

OK, MAXIT, STAGNATION, BREAKDOWN, NOT_SPD = 0, 1, 2, 3, 4
EINVAL, EHIP, ENOMEM = -1, -2, -3
PREC_FP64, PREC_MIXED = 0, 1
PC_NONE, PC_JACOBI, PC_ILDL0, PC_ILDLP, PC_CCT, PC_SMW = 0, 1, 2, 3, 4, 0x100

STATUS_NAMES = {OK: "OK", MAXIT: "MAXIT", STAGNATION: "STAGNATION", BREAKDOWN: "BREAKDOWN",
                NOT_SPD: "NOT_SPD", EINVAL: "EINVAL", EHIP: "EHIP", ENOMEM: "ENOMEM"}


class CSR(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p)]


class IldlpParams(C.Structure):
    _fields_ = [("fill", C.c_double), ("drop", C.c_double), ("sweeps", C.c_int32)]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("spmv_lanes", C.c_int32), ("autotune", C.c_int32),
                ("stag_window", C.c_int32), ("keep_best", C.c_int32), ("block_size", C.c_int32),
                ("chunk", C.c_int32), ("profile", C.c_int32), ("mmr_form", C.c_int32),
                ("spmv_format", C.c_int32), ("eager", C.c_int32), ("xcd_order", C.c_int32),
                ("reserved", C.c_int32 * 4)]


class Stats(C.Structure):
    _fields_ = [("status", C.c_int32), ("outer_its", C.c_int32), ("inner_its_total", C.c_int64),
                ("final_relres", C.c_double), ("bnorm", C.c_double), ("hist_cap", C.c_int32),
                ("inner_its", C.POINTER(C.c_int64)), ("relres", C.POINTER(C.c_double)),
                ("phibar", C.POINTER(C.c_double))]


class EigOptions(C.Structure):
    _fields_ = [("block", C.c_int32), ("degree", C.c_int32), ("max_outer", C.c_int32),
                ("reserved0", C.c_int32), ("tol", C.c_double), ("seed", C.c_uint64)]


class EigStats(C.Structure):
    _fields_ = [("outer_its", C.c_int32), ("spmm_calls", C.c_int32), ("negative", C.c_int32),
                ("converged", C.c_int32), ("max_residual", C.c_double), ("bound", C.c_double),
                ("next_ritz", C.c_double)]


class BatchStats(C.Structure):
    _fields_ = [("status", C.POINTER(C.c_int32)), ("outer_its", C.POINTER(C.c_int32)),
                ("inner_its", C.POINTER(C.c_int64)), ("relres", C.POINTER(C.c_double))]


_lib = None


class LibraryMissing(RuntimeError):
    pass


def lib():
    """The loaded library; raises LibraryMissing if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(
            "libminrescg.so not found at %s: build it with "
            "`python -m paper_1805_12417_amd.csrc.build` (hipcc, gfx950)" % LIB_PATH)
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.minres_cg_default_options.argtypes = [C.POINTER(Options)]
    L.minres_cg_default_options.restype = None
    L.minres_cg_create.argtypes = [C.POINTER(vp), C.POINTER(CSR), i32, vp, vp, C.POINTER(Options), vp]
    L.minres_cg_free.argtypes = [vp]
    L.minres_cg_free.restype = None
    L.minres_cg_precond_create.argtypes = [C.POINTER(vp), vp, i32, vp, vp]
    L.minres_cg_precond_free.argtypes = [vp]
    L.minres_cg_precond_free.restype = None
    L.minres_cg_solve.argtypes = [vp, vp, vp, vp, i32, d, d, i32, i64, C.POINTER(Stats), vp]
    L.minres_cg_create_batch.argtypes = [C.POINTER(vp), i32, C.POINTER(CSR), C.POINTER(i32),
                                         C.POINTER(vp), C.POINTER(vp), i32, C.POINTER(Options), vp]
    L.minres_cg_create_batch.restype = C.c_int
    L.mcg_spmv.argtypes = [vp, i32, vp, vp, vp]
    L.mcg_mmr_apply.argtypes = [vp, i32, vp, vp, vp]
    L.mcg_precond_apply.argtypes = [vp, i32, vp, vp, vp]
    L.mcg_pcg_solve.argtypes = [vp, vp, vp, vp, d, i64, C.POINTER(i64), vp]
    L.minres_cg_kernel_time.argtypes = [vp, C.POINTER(d), C.POINTER(i64), i32]
    L.minres_cg_spmv_lanes.argtypes = [vp]
    L.minres_cg_spmv_lanes.restype = C.c_int
    L.minres_cg_mmr_split.argtypes = [vp]
    L.minres_cg_mmr_split.restype = C.c_int
    L.minres_cg_block_csr.argtypes = [vp]
    L.minres_cg_block_csr.restype = C.c_int
    L.minres_cg_sliced_ell.argtypes = [vp]
    L.minres_cg_sliced_ell.restype = C.c_int
    L.minres_cg_sliced_blocks.argtypes = [vp]
    L.minres_cg_sliced_blocks.restype = C.c_int
    L.minres_cg_xcd_sections.argtypes = [vp]
    L.minres_cg_xcd_sections.restype = C.c_int
    L.minres_cg_batch_create.argtypes = [C.POINTER(vp), i32, C.POINTER(CSR), C.POINTER(i32),
                                         C.POINTER(vp), C.POINTER(vp), i32, C.POINTER(Options), vp]
    L.minres_cg_batch_solve.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), d, d, i32, i64, i32,
                                        C.POINTER(BatchStats), vp]
    L.minres_cg_batch_solve_streams.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), d, d, i32, i64,
                                                i32, C.POINTER(BatchStats), vp]
    L.minres_cg_batch_info.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
    L.minres_cg_batch_system.argtypes = [vp, i32, C.POINTER(vp)]
    L.minres_cg_batch_system.restype = C.c_int
    L.minres_cg_batch_solve_streams_pc.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                                                   d, d, i32, i64, i32, C.POINTER(BatchStats), vp]
    L.minres_cg_batch_solve_streams_pc.restype = C.c_int
    L.minres_cg_batch_profile.argtypes = [vp, vp, vp, vp, vp, vp, C.POINTER(d)]
    L.minres_cg_batch_profile.restype = C.c_int
    L.minres_cg_batch_rebalance.argtypes = [vp, C.POINTER(d)]
    L.minres_cg_batch_rebalance_measured.argtypes = [vp]
    L.minres_cg_batch_rebalance_measured.restype = C.c_int
    L.minres_cg_batch_free.argtypes = [vp]
    L.minres_cg_batch_free.restype = None
    L.minres_cg_eig_default_options.argtypes = [C.POINTER(EigOptions)]
    L.minres_cg_eig_default_options.restype = None
    L.minres_cg_lowest_eigs.argtypes = [C.POINTER(CSR), i32, C.POINTER(EigOptions), vp, vp,
                                        C.POINTER(EigStats), vp]
    L.minres_cg_lowest_eigs.restype = C.c_int
    L.minres_cg_solve_record.argtypes = [vp, vp, vp, vp, d, d, i32, i64, vp, vp, i32,
                                         C.POINTER(i32), C.POINTER(Stats), vp]
    L.minres_cg_solve_record.restype = C.c_int
    L.mcg_ildlp_factor_get.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, C.POINTER(i64)]
    L.mcg_ildlp_factor_get.restype = C.c_int
    L.mcg_mmr_apply_noalloc.argtypes = [C.POINTER(CSR), i32, vp, vp, vp, vp, vp]
    L.mcg_mmr_apply_noalloc.restype = C.c_int
    L.minres_cg_workspace_vectors.argtypes = [i32, i32, i32, C.POINTER(i32), C.POINTER(i32)]
    L.minres_cg_strerror.argtypes = [C.c_int]
    L.minres_cg_strerror.restype = C.c_char_p
    L.minres_cg_version.restype = C.c_char_p
    f32 = C.c_float
    L.mcg_learned_create.argtypes = [C.POINTER(vp), C.POINTER(CSR), i32, vp]
    L.mcg_learned_free.argtypes = [vp]
    L.mcg_learned_free.restype = None
    L.mcg_learned_num_params.argtypes = [vp]
    L.mcg_learned_num_params.restype = i64
    L.mcg_learned_sizes.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
    L.mcg_learned_set_params.argtypes = [vp, vp, vp]
    L.mcg_learned_get_params.argtypes = [vp, vp, vp]
    L.mcg_learned_forward.argtypes = [vp, vp]
    L.mcg_learned_factor.argtypes = [vp, C.POINTER(CSR)]
    L.mcg_learned_factor_copy.argtypes = [vp, vp, vp, vp, vp]
    L.mcg_learned_loss_grad.argtypes = [vp, vp, vp, i32, C.POINTER(d), vp, vp]
    L.mcg_learned_adam.argtypes = [i64, vp, vp, vp, vp, f32, f32, f32, f32, i32, vp]
    L.mcg_learned_forward_ms.argtypes = [vp]
    L.mcg_learned_forward_ms.restype = d
    for name in ("mcg_learned_create", "mcg_learned_sizes", "mcg_learned_set_params",
                 "mcg_learned_get_params", "mcg_learned_forward", "mcg_learned_factor",
                 "mcg_learned_factor_copy",
                 "mcg_learned_loss_grad", "mcg_learned_adam"):
        getattr(L, name).restype = C.c_int
    for name in ("minres_cg_create", "minres_cg_precond_create", "minres_cg_solve", "mcg_spmv",
                 "mcg_mmr_apply", "mcg_precond_apply", "mcg_pcg_solve",
                 "minres_cg_workspace_vectors", "minres_cg_kernel_time", "minres_cg_batch_create",
                 "minres_cg_batch_solve", "minres_cg_batch_solve_streams",
                 "minres_cg_batch_info"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def strerror(code: int) -> str:
    return lib().minres_cg_strerror(int(code)).decode()
