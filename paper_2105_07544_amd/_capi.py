"""ctypes declarations of libgmresir.so (include/gmres_ir.h).

Argument marshalling only: every step of the solver runs in the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgmresir.so")

GMR_F32, GMR_F64 = 0, 1
GMR_FLAG_GRAPH = 1
GMR_FLAG_PERSISTENT = 2
GMR_FLAG_STOP_ON_LOSS = 4
GMR_FLAG_HALF_BASIS = 8
STATUS = {0: "GMR_OK", 1: "GMR_NOT_CONVERGED", 2: "GMR_STAGNATED", 3: "GMR_LOSS_OF_ACCURACY",
          4: "GMR_SYSTEMS_FAILED", -1: "GMR_ERR_INVALID",
          -2: "GMR_ERR_HIP", -3: "GMR_ERR_WORKSPACE", -4: "GMR_ERR_NONFINITE",
          -5: "GMR_ERR_UNSUPPORTED"}
PROF = {"none": 0, "spmv": 1, "cgs_dots": 2, "cgs_update_dots": 3, "cgs_update_norm": 4,
        "poly_step": 5, "residual": 6, "bjac": 7}

# Every symbol include/gmres_ir.h declares.
EXPORTED = ["gmres_workspace_bytes", "spmv", "cgs2_orth", "cgs2_orth_noalloc", "poly_prec_setup", "poly_prec_apply",
            "poly_prec_destroy", "bjac_prec_bytes", "bjac_prec_setup", "prec_block_size", "poly_prec_degree", "poly_prec_roots", "poly_prec_hessenberg", "gmres_solve",
            "gmres_ir_solve", "gmres_f32prec_solve", "gmres_fd_workspace_bytes", "gmres_fd_solve", "csr_values_to_f32", "gmr_hessenberg_eigvals", "gmr_harmonic_ritz", "gmr_leja_order",
            "gmr_last_error", "batch_create", "batch_destroy", "batch_workspace_bytes",
            "batch_set_tiling", "batch_set_graph", "batch_get_tiling", "batch_autotune", "batch_gmres_ir_solve", "batch_gmres_solve",
            "batch_bcgs_step", "batch_system_status", "mlp_param_count", "mlp_workspace_bytes", "mlp_forward",
            "mlp_loss_grad", "mlp_adam_step", "matrix_stats", "matrix_features_workspace_bytes",
            "matrix_features"]


class gmr_csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("val", C.c_void_p), ("dtype", C.c_int32)]


class gmr_params(C.Structure):
    _fields_ = [("restart", C.c_int32), ("tol", C.c_double), ("max_iters", C.c_int64),
                ("max_cycles", C.c_int32), ("stagnation_cycles", C.c_int32),
                ("prof_kernel", C.c_int32), ("flags", C.c_int32)]


class gmr_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("cycles", C.c_int32), ("iters", C.c_int64),
                ("rel_res", C.c_double), ("implicit_rel_res", C.c_double),
                ("seconds", C.c_double), ("history_len", C.c_int32), ("loss_of_accuracy", C.c_int32),
                ("prof_ms", C.c_double), ("prof_launches", C.c_int64),
                ("prof_bytes", C.c_double)]


class gmr_batch_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("cycles", C.c_int32), ("block_iters", C.c_int64),
                ("max_rel_res", C.c_double), ("seconds", C.c_double)]


_lib = None


def load() -> C.CDLL:
    """Load the built library; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2105_07544_amd.build.build()")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    st = C.c_int
    lib.gmres_workspace_bytes.argtypes = [C.c_int32, C.POINTER(gmr_params), C.c_int32, C.c_int32]
    lib.gmres_workspace_bytes.restype = C.c_size_t
    lib.spmv.argtypes = [C.POINTER(gmr_csr), P, P, P]
    lib.spmv.restype = st
    lib.cgs2_orth.argtypes = [C.c_int32, C.c_int32, C.c_int32, P, C.c_int64, P, P, P, C.c_size_t, P]
    lib.cgs2_orth.restype = st
    lib.cgs2_orth_noalloc.argtypes = [C.c_int32, C.c_int32, C.c_int32, P, C.c_int64, P, P, P]
    lib.cgs2_orth_noalloc.restype = st
    lib.poly_prec_setup.argtypes = [C.POINTER(gmr_csr), C.c_int32, P, P, C.c_size_t, C.POINTER(P), P]
    lib.poly_prec_setup.restype = st
    lib.poly_prec_apply.argtypes = [P, C.POINTER(gmr_csr), P, P, P, C.c_size_t, P]
    lib.poly_prec_apply.restype = st
    lib.poly_prec_destroy.argtypes = [P]
    lib.poly_prec_destroy.restype = None
    lib.poly_prec_degree.argtypes = [P]
    lib.poly_prec_degree.restype = C.c_int32
    lib.poly_prec_roots.argtypes = [P, P, P]
    lib.poly_prec_roots.restype = st
    lib.gmres_solve.argtypes = [C.POINTER(gmr_csr), P, P, P, C.POINTER(gmr_params), P, C.c_size_t,
                                C.POINTER(gmr_result), P, P]
    lib.gmres_solve.restype = st
    lib.gmres_ir_solve.argtypes = [C.POINTER(gmr_csr), C.POINTER(gmr_csr), P, P, P,
                                   C.POINTER(gmr_params), P, C.c_size_t, C.POINTER(gmr_result), P, P]
    lib.gmres_ir_solve.restype = st
    lib.bjac_prec_bytes.argtypes = [C.c_int32, C.c_int32, C.c_int32]
    lib.bjac_prec_bytes.restype = C.c_size_t
    lib.bjac_prec_setup.argtypes = [C.POINTER(gmr_csr), C.c_int32, P, C.c_size_t, C.POINTER(C.c_void_p), P]
    lib.bjac_prec_setup.restype = st
    lib.prec_block_size.argtypes = [P]
    lib.prec_block_size.restype = C.c_int32
    lib.gmres_f32prec_solve.argtypes = [C.POINTER(gmr_csr), C.POINTER(gmr_csr), P, P, P,
                                        C.POINTER(gmr_params), P, C.c_size_t, C.POINTER(gmr_result), P, P]
    lib.gmres_f32prec_solve.restype = st
    lib.gmres_fd_workspace_bytes.argtypes = [C.c_int32, C.POINTER(gmr_params)]
    lib.gmres_fd_workspace_bytes.restype = C.c_size_t
    lib.gmres_fd_solve.argtypes = [C.POINTER(gmr_csr), C.POINTER(gmr_csr), P, P, C.POINTER(gmr_params),
                                   C.c_int64, P, C.c_size_t, C.POINTER(gmr_result), C.POINTER(gmr_result),
                                   P, P]
    lib.gmres_fd_solve.restype = st
    lib.csr_values_to_f32.argtypes = [P, P, C.c_int64, P]
    lib.csr_values_to_f32.restype = st
    lib.gmr_hessenberg_eigvals.argtypes = [C.c_int32, P, P, P]
    lib.gmr_hessenberg_eigvals.restype = st
    lib.poly_prec_hessenberg.argtypes = [P, P]
    lib.poly_prec_hessenberg.restype = st
    lib.gmr_harmonic_ritz.argtypes = [C.c_int32, P, C.c_int32, P, P]
    lib.gmr_harmonic_ritz.restype = st
    lib.gmr_leja_order.argtypes = [C.c_int32, P, P]
    lib.gmr_leja_order.restype = st
    lib.batch_create.argtypes = [C.c_int32, P, C.c_int32, C.c_int32, C.POINTER(P)]
    lib.batch_create.restype = st
    lib.batch_destroy.argtypes = [P]
    lib.batch_destroy.restype = None
    lib.batch_workspace_bytes.argtypes = [P, C.c_int32]
    lib.batch_workspace_bytes.restype = C.c_size_t
    lib.batch_set_tiling.argtypes = [P, C.c_int32, C.c_int32]
    lib.batch_set_tiling.restype = st
    lib.batch_set_graph.argtypes = [P, C.c_int32]
    lib.batch_set_graph.restype = st
    lib.batch_get_tiling.argtypes = [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.batch_get_tiling.restype = st
    lib.batch_autotune.argtypes = [P, P, C.c_size_t, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                   C.POINTER(C.c_double), P]
    lib.batch_autotune.restype = st
    lib.batch_gmres_ir_solve.argtypes = [P, C.POINTER(gmr_csr), C.POINTER(gmr_csr), P, P, P, C.c_double,
                                         C.c_int32, P, C.c_size_t, C.POINTER(gmr_batch_result), P, P, P]
    lib.batch_gmres_ir_solve.restype = st
    lib.batch_gmres_solve.argtypes = [P, C.POINTER(gmr_csr), P, P, P, C.c_double, C.c_int32, P, C.c_size_t,
                                      C.POINTER(gmr_batch_result), P, P, P]
    lib.batch_gmres_solve.restype = st
    lib.batch_bcgs_step.argtypes = [P, P, C.c_int32, P, P, P, C.c_size_t, P]
    lib.batch_bcgs_step.restype = st
    lib.batch_system_status.argtypes = [P, P]
    lib.batch_system_status.restype = st
    lib.mlp_param_count.argtypes = []
    lib.mlp_param_count.restype = C.c_int32
    lib.mlp_workspace_bytes.argtypes = [C.c_int32]
    lib.mlp_workspace_bytes.restype = C.c_size_t
    lib.mlp_forward.argtypes = [P, P, P, P, C.c_int32, P, P]
    lib.mlp_forward.restype = st
    lib.mlp_loss_grad.argtypes = [P, P, P, P, P, C.c_int32, P, P, P, C.c_size_t, P]
    lib.mlp_loss_grad.restype = st
    lib.mlp_adam_step.argtypes = [P, P, P, P, C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float, P]
    lib.mlp_adam_step.restype = st
    lib.matrix_stats.argtypes = [C.POINTER(gmr_csr), P, P, C.c_size_t, P]
    lib.matrix_stats.restype = st
    lib.matrix_features_workspace_bytes.argtypes = [C.c_int32, C.c_int32]
    lib.matrix_features_workspace_bytes.restype = C.c_size_t
    lib.matrix_features.argtypes = [C.POINTER(gmr_csr), P, P, P, C.c_size_t, P]
    lib.matrix_features.restype = st
    lib.gmr_last_error.argtypes = []
    lib.gmr_last_error.restype = C.c_char_p
    _lib = lib
    return lib


class GmresError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def check(status: int) -> int:
    if status < 0:
        raise GmresError(status, load().gmr_last_error().decode())
    return status
