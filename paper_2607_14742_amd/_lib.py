"""ctypes declarations of the C ABI in include/mpcare.h (argument marshalling
only: every computation runs in libmpcare.so)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpcare.so")

CARE_OK, CARE_WARN_STAGNATED, CARE_WARN_MAXIT = 0, 1, 2
CARE_ERR_ARG, CARE_ERR_CAPACITY, CARE_ERR_UNSTABLE, CARE_ERR_BREAKDOWN = -1, -2, -3, -4
CARE_ERR_NONFINITE, CARE_ERR_DEVICE, CARE_ERR_NOMEM, CARE_ERR_NOT_IMPLEMENTED = -5, -6, -7, -8
CARE_FP64, CARE_FP32, CARE_BF16_SPMM, CARE_AUTO, CARE_FP16_SPMM = 0, 1, 2, 3, 4

STATUS_NAMES = {
    0: "CARE_OK", 1: "CARE_WARN_STAGNATED", 2: "CARE_WARN_MAXIT", -1: "CARE_ERR_ARG",
    -2: "CARE_ERR_CAPACITY", -3: "CARE_ERR_UNSTABLE", -4: "CARE_ERR_BREAKDOWN",
    -5: "CARE_ERR_NONFINITE", -6: "CARE_ERR_DEVICE", -7: "CARE_ERR_NOMEM", -8: "CARE_ERR_NOT_IMPLEMENTED",
}


class care_csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p), ("val", C.c_void_p)]


class care_shift(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class care_opts(C.Structure):
    _fields_ = [
        ("inner_prec", C.c_int32), ("k_max", C.c_int32), ("k0_max", C.c_int32), ("j_max", C.c_int32),
        ("eta_r_rel", C.c_double), ("eta_s_rel", C.c_double), ("tau_L", C.c_double), ("tau_0", C.c_double),
        ("stagnation", C.c_double), ("krylov_maxit", C.c_int32), ("krylov_tol", C.c_double),
        ("check_every", C.c_int32), ("penzl_l0", C.c_int32), ("penzl_kp", C.c_int32), ("penzl_km", C.c_int32),
        ("profile", C.c_int32), ("Z_init", C.c_void_p), ("ldz_init", C.c_int64), ("r_init", C.c_int32),
        ("adi_deflate", C.c_int32), ("krylov_block_tol", C.c_int32), ("penzl_real", C.c_int32),
        ("spmm_split", C.c_int32), ("krylov_relax", C.c_int32), ("refine_forcing", C.c_double),
        ("tau_L0", C.c_double), ("spmm_tune", C.c_int32), ("shift_update", C.c_int32),
        ("krylov_method", C.c_int32), ("krylov_restart", C.c_int32), ("krylov_compact", C.c_int32),
        ("adi_rotate", C.c_int32), ("krylov_rb", C.c_int32), ("krylov_precond", C.c_int32),
    ]


class care_stats(C.Structure):
    _fields_ = [
        ("iter0_outer", C.c_int32), ("iter0_inner", C.c_int32), ("iter_outer", C.c_int32),
        ("iter_inner", C.c_int32), ("rank", C.c_int32), ("stagnated", C.c_int32),
        ("res_rel", C.c_double), ("res_paper", C.c_double), ("eta_n", C.c_double),
        ("t_total", C.c_double), ("t_stage0", C.c_double), ("t_refine", C.c_double), ("t_setup", C.c_double),
        ("spmm_calls", C.c_int64), ("spmm_bytes", C.c_double), ("t_spmm", C.c_double),
        ("krylov_iters", C.c_int64), ("hist_len", C.c_int32), ("res_hist", C.c_double * 48),
        ("inner_prec", C.c_int32), ("krylov_compactions", C.c_int32), ("adi_rotations", C.c_int32),
    ]

    def to_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "res_hist"}
        d["res_hist"] = [self.res_hist[i] for i in range(self.hist_len)]
        return d


class care_instance(C.Structure):
    _fields_ = [("A", C.POINTER(care_csr)), ("A_dense", C.c_void_p), ("n_dense", C.c_int64),
                ("lda_dense", C.c_int64), ("B", C.c_void_p), ("m", C.c_int32), ("C", C.c_void_p),
                ("p", C.c_int32), ("shifts", C.POINTER(care_shift)), ("nshifts", C.c_int32),
                ("Z", C.c_void_p), ("ldz", C.c_int64), ("rmax", C.c_int32)]


class care_instance_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("r", C.c_int32), ("stats", care_stats), ("message", C.c_char * 128)]


P = C.c_void_p
I32, I64, DBL = C.c_int32, C.c_int64, C.c_double
PI32 = C.POINTER(C.c_int32)
PDBL = C.POINTER(C.c_double)

# device-memory hooks of care_ctx_create
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
DEALLOC_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)

SIGNATURES = {
    "care_ctx_create": (I32, [C.POINTER(P), I32, P, ALLOC_FN, DEALLOC_FN, P]),
    "care_ctx_destroy": (None, [P]),
    "care_opts_default": (None, [C.POINTER(care_opts), I32]),
    "care_last_error": (C.c_char_p, []),
    "care_version": (C.c_char_p, []),
    "care_struct_sizes": (I32, [C.POINTER(I64), I32]),
    "care_spmm": (I32, [P, C.POINTER(care_csr), I32, care_shift, P, I64, I32, P, I64]),
    "care_spmm_timing": (I32, [P, C.POINTER(care_csr), I32, care_shift, I32, I32, I32, I32, I32, PDBL, PDBL]),
    "care_shifted_solve": (I32, [P, C.POINTER(care_csr), P, I64, P, I64, I32, care_shift, P, I64, I32, I32, DBL,
                                 I32, P, I64, PI32]),
    "care_shifted_solve_opts": (I32, [P, C.POINTER(care_csr), P, I64, P, I64, I32, care_shift, P, I64, I32, I32,
                                      DBL, I32, C.POINTER(care_opts), P, I64, PI32]),
    "care_ilu0_colouring": (I32, [I64, I64, PI32, PI32, PI32, PI32]),
    "care_ilu0_factor": (I32, [P, C.POINTER(care_csr), I32, DBL, PI32, PDBL, I64, PDBL]),
    "care_ilu0_apply": (I32, [P, C.POINTER(care_csr), I32, DBL, P, I64, I32, P, I64]),
    "care_gram": (I32, [P, I64, P, I64, I32, P, I64, I32, P, I64]),
    "care_gram_noalloc": (I32, [P, I64, P, I64, I32, P, I64, I32, P, I64]),
    "care_tsgemm": (I32, [P, I64, P, I64, I32, P, I64, I32, DBL, DBL, P, I64]),
    "lyap_lradi": (I32, [P, C.POINTER(care_csr), P, P, I32, P, I64, I32, C.POINTER(care_shift), I32, DBL,
                         C.POINTER(care_opts), P, I64, I32, PI32, C.POINTER(care_stats)]),
    "care_residual_factor": (I32, [P, C.POINTER(care_csr), P, I32, P, I32, P, I64, I32, DBL, P, PI32, P, PI32,
                                   I64, I32, PDBL]),
    "lowrank_truncate": (I32, [P, I64, P, I64, I32, C.POINTER(C.c_int8), DBL, P, I64, I32, PI32, PDBL]),
    "care_solve": (I32, [P, C.POINTER(care_csr), P, I32, P, I32, DBL, C.POINTER(care_shift), I32,
                         C.POINTER(care_opts), P, I64, I32, PI32, C.POINTER(care_stats)]),
    "care_penzl_shifts": (I32, [P, C.POINTER(care_csr), I32, I32, I32, I32, C.POINTER(care_shift), PI32]),
    "care_solve_dense": (I32, [P, P, I64, I64, P, I32, P, I32, DBL, C.POINTER(care_shift), I32,
                               C.POINTER(care_opts), P, I64, I32, PI32, C.POINTER(care_stats)]),
    "care_solve_batch": (I32, [P, I32, C.POINTER(care_instance), DBL, C.POINTER(care_opts), I32,
                               C.POINTER(care_instance_result)]),
    "care_projection_shifts": (I32, [P, C.POINTER(care_csr), P, P, I32, P, I64, I32, I32, I32,
                                     C.POINTER(care_shift), PI32]),
    "care_shifted_lu_factor": (I32, [P, I32, I64, P, PDBL, I32, P, P, PI32]),
    "care_shifted_lu_solve": (I32, [P, I32, I64, P, P, I32, P, I64, P, I64]),
    "care_ritz_values": (I32, [PDBL, I32, I64, PDBL, PDBL]),
    "care_penzl_select": (I32, [PDBL, PDBL, I32, I32, C.POINTER(care_shift), PI32]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libmpcare.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first "
                           "(python -m paper_2607_14742_amd.build)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
