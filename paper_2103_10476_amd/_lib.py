"""ctypes binding of libsaamg.so (the C ABI declared in include/saamg.h).

Argument marshalling only: every step of setup and solve runs in the library's HIP kernels.
Loading fails loudly when the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsaamg.so")

SA_OK, SA_NOT_CONVERGED, SA_PENDING = 0, 1, 2
STATUS_NAMES = {
    0: "SA_OK", 1: "SA_NOT_CONVERGED", 2: "SA_PENDING", -1: "SA_ERR_INVALID_ARG",
    -2: "SA_ERR_BAD_CSR", -3: "SA_ERR_NONPOSITIVE_DIAG", -4: "SA_ERR_NEGATIVE_EIGENVALUE",
    -5: "SA_ERR_COARSEN_STALLED", -6: "SA_ERR_COARSE_FACTOR", -7: "SA_ERR_OOM",
    -8: "SA_ERR_HIP", -9: "SA_ERR_BREAKDOWN",
}
SA_HOST, SA_DEVICE = 0, 1

PARTS = {"A_rp": 0, "A_col": 1, "A_val": 2, "mask": 3, "agg": 4, "root": 5, "Abar_rp": 6,
         "Abar_col": 7, "Abar_val": 8, "invD": 9, "P_rp": 10, "P_col": 11, "P_val": 12,
         "R_rp": 13, "R_col": 14, "R_val": 15, "sm_invD": 16, "coarse_inv": 17,
         "coords": 18, "Pt_rp": 19, "Pt_col": 20, "Pt_val": 21, "nullspace": 22,
         "node_mask": 23, "node_rp": 24, "node_col": 25}
PART_DTYPE = {"A_rp": "int32", "A_col": "int32", "A_val": "float64", "mask": "uint8",
              "agg": "int32", "root": "uint8", "Abar_rp": "int32", "Abar_col": "int32",
              "Abar_val": "float64", "invD": "float64", "P_rp": "int32", "P_col": "int32",
              "P_val": "float64", "R_rp": "int32", "R_col": "int32", "R_val": "float64",
              "sm_invD": "float64", "coarse_inv": "float64", "coords": "float64",
              "Pt_rp": "int32", "Pt_col": "int32", "Pt_val": "float64", "nullspace": "float64",
              "node_mask": "uint8", "node_rp": "int32", "node_col": "int32"}

EXPORTED = ["sa_default_options", "sa_setup", "sa_solve", "sa_vcycle", "sa_hierarchy_info",
            "sa_export_size", "sa_export_level", "sa_destroy", "sa_status_string",
            "sa_last_error", "sa_profile_enable", "sa_profile_read", "sa_estimate_bytes",
            "sa_solve_many", "sa_resetup", "sa_setup_coords", "sa_solve_gmres",
            "sa_solve_gmres_noalloc", "sa_setup_system",
            "sa_server_create", "sa_server_submit", "sa_server_submit_borrowed",
            "sa_server_poll", "sa_server_wait", "sa_server_drain", "sa_server_get_stats", "sa_server_destroy"]


class SaOptions(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("variants", C.c_uint32), ("theta", C.c_double),
                ("tau", C.c_double), ("sigma", C.c_double), ("one_norm_power", C.c_int32),
                ("power_iters", C.c_int32), ("seed", C.c_uint64), ("agg_order", C.c_int32),
                ("max_levels", C.c_int32), ("max_coarse", C.c_int32), ("smoother", C.c_int32),
                ("degree", C.c_int32), ("precision", C.c_int32), ("cheb_ratio", C.c_double),
                ("cheb_boost", C.c_double), ("rtol", C.c_double), ("max_iter", C.c_int32),
                ("pcg_beta", C.c_int32), ("dist_power", C.c_int32),
                ("coarse_solver", C.c_int32), ("isolated", C.c_int32)]


class SaCsr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p), ("loc", C.c_int32)]


class SaContext(C.Structure):
    _fields_ = [("stream", C.c_void_p)]


class SaInfo(C.Structure):
    _fields_ = [("levels", C.c_int32), ("n", C.c_int32 * 16), ("nnz", C.c_int64 * 16),
                ("nnz_p", C.c_int64 * 16), ("lambda_", C.c_double * 16),
                ("omega", C.c_double * 16), ("smoother_lambda", C.c_double * 16),
                ("mis_rounds", C.c_int32 * 16), ("operator_complexity", C.c_double),
                ("device_bytes", C.c_int64), ("setup_seconds", C.c_double)]


class SaResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("n", C.c_int32), ("iterations", C.c_int32),
                ("levels", C.c_int32), ("rel_residual", C.c_double),
                ("queue_seconds", C.c_double), ("setup_seconds", C.c_double),
                ("solve_seconds", C.c_double), ("latency_seconds", C.c_double),
                ("reserved_bytes", C.c_int64), ("peak_bytes", C.c_int64)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["status"] = STATUS_NAMES.get(self.status, str(self.status))
        return d


class SaServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("queued", C.c_int64), ("running", C.c_int64), ("budget_bytes", C.c_int64),
                ("reserved_bytes", C.c_int64), ("peak_reserved_bytes", C.c_int64),
                ("peak_measured_bytes", C.c_int64), ("solve_ticks", C.c_int64),
                ("mean_group", C.c_double), ("max_group", C.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


class LibraryMissing(RuntimeError):
    pass


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(
                f"{LIB_PATH} is not built; run __graft_entry__.build() "
                "(or python -m paper_2103_10476_amd.build)")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.sa_default_options.argtypes = [C.POINTER(SaOptions)]
        L.sa_setup.argtypes = [C.POINTER(SaContext), C.POINTER(SaCsr), P, C.POINTER(SaOptions),
                               C.POINTER(C.c_void_p)]
        L.sa_setup.restype = C.c_int
        L.sa_setup_coords.argtypes = [C.POINTER(SaContext), C.POINTER(SaCsr), P, P, C.c_int32,
                                      C.POINTER(SaOptions), C.POINTER(C.c_void_p)]
        L.sa_setup_coords.restype = C.c_int
        L.sa_setup_system.argtypes = [C.POINTER(SaContext), C.POINTER(SaCsr), C.c_int32, P,
                                      C.c_int32, P, C.c_int32, C.POINTER(SaOptions),
                                      C.POINTER(C.c_void_p)]
        L.sa_setup_system.restype = C.c_int
        L.sa_resetup.argtypes = [P, P, P, C.c_int32]
        L.sa_resetup.restype = C.c_int
        L.sa_solve.argtypes = [P, P, P, C.c_int32, C.POINTER(C.c_int32),
                               C.POINTER(C.c_double)]
        L.sa_solve.restype = C.c_int
        L.sa_solve_gmres.argtypes = [P, P, P, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                                     C.POINTER(C.c_double)]
        L.sa_solve_gmres.restype = C.c_int
        L.sa_solve_gmres_noalloc.argtypes = [P, P, P, C.c_int32, C.c_int32,
                                             C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        L.sa_solve_gmres_noalloc.restype = C.c_int
        L.sa_solve_many.argtypes = [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p),
                                    C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_int32),
                                    C.POINTER(C.c_double), C.POINTER(C.c_int)]
        L.sa_solve_many.restype = C.c_int
        L.sa_vcycle.argtypes = [P, P, P]
        L.sa_vcycle.restype = C.c_int
        L.sa_hierarchy_info.argtypes = [P, C.POINTER(SaInfo)]
        L.sa_hierarchy_info.restype = C.c_int
        L.sa_export_size.argtypes = [P, C.c_int32, C.c_int32, C.POINTER(C.c_int64)]
        L.sa_export_size.restype = C.c_int
        L.sa_export_level.argtypes = [P, C.c_int32, C.c_int32, P, C.c_size_t]
        L.sa_export_level.restype = C.c_int
        L.sa_profile_enable.argtypes = [P, C.c_int32]
        L.sa_profile_enable.restype = C.c_int
        L.sa_profile_read.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double)]
        L.sa_profile_read.restype = C.c_int
        L.sa_estimate_bytes.argtypes = [C.c_int32, C.c_int64]
        L.sa_estimate_bytes.restype = C.c_int64
        L.sa_server_create.argtypes = [C.POINTER(SaContext), C.c_size_t, C.c_int32,
                                       C.POINTER(C.c_void_p)]
        L.sa_server_create.restype = C.c_int
        for f in (L.sa_server_submit, L.sa_server_submit_borrowed):
            f.argtypes = [P, C.POINTER(SaCsr), P, C.POINTER(SaOptions), C.POINTER(C.c_uint64)]
            f.restype = C.c_int
        for f in (L.sa_server_poll, L.sa_server_wait):
            f.argtypes = [P, C.c_uint64, P, C.c_int32, C.POINTER(SaResult)]
            f.restype = C.c_int
        L.sa_server_drain.argtypes = [P]
        L.sa_server_drain.restype = C.c_int
        L.sa_server_get_stats.argtypes = [P, C.POINTER(SaServerStats)]
        L.sa_server_get_stats.restype = C.c_int
        L.sa_server_destroy.argtypes = [P]
        L.sa_server_destroy.restype = None
        L.sa_destroy.argtypes = [P]
        L.sa_destroy.restype = None
        L.sa_status_string.argtypes = [C.c_int]
        L.sa_status_string.restype = C.c_char_p
        L.sa_last_error.restype = C.c_char_p
        _lib = L
    return _lib


class SaError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib().sa_last_error().decode()
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)} ({msg})")
        self.code = code
        self.status = STATUS_NAMES.get(code, str(code))


def check(code: int, where: str) -> int:
    if code < 0:
        raise SaError(code, where)
    return code
