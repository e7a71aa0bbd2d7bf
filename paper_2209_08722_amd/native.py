"""ctypes binding of libipmsk.so (the C ABI declared in include/ipmsk.h).

Argument marshalling only: every computation runs in the library's HIP kernels. Device
memory comes from torch tensors on a ROCm device; the library orders its work on the
tensor device's current torch stream.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_int32, c_int64, c_uint64, c_void_p

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libipmsk.so")

# status codes (include/ipmsk.h)
IPM_OK = 0
IPM_CONVERGED = 1
IPM_PCG_MAXIT = 2
IPM_PCG_STAGNATED = 3
IPM_ERR_ARG = -1
IPM_ERR_HIP = -2
IPM_ERR_NOT_SPD = -3
IPM_ERR_BREAKDOWN = -4
IPM_ERR_STALL = -5
IPM_ERR_NOMEM = -6

IPM_F64, IPM_F32, IPM_BF16 = 0, 1, 2
IPM_DENSE_ROWMAJOR, IPM_CSR = 0, 1
IPM_KERNEL_MATVEC, IPM_KERNEL_SKETCH, IPM_KERNEL_GRAM, IPM_KERNEL_MATVEC32, IPM_KERNEL_RESID64 = 0, 1, 2, 3, 4
IPM_KERNEL_STREAM_READ, IPM_KERNEL_STREAM_COPY, IPM_KERNEL_WARM = 5, 6, 7
IPM_PLAIN, IPM_MIXED, IPM_MIXED_F32ACC = 0, 1, 2
IPM_WARM_NONE, IPM_WARM_PREV, IPM_WARM_GIVEN = 0, 1, 2

STATUS_NAMES = {
    IPM_OK: "IPM_OK", IPM_CONVERGED: "IPM_CONVERGED", IPM_PCG_MAXIT: "IPM_PCG_MAXIT",
    IPM_PCG_STAGNATED: "IPM_PCG_STAGNATED", IPM_ERR_ARG: "IPM_ERR_ARG", IPM_ERR_HIP: "IPM_ERR_HIP",
    IPM_ERR_NOT_SPD: "IPM_ERR_NOT_SPD", IPM_ERR_BREAKDOWN: "IPM_ERR_BREAKDOWN",
    IPM_ERR_STALL: "IPM_ERR_STALL", IPM_ERR_NOMEM: "IPM_ERR_NOMEM",
}


class IpmMatrix(ctypes.Structure):
    _fields_ = [("m", c_int64), ("n", c_int64), ("ld", c_int64), ("layout", c_int32),
                ("dtype", c_int32), ("val", c_void_p), ("nnz", c_int64), ("row_ptr", c_void_p),
                ("col_idx", c_void_p), ("csc_val", c_void_p), ("col_ptr", c_void_p), ("row_idx", c_void_p)]


class IpmProblem(ctypes.Structure):
    _fields_ = [("A", IpmMatrix), ("b", c_void_p), ("c", c_void_p)]


class IpmState(ctypes.Structure):
    _fields_ = [("x", c_void_p), ("y", c_void_p), ("s", c_void_p), ("k", c_int64),
                ("mu0", c_double), ("r0norm", c_double)]


class IpmParams(ctypes.Structure):
    _fields_ = [("sigma", c_double), ("gamma", c_double), ("theta", c_double), ("tol_pcg", c_double),
                ("gap_tol", c_double), ("min_step", c_double), ("stag_ratio", c_double),
                ("w", c_int32), ("s", c_int32), ("maxit_pcg", c_int32), ("stag_window", c_int32),
                ("max_redraws", c_int32), ("vcorr", c_int32), ("precision", c_int32), ("warm_start", c_int32),
                ("inner_tol", c_double), ("max_refine", c_int32), ("max_shifts", c_int32), ("feasible", c_int32),
                ("solver", c_int32), ("sketch", c_int32), ("reserved", c_int32), ("seed", c_uint64)]


class IpmPcgInfo(ctypes.Structure):
    _fields_ = [("iters", c_int32), ("status", c_int32), ("warm_used", c_int32), ("rounds", c_int32),
                ("relres", c_double), ("rho_star", c_double)]


class IpmStepInfo(ctypes.Structure):
    _fields_ = [("status", c_int32), ("pcg_status", c_int32), ("pcg_iters", c_int32), ("attempts", c_int32),
                ("k", c_int64), ("w_used", c_int32), ("s_used", c_int32),
                ("mu", c_double), ("gap", c_double), ("relgap", c_double), ("rp_rel", c_double),
                ("rd_rel", c_double), ("obj", c_double), ("alpha_max", c_double), ("alpha", c_double),
                ("pcg_relres", c_double), ("vnorm", c_double), ("refine_rounds", c_int32), ("warm_used", c_int32),
                ("dy_norm", c_double), ("shift", c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class IpmMlp(ctypes.Structure):
    _fields_ = [("n_in", c_int32), ("n_hidden", c_int32), ("n_out", c_int32), ("reserved", c_int32),
                ("params", c_void_p)]


# (name, restype, argtypes) of every exported function
SIGNATURES = [
    ("ipm_ctx_create", c_int, [POINTER(c_void_p), c_int, c_void_p]),
    ("ipm_ctx_destroy", None, [c_void_p]),
    ("ipm_ctx_set_stream", c_int, [c_void_p, c_void_p]),
    ("ipm_last_error", ctypes.c_char_p, [c_void_p]),
    ("ipm_params_default", None, [POINTER(IpmParams)]),
    ("ipm_sketch", c_int, [c_void_p, POINTER(IpmMatrix), c_void_p, c_uint64, c_int64, c_int32, c_int32,
                           c_int32, c_void_p]),
    ("ipm_sketch_gaussian", c_int, [c_void_p, POINTER(IpmMatrix), c_void_p, c_uint64, c_int64, c_int32,
                                    c_void_p]),
    ("ipm_precond_factor", c_int, [c_void_p, c_int64, c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                   POINTER(c_int64)]),
    ("ipm_pcg_solve", c_int, [c_void_p, POINTER(IpmMatrix), c_void_p, c_void_p, c_void_p, c_void_p, c_int32,
                              POINTER(IpmParams), POINTER(IpmPcgInfo)]),
    ("ipm_step", c_int, [c_void_p, POINTER(IpmProblem), POINTER(IpmState), POINTER(IpmParams),
                         POINTER(IpmStepInfo)]),
    ("ipm_step_warm", c_int, [c_void_p, POINTER(IpmProblem), POINTER(IpmState), POINTER(IpmParams), c_void_p,
                              c_int32, POINTER(IpmStepInfo)]),
    ("ipm_last_dy", c_int, [c_void_p, c_int64, c_void_p]),
    ("ipm_normal_matvec", c_int, [c_void_p, POINTER(IpmMatrix), c_void_p, c_void_p, c_void_p]),
    ("ipm_normal_matvec_noalloc", c_int, [c_void_p, POINTER(IpmMatrix), c_void_p, c_void_p, c_void_p]),
    ("ipm_stream_read", c_int, [c_void_p, c_void_p, c_int64, c_void_p]),
    ("ipm_stream_copy", c_int, [c_void_p, c_void_p, c_void_p, c_int64]),
    ("ipm_mlp_param_count", c_int64, [c_int32, c_int32, c_int32]),
    ("ipm_mlp_features", c_int, [c_void_p, c_int64, c_int64, c_void_p, c_void_p, c_void_p, c_int64, c_int64,
                                 c_void_p]),
    ("ipm_mlp_target", c_int, [c_void_p, c_int64, c_void_p, c_void_p, c_void_p]),
    ("ipm_mlp_forward", c_int, [c_void_p, POINTER(IpmMlp), c_int32, c_void_p, c_void_p]),
    ("ipm_mlp_backward", c_int, [c_void_p, POINTER(IpmMlp), c_int32, c_void_p, c_void_p, c_void_p,
                                 POINTER(c_double)]),
    ("ipm_mlp_adam", c_int, [c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_double,
                             c_double, c_double, c_double]),
    ("ipm_mlp_predict", c_int, [c_void_p, POINTER(IpmMlp), c_int64, c_void_p, c_void_p, c_void_p, c_int64,
                                c_int64, c_void_p]),
    ("ipm_ctx_set_timing", c_int, [c_void_p, c_int32]),
    ("ipm_kernel_time", c_int, [c_void_p, c_int32, POINTER(c_double), POINTER(c_int64)]),
]

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the HIP library; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2209_08722_amd.build (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
