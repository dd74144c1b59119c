"""ctypes declarations for libshipwave.so (argument marshalling only).

The structures mirror include/shipwave.h field for field.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SHIPWAVE_LIB") or os.path.join(HERE, "libshipwave.so")


class SwMesh(C.Structure):
    _fields_ = [("N", C.c_int32), ("M", C.c_int32)]


class SwDomain(C.Structure):
    _fields_ = [("x1", C.c_double), ("xN", C.c_double), ("yM", C.c_double)]


class SwParams(C.Structure):
    _fields_ = [("F", C.c_double), ("eps", C.c_double), ("nu", C.c_double),
                ("weights", C.c_int32), ("spline_bc", C.c_int32), ("precision", C.c_int32),
                ("reserved", C.c_int32)]


class SwProblem(C.Structure):
    _fields_ = [("mesh", SwMesh), ("domain", SwDomain), ("params", SwParams)]


class SwSolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_newton", C.c_int32), ("gmres_restart", C.c_int32),
                ("max_gmres", C.c_int32), ("q_blocks", C.c_int32), ("precision", C.c_int32),
                ("weights", C.c_int32), ("spline_bc", C.c_int32), ("init", C.c_int32),
                ("nu", C.c_double), ("eta_max", C.c_double), ("precond", C.c_void_p)]


class SwSolveInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("newton_iters", C.c_int32), ("gmres_iters", C.c_int32),
                ("residual_evals", C.c_int32), ("final_norm", C.c_double),
                ("time_total_s", C.c_double), ("time_precond_s", C.c_double),
                ("fp32_error", C.c_double), ("linesearch_backtracks", C.c_int32),
                ("reserved", C.c_int32)]


class SwServerOpts(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_double), ("max_slots", C.c_int32),
                ("fallback_fp64", C.c_int32), ("tol", C.c_double), ("q_blocks", C.c_int32),
                ("precision", C.c_int32)]


class SwRequest(C.Structure):
    _fields_ = [("mesh", SwMesh), ("domain", SwDomain), ("F", C.c_double), ("eps", C.c_double)]


class SwResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("newton_iters", C.c_int32), ("gmres_iters", C.c_int32),
                ("residual_evals", C.c_int32), ("used_fallback", C.c_int32),
                ("final_norm", C.c_double), ("t_submit_s", C.c_double),
                ("t_admit_s", C.c_double), ("t_done_s", C.c_double),
                ("fp32_error", C.c_double)]


P = C.c_void_p
I32 = C.c_int32
D = C.c_double

# name -> (restype, argtypes); every symbol declared in include/shipwave.h
SIGNATURES = {
    "shipwave_abi_version": (I32, []),
    "shipwave_last_error": (C.c_char_p, []),
    "shipwave_residual": (I32, [C.POINTER(SwProblem), P, P, P]),
    "shipwave_residual_batched": (I32, [I32, C.POINTER(SwProblem), C.POINTER(P), C.POINTER(P),
                                        P]),
    "shipwave_residual_noalloc": (I32, [C.POINTER(SwProblem), P, P, P]),
    "shipwave_jvp": (I32, [C.POINTER(SwProblem), P, P, P, D, P, P]),
    "shipwave_precond_build_banded": (I32, [C.POINTER(SwProblem), I32, C.POINTER(P), P]),
    "shipwave_precond_apply": (I32, [P, P, P, P]),
    "shipwave_precond_apply_batched": (I32, [I32, C.POINTER(P), C.POINTER(P), C.POINTER(P), P]),
    "shipwave_precond_destroy": (None, [P]),
    "shipwave_solve_opts_default": (None, [C.POINTER(SwSolveOpts)]),
    "shipwave_solve": (I32, [D, D, C.POINTER(SwMesh), C.POINTER(SwDomain),
                             C.POINTER(SwSolveOpts), P, P, C.POINTER(SwSolveInfo), P]),
    "shipwave_zeta": (I32, [C.POINTER(SwProblem), P, P, P]),
    "shipwave_profile_enable": (I32, [I32]),
    "shipwave_profile_read": (I32, [C.POINTER(C.c_int64), C.POINTER(D), C.POINTER(D)]),
    "shipwave_debug_inject_nonfinite": (I32, [I32, I32]),
    "shipwave_server_create": (I32, [C.POINTER(SwServerOpts), C.POINTER(P)]),
    "shipwave_server_request_bytes": (I32, [C.POINTER(SwServerOpts), C.POINTER(SwRequest),
                                            C.POINTER(C.c_uint64)]),
    "shipwave_server_submit": (I32, [P, C.POINTER(SwRequest), C.POINTER(C.c_uint64)]),
    "shipwave_server_poll": (I32, [P, C.c_uint64, C.POINTER(SwResult), P]),
    "shipwave_server_drain": (I32, [P]),
    "shipwave_server_destroy": (None, [P]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with paper_1403_5044_amd.build.build()")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        if not hasattr(lib, name):
            continue  # reported by the ABI test; calling it raises AttributeError
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class ShipwaveError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"shipwave error {code}: {msg}")
        self.code = code


def check(code: int):
    if code != 0:
        msg = _lib.shipwave_last_error().decode(errors="replace") if _lib else ""
        raise ShipwaveError(code, msg)
    return code
