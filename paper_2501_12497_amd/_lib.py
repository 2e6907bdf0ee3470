"""ctypes declarations of libmmof.so (the C ABI in include/mmof.h).

Loading fails loudly when the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmmof.so")

MMOF_F32, MMOF_F64 = 0, 1
MMOF_FLOW_FWD, MMOF_FLOW_ADJ, MMOF_FLOW_DV = 0, 1, 2
MMOF_INTERP_BILINEAR, MMOF_INTERP_ROUND = 0, 1
MMOF_FLOW_SCALE_AUTO = -1
MMOF_FLOW_HS, MMOF_FLOW_GKS = 0, 1
STATUS = {0: "OK", -1: "MMOF_ERR_INVALID", -2: "MMOF_ERR_SHAPE", -3: "MMOF_ERR_DTYPE", -4: "MMOF_ERR_HIP",
          -5: "MMOF_ERR_OOM", -6: "MMOF_ERR_NONFINITE", 1: "MMOF_WARN_KMAX", 2: "MMOF_WARN_DP_CLAMPED",
          3: "MMOF_WARN_BREAKDOWN"}


class mmof_stack(C.Structure):
    _fields_ = [("n_seq", C.c_int32), ("n_t", C.POINTER(C.c_int32)), ("ny", C.POINTER(C.c_int32)),
                ("nx", C.POINTER(C.c_int32))]


MMOF_REG_PSI, MMOF_REG_ANISO, MMOF_REG_ISO, MMOF_REG_GS = 0, 1, 2, 3
REGS = {"psi": MMOF_REG_PSI, "aniso": MMOF_REG_ANISO, "iso": MMOF_REG_ISO, "gs": MMOF_REG_GS}
MMOF_REORTH_AUTO, MMOF_REORTH_TWICE, MMOF_REORTH_IMPLICIT = 0, 1, 2
REORTHS = {"auto": MMOF_REORTH_AUTO, "twice": MMOF_REORTH_TWICE, "implicit": MMOF_REORTH_IMPLICIT}


class mmof_solve_params(C.Structure):
    _fields_ = [("ell", C.c_int32), ("k_max", C.c_int32), ("tau", C.c_int32), ("n_sweeps", C.c_int32),
                ("delta_r", C.c_int32), ("use_flow", C.c_int32), ("use_reverse", C.c_int32),
                ("interp", C.c_int32), ("op_dtype", C.c_int32), ("refine_iters", C.c_int32),
                ("eps", C.c_double), ("eta", C.c_double), ("alpha", C.c_double), ("fixed_lambda", C.c_double),
                ("rre_target", C.c_double), ("u_true", C.c_void_p), ("use_graph", C.c_int32),
                ("flow_scale", C.c_int32), ("flow_solver", C.c_int32), ("of_ell", C.c_int32),
                ("of_iters", C.c_int32), ("reg", C.c_int32), ("reorth", C.c_int32)]


class mmof_report(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("n_cols", C.c_int32), ("capacity", C.c_int32),
                ("lambda_", C.POINTER(C.c_double)), ("resid", C.POINTER(C.c_double)),
                ("rre", C.POINTER(C.c_double)), ("dp_status", C.POINTER(C.c_int32)),
                ("n_A", C.c_int64), ("n_At", C.c_int64), ("n_theta", C.c_int64), ("n_thetaT", C.c_int64),
                ("n_flow_updates", C.c_int64), ("n_L", C.c_int64),
                ("n_factorizations", C.c_int64)]


_P = C.c_void_p
_I = C.c_int
_SIGS = {
    "mmof_version": (C.c_char_p, []),
    "mmof_last_error": (C.c_char_p, [_P]),
    "mmof_create": (_I, [C.POINTER(_P), _P]),
    "mmof_destroy": (_I, [_P]),
    "mmof_set_stream": (_I, [_P, _P]),
    "mmof_plan_radon": (_I, [_P, C.POINTER(mmof_stack), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                             C.POINTER(C.c_double), C.POINTER(_P)]),
    "mmof_plan_fan": (_I, [_P, C.POINTER(mmof_stack), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                           C.POINTER(C.c_double), C.c_double, C.c_double, C.c_double, C.POINTER(_P)]),
    "mmof_plan_blur": (_I, [_P, C.POINTER(mmof_stack), C.c_int32, C.c_double, C.POINTER(_P)]),
    "mmof_plan_destroy": (_I, [_P]),
    "mmof_plan_sizes": (_I, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "mmof_apply_A": (_I, [_P, _I, _P, _P]),
    "mmof_apply_At": (_I, [_P, _I, _P, _P]),
    "mmof_apply_grad": (_I, [_P, C.POINTER(mmof_stack), _I, _I, _P, _P, _P, _P, _P]),
    "mmof_apply_flow_op": (_I, [_P, C.POINTER(mmof_stack), _I, _I, _I, _I, _P, _P, _P, _P]),
    "mmof_mm_weights": (_I, [_P, _I, C.c_int64, _P, C.c_double, _P]),
    "mmof_of_derivs": (_I, [_P, C.POINTER(mmof_stack), _I, _P, _P, C.c_int32]),
    "mmof_flow_update": (_I, [_P, C.POINTER(mmof_stack), _I, _P, _P, _P, C.c_double, C.c_int32, C.c_int32]),
    "mmof_flow_update_scaled": (_I, [_P, C.POINTER(mmof_stack), _I, _P, _P, _P, C.c_double, C.c_int32, C.c_int32,
                                     C.c_int32]),
    "mmof_flow_solve_gks": (_I, [_P, C.POINTER(mmof_stack), _I, _P, _P, _P, C.c_int32, C.c_int32, C.c_int32,
                                 C.c_double, C.c_int32, _P]),
    "mmof_flow_solve_of": (_I, [_P, C.POINTER(mmof_stack), _I, _P, _P, _P, C.c_int32, C.c_int32, C.c_int32,
                                C.c_double, C.c_int32, C.c_int32, C.c_double, _P]),
    "mmof_reverse_flow": (_I, [_P, C.POINTER(mmof_stack), _I, _P, _P]),
    "mmof_solve_defaults": (None, [C.POINTER(mmof_solve_params)]),
    "mmof_solve_joint": (_I, [_P, _P, C.c_double, C.POINTER(mmof_solve_params), _P, _P, _P,
                              C.POINTER(mmof_report)]),
    "mmof_weighted_gram": (_I, [_P, _I, C.c_int64, C.c_int32, _P, C.c_int64, _P, C.c_double, _P, C.c_int32]),
    "mmof_weighted_gram_noalloc": (_I, [_P, _I, C.c_int64, C.c_int32, _P, C.c_int64, _P, C.c_double, _P,
                                        C.c_int32]),
    "mmof_apply_tdiff": (_I, [_P, C.POINTER(mmof_stack), _I, _I, _P, _P]),
    "mmof_reg_weights": (_I, [_P, C.POINTER(mmof_stack), _I, _I, C.c_int64, _P, C.c_double, _P]),
    "mmof_block_dot": (_I, [_P, _I, C.c_int64, C.c_int32, _P, C.c_int64, _P, _P]),
    "mmof_block_combine": (_I, [_P, _I, C.c_int64, C.c_int32, _P, C.c_int64, _P, C.c_double, _P, C.c_double, _P]),
    "mmof_cgs2": (_I, [_P, C.c_int64, C.c_int32, _P, C.c_int64, _P, _P]),
    "mmof_reorth": (_I, [_P, C.c_int64, C.c_int32, _P, C.c_int64, _P, _P, C.c_int32]),
    "mmof_basis_extend": (_I, [_P, C.c_int64, C.c_int32, _P, C.c_int64, _P, _P, _P]),
    "mmof_projected_solve": (_I, [_P, C.c_int32, _P, _P, _P, _P, C.c_double, _P, _P]),
    "mmof_profile_kernel": (_I, [_P, C.c_char_p]),
    "mmof_autotune": (_I, [_P, C.c_int32, C.c_char_p, C.c_int32]),
    "mmof_set_tile": (_I, [_P, C.c_char_p, C.c_int32, C.c_int32]),
    "mmof_kernel_timing": (_I, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                C.POINTER(C.c_double)]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libmmof.so once; raise if it is missing (build it with paper_2501_12497_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build the HIP library first "
                          f"(python -m paper_2501_12497_amd.build)")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class MMOFError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def check(rc: int) -> int:
    if rc < 0:
        raise MMOFError(rc, load().mmof_last_error(None).decode())
    return rc
