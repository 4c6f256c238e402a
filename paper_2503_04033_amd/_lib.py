"""ctypes binding of libhps_leaf.so (include/hps_leaf.h).  Marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhps_leaf.so")

HPS_OK, HPS_EINVAL, HPS_ENOMEM, HPS_EDEVICE, HPS_EUNSUPPORTED = 0, -1, -2, -3, -4
HPS_FP64, HPS_FP32_IR = 0, 1

# every symbol include/hps_leaf.h declares
EXPORTS = (
    "hps_plan_create", "hps_plan_destroy", "hps_plan_get_info", "hps_leaf_nodes", "hps_leaf_operators",
    "hps_leaf_factor", "hps_leaf_dtn", "hps_interface_reduce", "hps_leaf_reconstruct", "hps_leaf_adjoint_solve",
    "hps_leaf_adjoint_grad", "hps_status_string", "hps_plan_profile_enable", "hps_plan_profile_read",
    "hps_leaf_interior_solve", "hps_leaf_flux", "hps_plan_set_tuning", "hps_plan_get_tuning",
    "hps_leaf_interior_solve_noalloc", "hps_front_plan_create", "hps_front_plan_destroy", "hps_front_dinv_elems",
    "hps_front_init", "hps_front_block_add", "hps_front_segments", "hps_front_factor", "hps_front_solve",
    "hps_leaf_cn_rhs", "hps_leaf_workspace_bytes",
)

# hps_call: the calls whose workspace hps_leaf_workspace_bytes sizes
CALLS = {"dtn": 0, "interior_solve": 1, "adjoint_solve": 2}

# HPS_NOALLOC_SCRATCH_BYTES: the fixed scratch of hps_leaf_interior_solve_noalloc
NOALLOC_SCRATCH_BYTES = 32 << 20

HPS_TUNE_TRSM_SCHEDULE, HPS_TUNE_TRSM_WAVES, HPS_TUNE_RESIDUAL_COLS, HPS_TUNE_PANEL_THREADS = 0, 1, 2, 3
TUNING_KEYS = {"trsm_schedule": HPS_TUNE_TRSM_SCHEDULE, "trsm_waves": HPS_TUNE_TRSM_WAVES,
               "residual_cols": HPS_TUNE_RESIDUAL_COLS, "panel_threads": HPS_TUNE_PANEL_THREADS}

PROFILE_FAMILIES = ("lu_gemm", "lu_panel", "lu_leaf", "solve_fwd", "solve_bwd", "residual", "dtn", "operators")


class LeafDesc(C.Structure):
    _fields_ = [("p", C.c_int32), ("h", C.c_double * 3), ("kappa", C.c_double), ("precision", C.c_int32),
                ("ir_max_iter", C.c_int32), ("ir_tol", C.c_double)]


class PlanInfo(C.Structure):
    _fields_ = [("m", C.c_int32), ("n_i", C.c_int32), ("n_b", C.c_int32), ("n_pad", C.c_int32),
                ("nrhs", C.c_int32), ("ldx", C.c_int32), ("npanel", C.c_int32), ("elem_bytes", C.c_int32),
                ("a_bytes", C.c_size_t), ("perm_bytes", C.c_size_t), ("dinv_bytes", C.c_size_t),
                ("x_bytes", C.c_size_t), ("ws_bytes", C.c_size_t)]


class Profile(C.Structure):
    _fields_ = [("launches", C.c_int64 * 8), ("ms", C.c_double * 8), ("flops", C.c_double * 8),
                ("exec_flops", C.c_double * 8)]


class HpsError(RuntimeError):
    pass


_lib = None


def load() -> C.CDLL:
    """Load the HIP library; raise if it was not built (there is no CPU fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not found: build it with `python -m paper_2503_04033_amd.build` "
                          "(the leaf reduction has no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, SZ, D = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t, C.c_double
    sig = {
        "hps_plan_create": [C.POINTER(P), C.POINTER(LeafDesc)],
        "hps_plan_destroy": [P],
        "hps_plan_get_info": [P, C.POINTER(PlanInfo)],
        "hps_leaf_nodes": [P, I32, P, P, P, P],
        "hps_leaf_operators": [P, I32, P, P, P, P],
        "hps_leaf_factor": [P, I32, P, P, P, P, P],
        "hps_leaf_dtn": [P, I32, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P],
        "hps_interface_reduce": [I32, P, I64, P, P],
        "hps_leaf_reconstruct": [P, I32, P, P, P, P],
        "hps_leaf_adjoint_solve": [P, I32, P, P, P, P, P, P, P, P, P, P],
        "hps_leaf_adjoint_grad": [P, I32, P, P, P, P],
        "hps_leaf_interior_solve": [P, I32, P, P, P, P, P, P, P, P, I32, P, P, P],
        "hps_leaf_interior_solve_noalloc": [P, I32, P, P, P, P, P, P, P, P, I32, P, P],
        "hps_leaf_flux": [P, I32, P, P, P, P],
        "hps_plan_profile_enable": [P, I32],
        "hps_plan_profile_read": [P, C.POINTER(Profile)],
        "hps_plan_set_tuning": [P, I32, I32],
        "hps_plan_get_tuning": [P, I32, C.POINTER(C.c_int32)],
        "hps_leaf_workspace_bytes": [P, I32, I32, C.POINTER(SZ)],
        "hps_leaf_cn_rhs": [P, I32, P, D, P, P, P, P],
        "hps_front_plan_create": [C.POINTER(P), I32, I32],
        "hps_front_plan_destroy": [P],
        "hps_front_init": [I32, I32, I32, I32, I32, I32, P, P],
        "hps_front_block_add": [I32, P, I32, P, P, P],
        "hps_front_segments": [I32, P, I32, P, P, I32, P],
        "hps_front_factor": [P, I32, P, P, P, P, P],
        "hps_front_solve": [P, I32, P, P, P, P, I32, P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.hps_front_dinv_elems.argtypes = [P]
    lib.hps_front_dinv_elems.restype = SZ
    lib.hps_status_string.argtypes = [C.c_int]
    lib.hps_status_string.restype = C.c_char_p
    _lib = lib
    return lib


def check(status: int, what: str) -> None:
    if status != HPS_OK:
        msg = load().hps_status_string(status).decode()
        raise HpsError(f"{what} failed: {msg} ({status})")
