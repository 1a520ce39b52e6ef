"""ctypes declarations of the C ABI in include/sam.h (argument marshalling
only).  Loading fails loudly when the HIP library has not been built: there
is no fallback implementation."""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
# SAM_MI355X_LIB: another build of the library (the host-sanitizer build)
LIB_PATH = os.environ.get("SAM_MI355X_LIB") or os.path.join(HERE, "libsam_mi355x.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "sam.h")

c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_double = ctypes.c_double
c_void_p = ctypes.c_void_p
c_char_p = ctypes.c_char_p
P = c_void_p

SAM_OK = 0
(SAM_ERR_ARG, SAM_ERR_SHAPE, SAM_ERR_UNSORTED, SAM_ERR_OVERFLOW, SAM_ERR_RANK, SAM_ERR_NONFINITE, SAM_ERR_HIP,
 SAM_ERR_UNSUPPORTED, SAM_ERR_NOMEM) = range(1, 10)
STATUS_NAMES = {
    0: "SAM_OK", 1: "SAM_ERR_ARG", 2: "SAM_ERR_SHAPE", 3: "SAM_ERR_UNSORTED",
    4: "SAM_ERR_OVERFLOW", 5: "SAM_ERR_RANK", 6: "SAM_ERR_NONFINITE", 7: "SAM_ERR_HIP",
    8: "SAM_ERR_UNSUPPORTED", 9: "SAM_ERR_NOMEM",
}
SAM_PREC_F64 = 0
SAM_PREC_F32_REFINE = 1
SAM_NO_DEVICE = -1
SPARSIFY = {"none": 0, "global": 1, "column": 2, "lfil": 3}


class sam_csc(ctypes.Structure):
    _fields_ = [("n", c_int32), ("nnz", c_int32), ("colptr", c_void_p), ("rowind", c_void_p),
                ("val", c_void_p)]


class sam_pattern_spec(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("power", c_int32), ("thresh", c_double),
                ("global_scale", c_int32), ("tau", c_double), ("lfil", c_int32)]


CSCP = ctypes.POINTER(sam_csc)
SPECP = ctypes.POINTER(sam_pattern_spec)

# name -> (restype, argtypes)
SZ = ctypes.POINTER(ctypes.c_size_t)
c_size_t = ctypes.c_size_t

SIGNATURES = {
    "sam_create": (c_int32, [ctypes.POINTER(c_void_p), c_int32]),
    "sam_destroy": (c_int32, [P]),
    "sam_last_error": (c_char_p, [P]),
    "sam_status_string": (c_char_p, [c_int32]),
    "sam_version": (c_char_p, []),
    "sam_sync_status": (c_int32, [P, P, ctypes.POINTER(c_int32)]),
    "sam_check_csc": (c_int32, [P, CSCP, P]),
    "sam_pattern_workspace_size": (c_int32, [P, CSCP, SPECP, SZ, P]),
    "sam_pattern_count": (c_int32, [P, CSCP, SPECP, P, c_size_t, ctypes.POINTER(c_int64), P]),
    "sam_pattern_fill": (c_int32, [P, CSCP, SPECP, P, c_size_t, P, P, P]),
    "sam_plan_size": (c_int32, [P, CSCP, CSCP, P, P, c_int64, SZ, P]),
    "sam_plan_create": (c_int32, [P, CSCP, CSCP, P, P, c_int64, P, c_size_t, ctypes.POINTER(c_void_p), P]),
    "sam_plan_destroy": (c_int32, [P]),
    "sam_plan_info": (c_int32, [P, ctypes.POINTER(c_int32), ctypes.POINTER(c_int32),
                                ctypes.POINTER(c_int32), ctypes.POINTER(c_int64),
                                ctypes.POINTER(c_int32), ctypes.POINTER(c_int32)]),
    "sam_plan_cost": (c_int32, [P, c_int32, ctypes.POINTER(c_double), ctypes.POINTER(c_double),
                                ctypes.POINTER(c_double)]),
    "sam_plan_cost_weighted": (c_int32, [P, c_int32, c_int32, ctypes.POINTER(c_double), ctypes.POINTER(c_double)]),
    "sam_menu": (c_int32, [c_int32, c_int32, c_int32, ctypes.POINTER(c_int32), P, P, P, P]),
    "sam_plan_select": (c_int32, [P, c_int32, P, c_int32, P]),
    "sam_sequence_select": (c_int32, [P, P, c_int32, P]),
    "sam_build_planned": (c_int32, [P, P, P, c_int32, P, P, P, P]),
    "sam_workspace_size": (c_int32, [P, CSCP, CSCP, P, P, c_int64, c_int32, SZ, P]),
    "sam_build": (c_int32, [P, CSCP, CSCP, P, P, c_int64, c_int32, P, P, P, P, c_size_t, P]),
    "sam_build_noalloc": (c_int32, [P, CSCP, CSCP, P, P, c_int64, c_int32, P, P, P, P]),
    "sam_residual_workspace_size": (c_int32, [c_int32, c_int32, SZ]),
    "sam_residual": (c_int32, [P, CSCP, CSCP, P, P, c_int64, P, c_int32, P, P, P, c_size_t, P]),
    "sam_apply_workspace_size": (c_int32, [c_int32, SZ]),
    "sam_apply_prepare": (c_int32, [P, c_int32, P, P, c_int64, P, P, P, P, c_size_t, P]),
    "sam_apply": (c_int32, [P, c_int32, P, P, P, P, c_int32, P, P, P]),
    "sam_apply_permute": (c_int32, [P, c_int64, P, P, c_int32, P, P]),
    "sam_sequence_size": (c_int32, [P, CSCP, CSCP, SPECP, c_int32, c_int32, c_int32, P, c_size_t, SZ, P]),
    "sam_sequence_create": (c_int32, [P, CSCP, CSCP, SPECP, c_int32, c_int32, c_int32, P, c_size_t,
                                      ctypes.POINTER(c_void_p), P]),
    "sam_sequence_destroy": (c_int32, [P]),
    "sam_sequence_info": (c_int32, [P, ctypes.POINTER(c_int64)]),
    "sam_sequence_pattern": (c_int32, [P, c_int32, P, P, ctypes.POINTER(c_int64), P]),
    "sam_sequence_run": (c_int32, [P, P, P, P, P]),
    "sam_build_weighted": (c_int32, [P, P, P, P, c_double, c_int32, P, P, P, P]),
    "sam_backward_workspace_size": (c_int32, [P, SZ]),
    "sam_backward_prepare": (c_int32, [P, P, c_size_t, P]),
    "sam_backward": (c_int32, [P, P, P, P, c_double, c_double, c_int32, P, P, P, P, P, c_size_t, P]),
    "sam_candidate_weights": (c_int32, [P, c_int32, P, P, c_int64, P, P, c_int64, c_double, c_double, P, P]),
    "sam_topk_workspace_size": (c_int32, [c_int32, SZ]),
    "sam_pattern_topk": (c_int32, [P, c_int32, P, P, c_int64, P, P, c_int32, P, P, ctypes.POINTER(c_int64),
                                   P, c_size_t, P]),
    "sam_penalty_workspace_size": (c_int32, [c_int32, SZ]),
    "sam_penalty_scale": (c_int32, [P, CSCP, ctypes.POINTER(c_double), P, c_size_t, P]),
}


def header_symbols(path: str = HEADER) -> list[str]:
    """Function names declared in include/sam.h."""
    text = open(path).read()
    return sorted(set(re.findall(r"^\s*(?:sam_status|const char\s*\*)\s*(sam_\w+)\s*\(", text, re.M)))


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python paper_2406_17656_amd/build_lib.py or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib
