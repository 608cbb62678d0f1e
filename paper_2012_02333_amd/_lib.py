"""ctypes declarations of libcqc.so (include/cqc.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcqc.so")

CQC_OK = 0
STATUS = {0: "CQC_OK", 1: "CQC_ERR_INVALID_ARG", 2: "CQC_ERR_SHAPE", 3: "CQC_ERR_UNSUPPORTED",
          4: "CQC_ERR_WORKSPACE", 5: "CQC_ERR_HIP"}
F32, F64 = 0, 1
PREC = {"fp64": 0, "fp32": 1, "bf16x6": 2, "bf16x3": 3}
MAX_DD_QUBITS = 128

EXPORTS = [
    "cqc_fd_workspace_size", "cqc_reconstruct_fd", "cqc_dd_workspace_size", "cqc_reconstruct_dd",
    "cqc_backward_workspace_size", "cqc_reconstruct_backward", "cqc_cost", "cqc_autotune",
    "cqc_trace_enable", "cqc_trace_read", "cqc_status_string", "cqc_last_error_detail",
    "cqc_version", "cqc_selftest_mfma", "cqc_batch_create", "cqc_batch_run", "cqc_batch_destroy",
    "cqc_batch_backward_workspace_size", "cqc_batch_backward_create", "cqc_batch_backward_run",
    "cqc_batch_backward_destroy", "cqc_build_entries", "cqc_chi2", "cqc_xent_grad", "cqc_tune_reset",
    "cqc_reconstruct_fd_noalloc", "cqc_dd_query_workspace_size", "cqc_dd_query_create", "cqc_dd_query_run",
    "cqc_dd_query_destroy", "cqc_dd_query_run_range", "cqc_batch_create_xent",
]
NOALLOC_WORKSPACE_BYTES = 32 << 20


class CqcCut(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_sub", ctypes.c_int32), ("n_cuts", ctypes.c_int32),
                ("f", ctypes.POINTER(ctypes.c_int32)), ("edge_up", ctypes.POINTER(ctypes.c_int32)),
                ("edge_down", ctypes.POINTER(ctypes.c_int32)),
                ("out_qubit", ctypes.POINTER(ctypes.c_int32))]


class CqcInstance(ctypes.Structure):
    _fields_ = [("cut", CqcCut), ("entries", ctypes.POINTER(ctypes.c_void_p)),
                ("out", ctypes.c_void_p), ("mass", ctypes.c_void_p)]


class CqcEntryJob(ctypes.Structure):
    _fields_ = [("f", ctypes.c_int32), ("n_cuts", ctypes.c_int32),
                ("cut_kind", ctypes.POINTER(ctypes.c_int32)), ("variants", ctypes.c_void_p),
                ("entries", ctypes.c_void_p), ("form", ctypes.c_int32)]


class CqcDDParams(ctypes.Structure):
    _fields_ = [("n_active", ctypes.c_int32), ("n_recursions", ctypes.c_int32),
                ("first_active", ctypes.POINTER(ctypes.c_int32)), ("strategy", ctypes.c_int32),
                ("bins_per_round", ctypes.c_int32), ("bins_f32", ctypes.c_int32)]


class CqcDDRecord(ctypes.Structure):
    _fields_ = [("parent_rec", ctypes.c_int32), ("n_active", ctypes.c_int32),
                ("parent_bin", ctypes.c_int64), ("mass", ctypes.c_double),
                ("role", ctypes.c_int8 * MAX_DD_QUBITS)]


class CqcError(RuntimeError):
    def __init__(self, code, detail):
        super().__init__(f"{STATUS.get(code, code)}: {detail}")
        self.code = code
        self.detail = detail


_lib = None


def lib():
    """Load libcqc.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2012_02333_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, sz, i32, i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64
    L.cqc_fd_workspace_size.argtypes = [P(CqcInstance), i32, ctypes.c_int, ctypes.c_int, ctypes.c_int, P(sz)]
    L.cqc_reconstruct_fd.argtypes = [P(CqcInstance), i32, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, sz, vp]
    L.cqc_dd_workspace_size.argtypes = [P(CqcInstance), ctypes.c_int, ctypes.c_int, P(CqcDDParams), P(sz)]
    L.cqc_reconstruct_dd.argtypes = [P(CqcInstance), ctypes.c_int, ctypes.c_int, P(CqcDDParams), vp,
                                     P(CqcDDRecord), P(i32), vp, sz, vp]
    L.cqc_backward_workspace_size.argtypes = [P(CqcInstance), i32, ctypes.c_int, ctypes.c_int, P(sz)]
    L.cqc_reconstruct_backward.argtypes = [P(CqcInstance), i32, ctypes.c_int, ctypes.c_int,
                                           P(vp), P(P(vp)), vp, sz, vp]
    L.cqc_cost.argtypes = [P(CqcCut), P(ctypes.c_double), P(ctypes.c_double)]
    L.cqc_autotune.argtypes = [P(CqcInstance), i32, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, sz, vp]
    L.cqc_trace_enable.argtypes = [ctypes.c_int]
    L.cqc_trace_read.argtypes = [ctypes.c_char_p, sz, P(i32), P(ctypes.c_double), i32, P(i32)]
    L.cqc_status_string.restype = ctypes.c_char_p
    L.cqc_status_string.argtypes = [ctypes.c_int]
    L.cqc_last_error_detail.restype = ctypes.c_char_p
    L.cqc_last_error_detail.argtypes = []
    L.cqc_selftest_mfma.argtypes = [vp, vp]
    L.cqc_batch_create.argtypes = [P(CqcInstance), i32, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, sz, vp,
                                   P(vp)]
    L.cqc_batch_create_xent.argtypes = [P(CqcInstance), i32, ctypes.c_int, ctypes.c_int, ctypes.c_int, P(vp),
                                        P(vp), P(vp), vp, sz, vp, P(vp)]
    L.cqc_batch_run.argtypes = [vp, vp]
    L.cqc_batch_destroy.argtypes = [vp]
    L.cqc_batch_backward_workspace_size.argtypes = [vp, P(sz)]
    L.cqc_batch_backward_create.argtypes = [vp, P(vp), P(P(vp)), vp, sz, vp, P(vp)]
    L.cqc_batch_backward_run.argtypes = [vp, vp]
    L.cqc_batch_backward_destroy.argtypes = [vp]
    L.cqc_build_entries.argtypes = [P(CqcEntryJob), i32, ctypes.c_int, ctypes.c_int, vp]
    L.cqc_chi2.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int, i64, vp, vp, sz, vp]
    L.cqc_xent_grad.argtypes = [vp, vp, ctypes.c_int, i64, vp, vp, vp, sz, vp]
    L.cqc_tune_reset.argtypes = []
    L.cqc_dd_query_workspace_size.argtypes = [P(CqcInstance), ctypes.c_int, ctypes.c_int, P(CqcDDParams), P(sz)]
    L.cqc_dd_query_create.argtypes = [P(CqcInstance), ctypes.c_int, ctypes.c_int, P(CqcDDParams), vp, vp, vp, vp,
                                      sz, vp, P(vp)]
    L.cqc_dd_query_run.argtypes = [vp, vp]
    L.cqc_dd_query_run_range.argtypes = [vp, i32, i32, vp]
    L.cqc_dd_query_destroy.argtypes = [vp]
    L.cqc_reconstruct_fd_noalloc.argtypes = [P(CqcInstance), i32, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp]
    for name in EXPORTS:
        f = getattr(L, name)
        if f.restype is None or f.restype is ctypes.c_int:
            if name not in ("cqc_status_string", "cqc_last_error_detail"):
                f.restype = ctypes.c_int
    _lib = L
    return L


def check(code):
    if code != CQC_OK:
        detail = lib().cqc_last_error_detail().decode(errors="replace")
        raise CqcError(code, detail)
