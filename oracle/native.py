"""ctypes loader for the C/OpenMP twin of the FD definition (test infrastructure)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "c", "cqc_oracle.c")
LIB = os.path.join(_HERE, "_build", "libcqc_oracle.so")


def build():
    """Compile the twin with gcc (-O2, OpenMP)."""
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
                           SRC, "-o", tmp, "-lm"])
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        L.cqo_fd.restype = ctypes.c_int
        L.cqo_fd.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                             ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                             ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                             ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p,
                             ctypes.c_int64, ctypes.c_void_p, ctypes.c_int]
        L.cqo_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def max_threads():
    return int(lib().cqo_max_threads())


def reconstruct(entries, cut, xs=None, threads=0):
    """FD definition at indices xs (default all 2^n), FP64, by the C twin."""
    L = lib()
    ints = lambda v: (ctypes.c_int * len(v))(*[int(a) for a in v])
    ents = [np.ascontiguousarray(E, dtype=np.float64) for E in entries]
    ptrs = (ctypes.c_void_p * len(ents))(*[E.ctypes.data for E in ents])
    if xs is None:
        count = 2 ** cut.n
        xs_ptr = None
    else:
        xs = np.ascontiguousarray(xs, dtype=np.int64)
        count = xs.shape[0]
        xs_ptr = xs.ctypes.data
    out = np.empty(count, dtype=np.float64)
    rc = L.cqo_fd(cut.n, cut.n_sub, cut.n_cuts, ints(cut.f),
                  ints(cut.edge_up) if cut.n_cuts else None,
                  ints(cut.edge_down) if cut.n_cuts else None,
                  ints(cut.out_qubit), ptrs, xs_ptr, count, out.ctypes.data, int(threads))
    if rc != 0:
        raise ValueError("cqo_fd rejected its arguments")
    return out
