"""ctypes loader for the C/OpenMP twin of the FD definition and of the DD merge
and bins (test infrastructure)."""
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
        L.cqo_chi2.restype = ctypes.c_double
        L.cqo_chi2.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int]
        L.cqo_dd_merge.restype = ctypes.c_int
        L.cqo_dd_merge.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_int]
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


ACTIVE, MERGED = -2, -1


def dd_merge(entries, cut, role, threads=0):
    """The DD merge of every subcircuit (role per global qubit: -2 active, -1
    merged, 0/1 zoomed), by the C twin; columns enumerate each subcircuit's
    active bits in local order."""
    L = lib()
    out = []
    for c in range(cut.n_sub):
        E = np.ascontiguousarray(entries[c], dtype=np.float64)
        qs = cut.out_qubits_of(c)
        rl = np.array([role[q] for q in qs], dtype=np.int8)
        na = int(np.sum(rl == ACTIVE))
        o = np.empty((E.shape[0], 2 ** na), dtype=np.float64)
        if L.cqo_dd_merge(len(qs), E.shape[0], E.ctypes.data, rl.ctypes.data, o.ctypes.data, int(threads)) != 0:
            raise ValueError("cqo_dd_merge rejected its arguments")
        out.append(o)
    return out


def dd_bins(merged, cut, role, betas=None, threads=0):
    """Bins over the active qubits: the FD definition on the merged entries,
    with bin-index bits following the active qubits in ascending id (first
    most significant), by the C twin of the FD build."""
    from types import SimpleNamespace
    active = [q for q in range(cut.n) if role[q] == ACTIVE]
    pos = {q: i for i, q in enumerate(active)}
    f = [sum(1 for q in cut.out_qubits_of(c) if role[q] == ACTIVE) for c in range(cut.n_sub)]
    oq = [pos[q] for c in range(cut.n_sub) for q in cut.out_qubits_of(c) if role[q] == ACTIVE]
    sub = SimpleNamespace(n=len(active), n_sub=cut.n_sub, n_cuts=cut.n_cuts, f=f,
                          edge_up=cut.edge_up, edge_down=cut.edge_down, out_qubit=oq)
    return reconstruct(merged, sub, betas, threads)


def chi2(a, b, threads=0):
    """Eq. 16 by the C twin (terms with a_i + b_i > 0), FP64."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    if a.shape != b.shape:
        raise ValueError("shapes differ")
    return float(lib().cqo_chi2(a.ctypes.data, b.ctypes.data, a.size, int(threads)))
