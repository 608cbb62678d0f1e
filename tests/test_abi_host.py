"""Host-only checks of the C ABI: the library loads, exports every function
include/cqc.h declares, and rejects bad arguments before enqueuing anything.
No GPU is touched: every call here fails validation or is a pure host query."""
import ctypes
import os
import re

import pytest

from paper_2012_02333_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cqc.h")

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="libcqc.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cqc_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_function():
    L = _lib.lib()
    names = declared_functions()
    assert "cqc_reconstruct_fd" in names and "cqc_reconstruct_dd" in names
    assert "cqc_reconstruct_backward" in names
    for name in names:
        assert hasattr(L, name), name
    assert set(names) <= set(_lib.EXPORTS)


def _inst(n, f, edges, outq, nsub=None):
    I32 = ctypes.c_int32
    keep = []
    fa = (I32 * max(1, len(f)))(*f)
    up = (I32 * max(1, len(edges)))(*[u for u, _ in edges])
    dn = (I32 * max(1, len(edges)))(*[d for _, d in edges])
    oq = (I32 * max(1, len(outq)))(*outq)
    keep += [fa, up, dn, oq]
    cut = _lib.CqcCut(n, nsub if nsub is not None else len(f), len(edges), fa, up, dn, oq)
    ents = (ctypes.c_void_p * max(1, len(f)))(*([0x1000] * len(f)))
    keep.append(ents)
    inst = _lib.CqcInstance(cut, ents, 0x2000, None)
    inst._keep = keep
    return inst


def ws_size(inst, prec=1, in_t=0, out_t=0):
    nb = ctypes.c_size_t(0)
    rc = _lib.lib().cqc_fd_workspace_size(ctypes.byref(inst), 1, in_t, out_t, prec, ctypes.byref(nb))
    return rc, nb.value


def test_valid_cut_workspace_query():
    inst = _inst(24, [11, 13], [(0, 1), (0, 1)], list(range(24)))
    rc, nb = ws_size(inst)
    assert rc == 0 and nb > 0
    rc64, nb64 = ws_size(inst, prec=0, in_t=1, out_t=1)
    assert rc64 == 0
    # FP32 entries under FP64 arithmetic need a widened copy: more workspace
    rc_mix, nb_mix = ws_size(inst, prec=0, in_t=0, out_t=1)
    assert rc_mix == 0 and nb_mix > nb64


@pytest.mark.parametrize("n,f,edges,outq,code", [
    (8, [4, 3], [(0, 1)], list(range(8)), 2),            # sum f != n
    (8, [4, 4], [(0, 1)], [0, 1, 2, 3, 4, 5, 6, 6], 2),  # not a permutation
    (8, [4, 4], [(0, 1)], [0, 1, 2, 3, 4, 5, 6, 8], 2),  # qubit out of range
    (8, [4, 4], [(0, 2)], list(range(8)), 1),            # cut names a missing subcircuit
    (8, [4, 4], [(1, 1)], list(range(8)), 2),            # cut inside one subcircuit
    (41, [20, 21], [(0, 1)], list(range(41)), 3),        # 2^41 outputs: beyond FD limit
    (8, [-1, 9], [(0, 1)], list(range(8)), 2),           # negative f
])
def test_invalid_cuts(n, f, edges, outq, code):
    rc, _ = ws_size(_inst(n, f, edges, outq))
    assert rc == code
    detail = _lib.lib().cqc_last_error_detail().decode()
    assert detail


def test_bad_enums_and_pointers():
    L = _lib.lib()
    inst = _inst(8, [4, 4], [(0, 1)], list(range(8)))
    nb = ctypes.c_size_t(0)
    assert L.cqc_fd_workspace_size(ctypes.byref(inst), 1, 7, 0, 1, ctypes.byref(nb)) == 1
    assert L.cqc_fd_workspace_size(ctypes.byref(inst), 1, 0, 0, 9, ctypes.byref(nb)) == 1
    assert L.cqc_fd_workspace_size(ctypes.byref(inst), 0, 0, 0, 1, ctypes.byref(nb)) == 1
    assert L.cqc_fd_workspace_size(None, 1, 0, 0, 1, ctypes.byref(nb)) == 1
    assert L.cqc_fd_workspace_size(ctypes.byref(inst), 1, 0, 0, 1, None) == 1
    # null entry pointer is caught before anything is enqueued
    inst.entries[1] = None
    assert L.cqc_reconstruct_fd(ctypes.byref(inst), 1, 0, 0, 1, 0x3000, 1 << 30, None) == 1


def test_workspace_too_small_enqueues_nothing():
    L = _lib.lib()
    inst = _inst(8, [4, 4], [(0, 1)], list(range(8)))
    rc, need = ws_size(inst)
    assert rc == 0
    assert L.cqc_reconstruct_fd(ctypes.byref(inst), 1, 0, 0, 1, 0x3000, need - 1, None) == 4
    assert L.cqc_reconstruct_fd(ctypes.byref(inst), 1, 0, 0, 1, None, need, None) == 4
    assert L.cqc_reconstruct_fd(ctypes.byref(inst), 1, 0, 0, 1, 0x3010, need, None) == 4  # misaligned


def test_status_strings():
    L = _lib.lib()
    assert L.cqc_status_string(0) == b"CQC_OK"
    assert L.cqc_status_string(4) == b"CQC_ERR_WORKSPACE"
    assert L.cqc_version() >= 100


def test_cost_eq14():
    L = _lib.lib()
    inst = _inst(30, [9, 9, 12], [(0, 1)] * 3 + [(1, 2)] * 3, list(range(30)))
    a, b = ctypes.c_double(0), ctypes.c_double(0)
    assert L.cqc_cost(ctypes.byref(inst.cut), ctypes.byref(a), ctypes.byref(b)) == 0
    assert a.value == 4 ** 6 * (2 ** 18 + 2 ** 30)
    # library plan: A-B over 3 labels into 64 x 2^18, then 2^18 x 2^12 over 3 labels
    assert b.value == 64 * 64 * 2 ** 18 + 64 * 2 ** 30


def test_batch_backward_rejects_null_handles():
    """The batched adjoint's entry points refuse a null batch, handle or output
    pointer with CQC_ERR_INVALID_ARG before touching any device memory."""
    L = _lib.lib()
    nb = ctypes.c_size_t(0)
    assert L.cqc_batch_backward_workspace_size(None, ctypes.byref(nb)) == 1
    assert L.cqc_batch_backward_create(None, None, None, None, 0, None, None) == 1
    h = ctypes.c_void_p(0)
    assert L.cqc_batch_backward_create(None, None, None, None, 0, None, ctypes.byref(h)) == 1
    assert L.cqc_batch_backward_run(None, None) == 1
    assert L.cqc_batch_backward_destroy(None) == 0
    assert L.cqc_batch_run(None, None) != 0


def test_build_entries_validation():
    """cqc_build_entries refuses bad jobs before any launch: more than three
    incoming or four outgoing cuts, cut kinds other than 0/1, NULL tensors,
    f outside [0, 30], unknown dtypes."""
    L = _lib.lib()
    I32 = ctypes.c_int32

    def job(f, kinds, v=0x1000, e=0x2000, form=0):
        ck = (I32 * max(1, len(kinds)))(*kinds)
        j = _lib.CqcEntryJob(f, len(kinds), ck, v, e, form)
        j._keep = ck
        return j

    def call(j, in_t=0, out_t=0):
        arr = (_lib.CqcEntryJob * 1)(j)
        return L.cqc_build_entries(arr, 1, in_t, out_t, None)

    assert call(job(4, [0, 0, 0, 0])) == 3          # CQC_ERR_UNSUPPORTED
    assert call(job(4, [1, 1, 1, 1, 1])) == 3
    assert call(job(4, [0, 2])) == 1                # CQC_ERR_INVALID_ARG
    assert call(job(4, [0], v=None)) == 1
    assert call(job(4, [1], e=None)) == 1
    assert call(job(31, [1])) == 2                  # CQC_ERR_SHAPE
    assert call(job(-1, [1])) == 2
    assert call(job(4, [1]), in_t=7) == 1
    assert call(job(4, [1], form=2)) == 1
    assert L.cqc_build_entries(None, 1, 0, 0, None) == 1
    arr = (_lib.CqcEntryJob * 1)(job(4, [1]))
    assert L.cqc_build_entries(arr, 0, 0, 0, None) == 1


def test_chi2_validation():
    """cqc_chi2 refuses bad dtypes, n < 0, NULL output or inputs and a short
    workspace before any launch."""
    L = _lib.lib()
    out, ws = 0x3000, 0x4000
    assert L.cqc_chi2(0x1000, 7, 0x2000, 0, 10, out, ws, 8192, None) == 1
    assert L.cqc_chi2(0x1000, 0, 0x2000, 0, -1, out, ws, 8192, None) == 1
    assert L.cqc_chi2(0x1000, 0, 0x2000, 0, 10, None, ws, 8192, None) == 1
    assert L.cqc_chi2(None, 0, 0x2000, 0, 10, out, ws, 8192, None) == 1
    assert L.cqc_chi2(0x1000, 0, 0x2000, 0, 10, out, ws, 100, None) == 4
    assert L.cqc_chi2(0x1000, 0, 0x2000, 0, 10, out, None, 8192, None) == 4


def _dd_ws(inst, strategy=0, per_round=1, a=3, R=4, f32=0):
    params = _lib.CqcDDParams(a, R, None, strategy, per_round, f32)
    nb = ctypes.c_size_t(0)
    rc = _lib.lib().cqc_dd_workspace_size(ctypes.byref(inst), 0, 1, ctypes.byref(params), ctypes.byref(nb))
    return rc, nb.value


def test_dd_strategy_and_round_validation():
    """Strategies 0..2 and bins_per_round 0..64 are accepted (the workspace grows
    with the per-round read-back slots); anything else is refused on the host."""
    inst = _inst(10, [5, 5], [(0, 1), (0, 1)], list(range(10)))
    for s in (0, 1, 2):
        assert _dd_ws(inst, s)[0] == 0
    assert _dd_ws(inst, 3)[0] == 1
    assert _dd_ws(inst, -1)[0] == 1
    assert _dd_ws(inst, 0, -1)[0] == 1
    assert _dd_ws(inst, 0, 65)[0] == 1
    rc0, nb0 = _dd_ws(inst, 0, 0)
    rc1, nb1 = _dd_ws(inst, 0, 1)
    rc64, nb64 = _dd_ws(inst, 2, 64)
    assert rc0 == rc1 == rc64 == 0 and nb0 == nb1 and nb64 > nb1


def test_dd_plan_cache_keys_on_every_input():
    """Alternating queries that differ in one input each get their own plan."""
    inst = _inst(12, [6, 6], [(0, 1), (0, 1)], list(range(12)))
    inst_perm = _inst(12, [6, 6], [(0, 1), (0, 1)], list(range(11, -1, -1)))
    ref = {key: _dd_ws(*args)[1] for key, args in
           {"a3": (inst, 0, 1, 3), "a5": (inst, 0, 1, 5), "r16": (inst, 2, 16, 3), "perm": (inst_perm, 0, 1, 5)}.items()}
    assert ref["a3"] != ref["a5"] and ref["r16"] > ref["a3"]
    for _ in range(3):
        assert _dd_ws(inst, 0, 1, 5)[1] == ref["a5"]
        assert _dd_ws(inst, 0, 1, 3)[1] == ref["a3"]
        assert _dd_ws(inst, 2, 16, 3)[1] == ref["r16"]
        assert _dd_ws(inst_perm, 0, 1, 5)[1] == ref["perm"]


def test_dd_active_limit_and_bin_dtype():
    """Up to 36 active qubits (2^36 bins); the bins flag is 0 (FP64) or 1
    (FP32) and both are accepted for a 100-qubit, five-subcircuit cut."""
    edges = [(0, 1), (0, 1), (1, 2), (1, 2), (2, 3), (2, 3), (3, 4), (3, 4)]
    inst = _inst(100, [20] * 5, edges, list(range(100)))
    assert _dd_ws(inst, 0, 1, 35, 1, 1)[0] == 0
    assert _dd_ws(inst, 0, 1, 36, 1, 0)[0] == 0
    assert _dd_ws(inst, 0, 1, 37, 1, 1)[0] == 1
    assert _dd_ws(inst, 0, 1, 35, 1, 2)[0] == 1
    assert _dd_ws(inst, 0, 1, 35, 1, -1)[0] == 1


def test_xent_grad_validation():
    """cqc_xent_grad refuses a bad dtype, n < 0, NULL buffers and a loss
    without workspace before any launch."""
    L = _lib.lib()
    p, t, g, loss, ws = 0x1000, 0x2000, 0x3000, 0x4000, 0x5000
    assert L.cqc_xent_grad(p, t, 9, 10, g, None, None, 0, None) == 1
    assert L.cqc_xent_grad(p, t, 0, -1, g, None, None, 0, None) == 1
    assert L.cqc_xent_grad(None, t, 0, 10, g, None, None, 0, None) == 1
    assert L.cqc_xent_grad(p, t, 0, 10, None, None, None, 0, None) == 1
    assert L.cqc_xent_grad(p, t, 0, 10, g, loss, None, 0, None) == 4
    assert L.cqc_xent_grad(p, t, 0, 10, g, loss, ws, 100, None) == 4


def test_noalloc_rejects_before_enqueue():
    """The fixed-workspace FD call validates like cqc_reconstruct_fd, and
    rejects a call whose workspace exceeds its array (n = 30 with three cuts
    per boundary needs about 72 MiB) before touching any device."""
    L = _lib.lib()
    big = _inst(30, [9, 9, 12], [(0, 1)] * 3 + [(1, 2)] * 3, list(range(30)))
    rc, need = ws_size(big)
    assert rc == 0 and need > _lib.NOALLOC_WORKSPACE_BYTES
    assert L.cqc_reconstruct_fd_noalloc(ctypes.byref(big), 1, 0, 0, 1, None) == 4
    assert b"static workspace" in L.cqc_last_error_detail()
    bad = _inst(24, [11, 12], [(0, 1), (0, 1)], list(range(24)))   # sum f != n
    assert L.cqc_reconstruct_fd_noalloc(ctypes.byref(bad), 1, 0, 0, 1, None) == 2
    ok = _inst(24, [11, 13], [(0, 1), (0, 1)], list(range(24)))
    assert L.cqc_reconstruct_fd_noalloc(ctypes.byref(ok), 1, 0, 0, 9, None) == 1   # unknown precision
    assert L.cqc_reconstruct_fd_noalloc(None, 1, 0, 0, 1, None) == 1


def test_dd_query_validation():
    """The device-resident DD query plans on the host: one bin per recursion
    only, and the same parameter checks as the host-driven query."""
    L = _lib.lib()
    inst = _inst(12, [6, 6], [(0, 1), (0, 1)], list(range(12)))
    nb = ctypes.c_size_t(0)
    ok = _lib.CqcDDParams(4, 5, None, 0, 1, 0)
    assert L.cqc_dd_query_workspace_size(ctypes.byref(inst), 0, 1, ctypes.byref(ok), ctypes.byref(nb)) == 0
    assert nb.value > 0
    rounds = _lib.CqcDDParams(4, 5, None, 0, 4, 0)
    assert L.cqc_dd_query_workspace_size(ctypes.byref(inst), 0, 1, ctypes.byref(rounds), ctypes.byref(nb)) == 3
    bad = _lib.CqcDDParams(0, 5, None, 0, 1, 0)
    assert L.cqc_dd_query_workspace_size(ctypes.byref(inst), 0, 1, ctypes.byref(bad), ctypes.byref(nb)) == 1
    h = ctypes.c_void_p(0)
    # NULL outputs, and a workspace smaller than the query needs: nothing enqueued
    assert L.cqc_dd_query_create(ctypes.byref(inst), 0, 1, ctypes.byref(ok), None, None, None, None, 0, None,
                                 ctypes.byref(h)) == 1
    assert L.cqc_dd_query_create(ctypes.byref(inst), 0, 1, ctypes.byref(ok), 0x1000, 0x2000, 0x3000, 0x4000,
                                 16, None, ctypes.byref(h)) == 4


def test_xent_batch_rejects_before_enqueue():
    """cqc_batch_create_xent validates its bindings before any device work:
    one instance, NULL target/gradient arrays or entries, and a loss together
    with a mass are CQC_ERR_INVALID_ARG; a NULL output is allowed (p is not
    kept), so such a batch gets as far as the workspace check."""
    L = _lib.lib()
    I = _lib.CqcInstance * 2
    a = _inst(8, [4, 4], [(0, 1)], list(range(8)))
    b = _inst(10, [5, 5], [(0, 1), (0, 1)], list(range(10)))
    arr = I(a, b)
    VP2 = ctypes.c_void_p * 2
    tg, gr = VP2(0x4000, 0x5000), VP2(0x6000, 0x7000)
    h = ctypes.c_void_p(0)

    def create(n, t, g, losses, ws=0x100000, ws_bytes=1 << 40):
        return L.cqc_batch_create_xent(arr, n, 0, 0, 1, t, g, losses, ws, ws_bytes, None, ctypes.byref(h))

    assert create(1, tg, gr, None) == 1
    assert b"two instances" in L.cqc_last_error_detail()
    assert create(2, None, gr, None) == 1
    assert create(2, tg, None, None) == 1
    assert create(2, tg, VP2(0x6000, 0), None) == 1
    arr[1].mass = 0x8000
    assert create(2, tg, gr, VP2(0, 0x9000)) == 1
    assert b"loss and a mass" in L.cqc_last_error_detail()
    arr[1].mass = None
    arr[0].out = None
    assert create(2, tg, gr, VP2(0, 0x9000), ws_bytes=16) == 4
    assert not h.value
