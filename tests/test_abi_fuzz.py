"""Host-side fuzz of the C ABI's validation and planning: seeded random cut
maps (valid and invalid: negative or oversized f, edges naming missing
subcircuits, repeated output qubits, out-of-range DD parameters) through the
workspace-size queries and cqc_cost.  Every call must return a documented
status (0..3), never crash, and a success must report a workspace size.  No
GPU is touched: these calls validate and plan on the host only.  (The same
sweep runs clean under AddressSanitizer on the host objects.)"""
import ctypes
import os
import random

import pytest

from paper_2012_02333_amd import _lib

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="libcqc.so not built")
I32 = ctypes.c_int32


def _random_inst(rng):
    nsub = rng.randint(0, 6)
    f = [rng.randint(-1, 14) for _ in range(nsub)]
    n = sum(max(0, v) for v in f) + (rng.randint(-1, 1) if rng.random() < 0.2 else 0)
    K = rng.randint(0, 9)
    up = [rng.randint(-1, nsub) for _ in range(K)]
    down = [rng.randint(-1, nsub) for _ in range(K)]
    oq = list(range(max(0, n)))
    rng.shuffle(oq)
    if oq and rng.random() < 0.1:
        oq[0] = oq[-1]
    keep = [(I32 * max(1, nsub))(*f) if nsub else None, (I32 * max(1, K))(*up) if K else None,
            (I32 * max(1, K))(*down) if K else None, (I32 * max(1, len(oq)))(*oq) if oq else None]
    cut = _lib.CqcCut(n, nsub, K, *keep)
    ents = (ctypes.c_void_p * max(1, nsub))(*([0x1000] * max(1, nsub)))
    inst = _lib.CqcInstance(cut, ents, 0x2000, None)
    return inst, cut, keep + [ents], n


def test_host_entry_points_return_documented_codes():
    L = _lib.lib()
    rng = random.Random(7)
    ok = {"fd": 0, "dd": 0, "bwd": 0, "cost": 0}
    for _ in range(600):
        inst, cut, keep, n = _random_inst(rng)
        nb = ctypes.c_size_t(0)
        prec = rng.randint(-1, 4)
        rc = L.cqc_fd_workspace_size(ctypes.byref(inst), 1, rng.randint(0, 1), rng.randint(0, 1), prec, ctypes.byref(nb))
        assert rc in (0, 1, 2, 3)
        if rc == 0:
            assert nb.value > 0
            ok["fd"] += 1
        a = rng.randint(0, 40)
        first = (I32 * a)(*[rng.randint(-1, max(0, n)) for _ in range(a)]) if (a and rng.random() < 0.3) else None
        params = _lib.CqcDDParams(a, rng.randint(0, 6), first, rng.randint(-1, 3), rng.randint(-1, 70), rng.randint(-1, 2))
        rc = L.cqc_dd_workspace_size(ctypes.byref(inst), rng.randint(0, 1), prec, ctypes.byref(params), ctypes.byref(nb))
        assert rc in (0, 1, 2, 3)
        ok["dd"] += rc == 0
        rc = L.cqc_backward_workspace_size(ctypes.byref(inst), 1, rng.randint(0, 1), prec, ctypes.byref(nb))
        assert rc in (0, 1, 2, 3)
        ok["bwd"] += rc == 0
        e14, macs = ctypes.c_double(0), ctypes.c_double(0)
        rc = L.cqc_cost(ctypes.byref(cut), ctypes.byref(e14), ctypes.byref(macs))
        assert rc in (0, 1, 2, 3)
        if rc == 0:
            assert e14.value >= 0 and macs.value >= 0
            ok["cost"] += 1
        if rc != 0:
            assert _lib.lib().cqc_last_error_detail()
    # the sweep reaches the accepting paths too, not only the rejections
    assert all(v > 0 for v in ok.values()), ok
