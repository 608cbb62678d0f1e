"""cqc_reconstruct_fd_noalloc: the FD call whose workspace is a fixed device
array inside the library (for callers that cannot allocate).

Called through the C ABI, its outputs and FP64 masses must equal those of
cqc_reconstruct_fd (caller workspace) on the same inputs bit for bit - the
kernels and their order of additions are the same - on two calls in a row,
the second with a smaller instance, so that the second call runs over the
first call's leftovers in the array.  The smaller instance is also checked
against the oracle.  A batch of instances goes through the same entry point.
"""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from oracle import fd, metrics
from tests.gpu_util import oracle_inputs

pytestmark = pytest.mark.gpu
cqc = pytest.importorskip("paper_2012_02333_amd")
from paper_2012_02333_amd import _lib  # noqa: E402

C = W.CutMap
PREC = {"fp32": (torch.float32, 0, 0, 1), "fp64": (torch.float64, 1, 1, 0), "bf16x6": (torch.float32, 0, 0, 2)}


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _table(cuts, ents, outs, mass):
    arr = (_lib.CqcInstance * len(cuts))()
    keep = []
    for i, (c, e) in enumerate(zip(cuts, ents)):
        ptrs = (ctypes.c_void_p * len(e))(*[E.data_ptr() for E in e])
        keep.append(ptrs)
        arr[i] = _lib.CqcInstance(c.c, ptrs, outs[i].data_ptr(), mass.data_ptr() + 8 * i)
    return arr, keep


def _both(cuts_w, seed, prec):
    """Runs the same instances through cqc_reconstruct_fd (a fresh caller
    workspace) and cqc_reconstruct_fd_noalloc; returns both outputs and masses."""
    dt, in_t, out_t, p = PREC[prec]
    np_dt = np.float32 if dt == torch.float32 else np.float64
    host = [[E.astype(np_dt) for E in W.random_entries(c, seed=seed + i)] for i, c in enumerate(cuts_w)]
    ents = [[torch.from_numpy(E).cuda() for E in h] for h in host]
    cuts = [cqc.CutMap.from_workload(c) for c in cuts_w]
    L = _lib.lib()
    s = torch.cuda.current_stream().cuda_stream
    res = []
    for noalloc in (False, True):
        outs = [torch.full((2 ** c.n,), float("nan"), dtype=dt, device="cuda") for c in cuts_w]
        mass = torch.full((len(cuts_w),), float("nan"), dtype=torch.float64, device="cuda")
        arr, keep = _table(cuts, ents, outs, mass)
        if noalloc:
            rc = L.cqc_reconstruct_fd_noalloc(arr, len(cuts), in_t, out_t, p, s)
        else:
            nb = ctypes.c_size_t(0)
            _lib.check(L.cqc_fd_workspace_size(arr, len(cuts), in_t, out_t, p, ctypes.byref(nb)))
            ws = torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device="cuda")
            rc = L.cqc_reconstruct_fd(arr, len(cuts), in_t, out_t, p, ws.data_ptr(), ws.numel(), s)
        _lib.check(rc)
        torch.cuda.synchronize()
        res.append((outs, mass))
    return host, res


@pytest.mark.parametrize("prec", ["fp32", "fp64", "bf16x6"])
def test_noalloc_equals_caller_workspace_two_calls(prec):
    _gpu()
    # first call: a three-subcircuit chain with three cuts per boundary (an
    # intermediate tensor and label lists in the workspace); second call: a
    # smaller two-subcircuit instance over what the first left in the array
    big = C(21, [7, 7, 7], [0, 0, 0, 1, 1, 1], [1, 1, 1, 2, 2, 2], list(range(21)))
    small = C(12, [5, 7], [0, 0, 0], [1, 1, 1], [3, 0, 7, 1, 11, 2, 4, 5, 6, 8, 9, 10])
    for k, cw in enumerate((big, small)):
        host, ((o_ref, m_ref), (o_na, m_na)) = _both([cw], 900 + k, prec)
        print(f"noalloc {prec} call {k}: n={cw.n}", flush=True)
        assert torch.equal(o_na[0], o_ref[0]), (prec, k)
        assert torch.equal(m_na, m_ref), (prec, k)
    ref = fd.reconstruct(oracle_inputs(host[0]), small)
    tol = 1e-12 if prec == "fp64" else 1e-6
    assert metrics.rel_l1(o_na[0].double().cpu().numpy(), ref) <= tol


def test_noalloc_batch_equals_caller_workspace():
    _gpu()
    cuts_w = [C(16, [8, 8], [0, 0, 0], [1, 1, 1], list(range(16))),
              C(9, [4, 5], [0, 0], [1, 1], [5, 0, 3, 8, 1, 2, 4, 7, 6]),
              C(12, [4, 4, 4], [0, 1, 2, 0], [1, 2, 0, 1], list(range(12))),
              C(7, [3, 4], [], [], list(range(7)))]
    _, ((o_ref, m_ref), (o_na, m_na)) = _both(cuts_w, 950, "fp32")
    for k in range(len(cuts_w)):
        assert torch.equal(o_na[k], o_ref[k]), k
    assert torch.equal(m_na, m_ref)


def test_noalloc_binding():
    _gpu()
    cw = C(14, [7, 7], [0, 0], [1, 1], list(range(14)))
    ents = [torch.from_numpy(E.astype(np.float32)).cuda() for E in W.random_entries(cw, seed=990)]
    cut = cqc.CutMap.from_workload(cw)
    call = cqc.FDCall(ents, cut, precision="fp32", noalloc=True)
    call.run()
    p_ref, m_ref = cqc.reconstruct_fd(ents, cut, precision="fp32")
    torch.cuda.synchronize()
    assert torch.equal(call.outs[0], p_ref) and torch.equal(call.mass[0], m_ref)
