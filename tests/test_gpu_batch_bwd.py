"""Batched adjoint (cqc_batch_backward_*): dL/dE of every instance of a
prepared batch from dL/dp, on the forward tensors the batch's run left in its
workspace.

Bar: each instance's gradients against the oracle's plain-definition
vector-Jacobian product fed the same dL/dp (relative L2 per entry tensor
<= 1e-5 in FP32, <= 1e-12 in FP64, as for the one-instance adjoint); bitwise
repeatability; forward + adjoint captured in one graph and replayed with eager
work in between, every replay equal to the eager result.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import adjoint, metrics
from tests.gpu_util import oracle_inputs

pytestmark = pytest.mark.gpu
cqc = pytest.importorskip("paper_2012_02333_amd")

C = W.CutMap
# permuted output order (dL/dp gathered), Kronecker product, single
# subcircuit, cyclic three-subcircuit graph (an intermediate level), ragged
# widths, three, four and five shared cuts (label blocks of 64, of 256 on the
# dX side at four in FP32, of 256 at five), a chain of three with two cuts per
# boundary, a larger two-cut pair, a four-cut pair with several output tiles
# and inner chunks per side, and three-cut pairs whose dY side has four and
# two output columns
MIXED = [C(9, [4, 5], [0, 0], [1, 1], [5, 0, 3, 8, 1, 2, 4, 7, 6]),
         C(7, [3, 4], [], [], list(range(7))),
         C(6, [6], [], [], [3, 1, 0, 5, 2, 4]),
         C(12, [4, 4, 4], [0, 1, 2, 0], [1, 2, 0, 1], list(range(12))),
         C(11, [1, 2, 8], [0, 1, 1, 2], [1, 2, 2, 0], list(range(11))),
         C(10, [5, 5], [0, 0, 0], [1, 1, 1], list(range(10))),
         C(10, [5, 5], [0, 0, 0, 0], [1, 1, 1, 1], list(range(10))),
         C(15, [5, 5, 5], [0, 0, 1, 1], [1, 1, 2, 2], list(range(15))),
         C(14, [7, 7], [0, 0], [1, 1], list(range(14))),
         C(12, [6, 6], [0] * 5, [1] * 5, list(range(12))),
         C(17, [9, 8], [0] * 4, [1] * 4, list(range(17))),
         C(10, [2, 8], [0] * 3, [1] * 3, list(range(10))),
         C(10, [1, 9], [0] * 3, [1] * 3, list(range(10)))]


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _setup(np_dt, seed):
    host = [[E.astype(np_dt) for E in W.random_entries(c, seed=seed + i)] for i, c in enumerate(MIXED)]
    ents = [[torch.from_numpy(E).cuda() for E in e] for e in host]
    cuts = [cqc.CutMap.from_workload(c) for c in MIXED]
    dt = torch.float32 if np_dt == np.float32 else torch.float64
    rng = np.random.default_rng(seed)
    gout = [torch.from_numpy(rng.standard_normal(2 ** c.n)).to(device="cuda", dtype=dt) for c in MIXED]
    return host, ents, cuts, gout


@pytest.mark.parametrize("prec,np_dt,tol", [("fp32", np.float32, 1e-5), ("fp64", np.float64, 1e-12),
                                            ("bf16x6", np.float32, 1e-5)])
def test_batch_backward_matches_oracle(prec, np_dt, tol):
    _gpu()
    host, ents, cuts, gout = _setup(np_dt, 400)
    batch = cqc.Batch(ents, cuts, precision=prec)
    bwd = cqc.BatchBackward(batch, gout)
    batch.run()
    bwd.run()
    torch.cuda.synchronize()
    for k, cw in enumerate(MIXED):
        ref = adjoint.vjp(oracle_inputs(host[k]), cw, gout[k].double().cpu().numpy())
        assert len(ref) == len(bwd.grads[k])
        for c, r in enumerate(ref):
            got = bwd.grads[k][c]
            assert got.dtype == ents[k][c].dtype
            err = metrics.rel_l2(got.double().cpu().numpy(), r)
            assert err <= tol, (k, c, err)


def test_batch_backward_graph_replay_and_repeatable():
    _gpu()
    host, ents, cuts, gout = _setup(np.float32, 500)
    batch = cqc.Batch(ents, cuts, precision="fp32")
    bwd = cqc.BatchBackward(batch, gout)
    batch.run()
    bwd.run()
    torch.cuda.synchronize()
    eager = [[g.clone() for g in gl] for gl in bwd.grads]
    batch.run()
    bwd.run()
    torch.cuda.synchronize()
    for k in range(len(eager)):
        for c in range(len(eager[k])):
            assert torch.equal(bwd.grads[k][c], eager[k][c]), ("repeat", k, c)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=s):
            batch.run()
            bwd.run()
    torch.cuda.synchronize()
    for rep in range(3):
        for gl in bwd.grads:
            for g in gl:
                g.fill_(7.0)
        for o in batch.outs:
            o.fill_(-1.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k in range(len(eager)):
            for c in range(len(eager[k])):
                assert torch.equal(bwd.grads[k][c], eager[k][c]), (rep, k, c)


def test_batch_backward_rejects_mismatched_grad_out():
    _gpu()
    host, ents, cuts, gout = _setup(np.float32, 600)
    batch = cqc.Batch(ents, cuts, precision="fp32")
    with pytest.raises(ValueError):
        cqc.BatchBackward(batch, gout[:-1])
    bad = list(gout)
    bad[0] = bad[0].double()
    with pytest.raises(ValueError):
        cqc.BatchBackward(batch, bad)
