"""Batched reconstruction: many instances of uneven n and K in one call.

Every instance's output must equal (bit for bit) the single-instance call on
the same inputs - the term order of each output does not depend on the tile
shape or on batching - and the single-instance path is itself checked against
the oracle.  The exception is an FP32 step of three or more shared cuts with
2^19 to 2^22 outputs: a batch runs it on the wide kernel, a single call on the
register kernel, and the two differ by FP32 rounding (checked against the
oracle and the single call's values to the FP32 bars).  A prepared batch is captured into a graph and replayed with eager
work in between; every replay must reproduce the eager result.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fd, metrics
from tests.gpu_util import oracle_inputs, REL_L1

pytestmark = pytest.mark.gpu
cqc = pytest.importorskip("paper_2012_02333_amd")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _instances(count, n_lo, n_hi, seed):
    insts = W.batch_instances(count=count, seed=seed, n_lo=n_lo, n_hi=n_hi)
    return insts


@pytest.mark.parametrize("prec,dtype", [("fp32", torch.float32), ("fp64", torch.float64),
                                        ("bf16x6", torch.float32), ("bf16x3", torch.float32)])
def test_batch_equals_single_calls(prec, dtype):
    _gpu()
    insts = _instances(24, 8, 14, seed=5)
    np_dt = np.float32 if dtype == torch.float32 else np.float64
    ents = [[torch.from_numpy(E.astype(np_dt)).cuda() for E in i.entries] for i in insts]
    cuts = [cqc.CutMap.from_workload(i.cut) for i in insts]
    call = cqc.FDCall(ents, cuts, precision=prec)
    call.run()
    torch.cuda.synchronize()
    for k, inst in enumerate(insts):
        p1, m1 = cqc.reconstruct_fd(ents[k], cuts[k], precision=prec)
        assert torch.equal(call.outs[k], p1), k
        assert abs(float(call.mass[k]) - float(m1)) <= 1e-12
        if k < 6:
            e64 = oracle_inputs([E.astype(np_dt) for E in inst.entries])
            ref = fd.reconstruct(e64, inst.cut)
            # simulated circuits: the flat relative-L1 bar of each precision
            tol = 1e-12 if prec == "fp64" else REL_L1[prec]
            err = metrics.rel_l1(call.outs[k].double().cpu().numpy(), ref)
            print(f"batch {prec} instance {k}: rel_l1={err:.3e} "
                  f"kappa={metrics.kappa(e64, inst.cut, np.abs(ref).sum()):.2f}")
            assert err <= tol


def test_batch_structures_mixed():
    """Batch mixing blocked and permuted outputs, single subcircuits, Kronecker
    products and cyclic cut graphs."""
    _gpu()
    C = W.CutMap
    cuts_w = [C(9, [4, 5], [0, 0], [1, 1], [5, 0, 3, 8, 1, 2, 4, 7, 6]),
              C(7, [3, 4], [], [], list(range(7))),
              C(6, [6], [], [], [3, 1, 0, 5, 2, 4]),
              C(12, [4, 4, 4], [0, 1, 2, 0], [1, 2, 0, 1], list(range(12))),
              C(11, [1, 2, 8], [0, 1, 1, 2], [1, 2, 2, 0], list(range(11))),
              C(10, [5, 5], [0, 0, 0], [1, 1, 1], list(range(10)))]
    ents_np = [W.random_entries(c, seed=300 + i, zero_rows=((0, 1),) if i == 5 else ()) for i, c in enumerate(cuts_w)]
    ents = [[torch.from_numpy(E.astype(np.float32)).cuda() for E in e] for e in ents_np]
    cuts = [cqc.CutMap.from_workload(c) for c in cuts_w]
    call = cqc.FDCall(ents, cuts, precision="fp32")
    call.run()
    torch.cuda.synchronize()
    for k in range(len(cuts)):
        p1, _ = cqc.reconstruct_fd(ents[k], cuts[k], precision="fp32")
        assert torch.equal(call.outs[k], p1), k


def test_batch_graph_replay():
    _gpu()
    insts = _instances(16, 8, 13, seed=6)
    ents = [[torch.from_numpy(E.astype(np.float32)).cuda() for E in i.entries] for i in insts]
    cuts = [cqc.CutMap.from_workload(i.cut) for i in insts]
    batch = cqc.Batch(ents, cuts, precision="fp32")
    batch.run()
    torch.cuda.synchronize()
    eager = [o.clone() for o in batch.outs]
    eager_mass = batch.mass.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        for o in batch.outs:
            o.zero_()
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            batch.run()
    torch.cuda.synchronize()
    for rep in range(4):
        for o in batch.outs:
            o.fill_(-1.0)
        batch.mass.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in range(len(eager)):
            assert torch.equal(batch.outs[k], eager[k]), (rep, k)
        assert torch.equal(batch.mass, eager_mass), rep


def test_batch_without_row_flags_runs_repeatedly():
    """A batch in which no instance's plan uses row flags (at most two cuts
    per contraction): the flag pass has no entry tensors and only zeroes the
    work-queue counters, so every run must redo all the work.  Three runs,
    the entries scaled by 2 in place before each later one: every output and
    mass bit for bit twice the previous (outputs scale exactly by 2), and the
    first run equals the one-instance calls."""
    _gpu()
    C = W.CutMap
    cuts_w = [C(18, [9, 9], [0, 0], [1, 1], list(range(18))),
              C(14, [7, 7], [0], [1], list(range(14))),
              C(15, [5, 5, 5], [0, 1], [1, 2], list(range(15)))]
    ents = [[torch.from_numpy(E.astype(np.float32)).cuda() for E in W.random_entries(c, seed=750 + i)]
            for i, c in enumerate(cuts_w)]
    cuts = [cqc.CutMap.from_workload(c) for c in cuts_w]
    batch = cqc.Batch(ents, cuts, precision="fp32")
    batch.run()
    torch.cuda.synchronize()
    for k in range(len(cuts)):
        p1, _ = cqc.reconstruct_fd(ents[k], cuts[k], precision="fp32")
        assert torch.equal(batch.outs[k], p1), k
    prev = [o.clone() for o in batch.outs]
    prev_m = batch.mass.clone()
    for rep in range(2):
        for e in ents:
            e[0].mul_(2.0)
        for o in batch.outs:
            o.fill_(-1.0)
        batch.run()
        torch.cuda.synchronize()
        for k in range(len(cuts)):
            assert torch.equal(batch.outs[k], 2.0 * prev[k]), (rep, k)
        assert torch.equal(batch.mass, 2.0 * prev_m), rep
        prev = [o.clone() for o in batch.outs]
        prev_m = batch.mass.clone()


def test_batch_strips_equal_single_calls():
    """Instances whose small-term steps run as two-tile strips in the batch
    (FP32, no row flags: two subcircuits with two cuts, a chain with two cuts
    per boundary) next to one whose plan needs row flags (three cuts): every
    output bit for bit the one-instance call's, and the strip queue ran."""
    _gpu()
    C = W.CutMap
    cuts_w = [C(18, [9, 9], [0, 0], [1, 1], list(range(18))),
              C(24, [8, 8, 8], [0, 0, 1, 1], [1, 1, 2, 2], list(range(24))),
              C(16, [8, 8], [0, 0, 0], [1, 1, 1], list(range(16))),
              C(17, [8, 9], [0], [1], list(range(17)))]
    ents = [[torch.from_numpy(E.astype(np.float32)).cuda() for E in W.random_entries(c, seed=700 + i)]
            for i, c in enumerate(cuts_w)]
    cuts = [cqc.CutMap.from_workload(c) for c in cuts_w]
    batch = cqc.Batch(ents, cuts, precision="fp32")
    with cqc.trace() as tr:
        batch.run()
        torch.cuda.synchronize()
    assert "contract_strip_queue" in tr.result, tr.result
    for k in range(len(cuts)):
        p1, m1 = cqc.reconstruct_fd(ents[k], cuts[k], precision="fp32")
        assert torch.equal(batch.outs[k], p1), k
        assert abs(float(batch.mass[k]) - float(m1)) <= 1e-12 * max(1.0, abs(float(m1))), k


def test_batch_fp32_wide_queue_equals_single_calls():
    """FP32 instances whose steps reach the persistent wide kernel inside a
    batch (64 terms over at least 2^22 outputs per step group): two 11-qubit
    subcircuits with three cuts, and a chain of three whose intermediate and
    final steps both qualify, next to small instances.  The FP32 wide queue
    runs; every output equals the one-instance call bit for bit; the wide
    instances' outputs match the oracle on a sample (relative L1 <= 1e-6 and
    every element within its rounding bound)."""
    _gpu()
    from oracle import native
    from tests.gpu_util import elementwise_ok, U32
    C = W.CutMap
    cuts_w = [C(22, [11, 11], [0, 0, 0], [1, 1, 1], list(range(22))),
              C(23, [8, 8, 7], [0, 0, 0, 1, 1, 1], [1, 1, 1, 2, 2, 2], list(range(23))),
              C(12, [6, 6], [0, 0], [1, 1], list(range(12))),
              C(9, [4, 5], [0, 0, 0], [1, 1, 1], [5, 0, 3, 8, 1, 2, 4, 7, 6]),
              C(13, [4, 5, 4], [0, 1, 1], [1, 2, 2], list(range(13)))]
    host = [[E.astype(np.float32) for E in W.random_entries(c, seed=800 + i)] for i, c in enumerate(cuts_w)]
    ents = [[torch.from_numpy(E).cuda() for E in h] for h in host]
    cuts = [cqc.CutMap.from_workload(c) for c in cuts_w]
    batch = cqc.Batch(ents, cuts, precision="fp32")
    with cqc.trace() as tr:
        batch.run()
        torch.cuda.synchronize()
    assert "wide_f32_queue" in tr.result, tr.result
    for k in range(len(cuts)):
        p1, m1 = cqc.reconstruct_fd(ents[k], cuts[k], precision="fp32")
        torch.cuda.synchronize()
        assert torch.equal(batch.outs[k], p1), k
        assert abs(float(batch.mass[k]) - float(m1)) <= 1e-12 * max(1.0, abs(float(m1))), k
    for k in (0, 1):
        xs = W.sample_outputs(cuts_w[k].n, 4096, seed=810 + k)
        got = batch.outs[k][torch.from_numpy(xs).cuda()].double().cpu().numpy()
        e64 = oracle_inputs(host[k])
        ref = native.reconstruct(e64, cuts_w[k], xs)
        T = native.reconstruct([np.abs(E) for E in e64], cuts_w[k], xs)
        err = metrics.rel_l1(got, ref)
        print(f"wide queue instance {k}: sampled rel_l1={err:.3e}")
        assert err <= 1e-6
        ok, info = elementwise_ok(got, ref, T, U32, 64 + 64)
        assert ok, (k, info)


def test_batch_fp32_wide_queue_below_single_call_threshold():
    """FP32 steps of three shared cuts with 2^19 to 2^22 outputs take the wide
    kernel inside a batch (its tiles share the launch with those of other
    steps), while a single call keeps the register kernel there.  The wide
    queue runs; those instances agree with their single calls to FP32 rounding
    (relative L1 <= 1e-6, mass within 1e-6) and with the oracle on a sample
    (relative L1 <= 1e-6 and every element within its rounding bound); an
    instance below 2^19 outputs still equals its single call bit for bit."""
    _gpu()
    from oracle import native
    from tests.gpu_util import elementwise_ok, U32
    C = W.CutMap
    cuts_w = [C(20, [10, 10], [0, 0, 0], [1, 1, 1], list(range(20))),
              C(19, [9, 10], [0, 0, 0], [1, 1, 1], list(range(19))),
              C(12, [6, 6], [0, 0, 0], [1, 1, 1], list(range(12)))]
    host = [[E.astype(np.float32) for E in W.random_entries(c, seed=820 + i)] for i, c in enumerate(cuts_w)]
    ents = [[torch.from_numpy(E).cuda() for E in h] for h in host]
    cuts = [cqc.CutMap.from_workload(c) for c in cuts_w]
    batch = cqc.Batch(ents, cuts, precision="fp32")
    with cqc.trace() as tr:
        batch.run()
        torch.cuda.synchronize()
    assert "wide_f32_queue" in tr.result, tr.result
    for k in range(len(cuts)):
        p1, m1 = cqc.reconstruct_fd(ents[k], cuts[k], precision="fp32")
        torch.cuda.synchronize()
        if k == 2:
            assert torch.equal(batch.outs[k], p1), k
            continue
        a, b = batch.outs[k].double(), p1.double()
        rel = float((a - b).abs().sum() / b.abs().sum())
        print(f"instance {k}: batch vs single call rel_l1={rel:.3e}")
        assert rel <= 1e-6, (k, rel)
        assert abs(float(batch.mass[k]) - float(m1)) <= 1e-6 * max(1.0, abs(float(m1))), k
        xs = W.sample_outputs(cuts_w[k].n, 4096, seed=830 + k)
        got = batch.outs[k][torch.from_numpy(xs).cuda()].double().cpu().numpy()
        e64 = oracle_inputs(host[k])
        ref = native.reconstruct(e64, cuts_w[k], xs)
        T = native.reconstruct([np.abs(E) for E in e64], cuts_w[k], xs)
        err = metrics.rel_l1(got, ref)
        print(f"instance {k}: sampled rel_l1 against the oracle={err:.3e}")
        assert err <= 1e-6
        ok, info = elementwise_ok(got, ref, T, U32, 64 + 64)
        assert ok, (k, info)
