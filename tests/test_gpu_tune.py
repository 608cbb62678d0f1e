"""The project's tile autotuner: tuned plans stay correct, the shape-class
cache round-trips through the CQC_TUNE_CACHE file, and a cache entry really
changes the kernel the planner launches."""
import os

import numpy as np
import pytest
import torch

import workloads as W
from oracle import fd, metrics
from tests.gpu_util import to_dev, oracle_inputs, abs_bound, elementwise_ok, sum_terms, U32

pytestmark = pytest.mark.gpu
cqc = pytest.importorskip("paper_2012_02333_amd")

# key fields of a cache line: acc (0 = FP32), mode (1 = blocked final),
# small (<= 16 terms), log2 M, log2 N, shared cuts, FP64 output; then tile
# (0 64x256, 1 32x128, 2 16x64, 3 256x16, 4 wide), XCD remap, microseconds


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture
def tune_env(tmp_path):
    old = os.environ.get("CQC_TUNE_CACHE")
    path = str(tmp_path / "tune.txt")
    os.environ["CQC_TUNE_CACHE"] = path
    cqc.tune_reset()
    yield path
    if old is None:
        del os.environ["CQC_TUNE_CACHE"]
    else:
        os.environ["CQC_TUNE_CACHE"] = old
    cqc.tune_reset()


def _check(p, host, wcut, xs=None):
    e64 = oracle_inputs(host)
    ref = fd.reconstruct(e64, wcut, xs)
    got = p.double().cpu().numpy() if xs is None else p[torch.from_numpy(xs).cuda()].double().cpu().numpy()
    ok, info = elementwise_ok(got, ref, abs_bound(e64, wcut, xs), U32, sum_terms("fp32", 4 ** wcut.n_cuts))
    assert ok, info
    return metrics.rel_l1(got, ref)


def test_autotuned_chain_stays_correct(tune_env):
    """n=23, three subcircuits, 4096 terms (a wide-kernel step): tune, then
    check sampled outputs and bitwise repeatability; the cache file holds a
    valid line for every tuned shape class."""
    _gpu()
    inst = W.make_instance((6, 5, 6), (3, 3), 6, seed=82)
    host, dev = to_dev(inst.entries, torch.float32)
    cut = cqc.CutMap.from_workload(inst.cut)
    call = cqc.FDCall(dev, cut, precision="fp32")
    cqc.autotune(call)
    call.run()
    a = call.outs[0].clone()
    call.run()
    assert torch.equal(a, call.outs[0])
    xs = W.sample_outputs(inst.n, 2048, seed=83)
    assert _check(a, host, inst.cut, xs) <= 1e-6
    lines = [l.split() for l in open(tune_env).read().splitlines() if l.strip()]
    assert len(lines) >= 2
    for f in lines:
        assert len(f) == 10
        assert 0 <= int(f[7]) <= 4 and int(f[8]) in (0, 1) and float(f[9]) > 0
    # a fresh load of the file gives the same plan and output
    cqc.tune_reset()
    call.run()
    assert torch.equal(a, call.outs[0])


def test_cache_entry_changes_the_kernel(tune_env):
    """f = (7, 9), two cuts: by default the two-tile strip kernel; a cache line
    for its shape class naming the 16 x 64 tile makes the planner launch that
    one instead, with a correct result either way."""
    _gpu()
    inst = W.make_instance((7, 7), (2,), 6, seed=84)
    assert list(inst.cut.f) == [7, 9]
    host, dev = to_dev(inst.entries, torch.float32)
    cut = cqc.CutMap.from_workload(inst.cut)
    with cqc.trace() as tr:
        p, _ = cqc.reconstruct_fd(dev, cut, precision="fp32")
        torch.cuda.synchronize()
    assert any(k.startswith("contract_small_strip") for k in tr.result), list(tr.result)
    _check(p, host, inst.cut)
    with open(tune_env, "w") as fh:
        fh.write("0 1 1 7 9 2 0 2 0 1.000\n")
    cqc.tune_reset()
    with cqc.trace() as tr:
        q, _ = cqc.reconstruct_fd(dev, cut, precision="fp32")
        torch.cuda.synchronize()
    assert "contract_small_16x64" in tr.result and not any(k.startswith("contract_small_strip") for k in tr.result)
    _check(q, host, inst.cut)


def test_wide_entry_skipped_where_operands_do_not_fit(tune_env):
    """A cache line names the wide tile for a shape class; a step of that class
    whose operand has a single column (a subcircuit without output qubits)
    cannot run the wide kernel, so the planner keeps its built-in tile and the
    result is still the oracle's."""
    _gpu()
    cut = W.CutMap(9, [0, 9], [0], [1], list(range(9)))
    rng = np.random.default_rng(85)
    host = [rng.standard_normal((4, 1)), rng.standard_normal((4, 2 ** 9))]
    dev = [torch.from_numpy(e).float().cuda() for e in host]
    with open(tune_env, "w") as fh:
        for mode in (1, 2):
            for lm, ln in ((0, 9), (9, 0)):
                fh.write(f"0 {mode} 1 {lm} {ln} 1 0 4 0 1.000\n")
    cqc.tune_reset()
    with cqc.trace() as tr:
        p, _ = cqc.reconstruct_fd(dev, cqc.CutMap.from_workload(cut), precision="fp32")
        torch.cuda.synchronize()
    assert not any("wide" in k for k in tr.result), list(tr.result)
    e64 = [np.asarray(e, dtype=np.float32).astype(np.float64) for e in host]
    ref = fd.reconstruct(e64, cut)
    ok, info = elementwise_ok(p.double().cpu().numpy(), ref, abs_bound(e64, cut), U32, sum_terms("fp32", 4))
    assert ok, info


def test_cache_entry_changes_the_batched_kernel(tune_env):
    """The batched launch consults the same shape-class cache: two instances
    with f = (7, 9) and two cuts run the two-tile strip queue by default; a
    cache line naming the 16 x 64 tile for that class makes the batch run the
    16 x 64 work-queue kernel, every output equal to the (equally tuned)
    one-instance call and within the oracle's rounding bound."""
    _gpu()
    insts = [W.make_instance((7, 7), (2,), 6, seed=86 + k) for k in range(2)]
    assert all(list(i.cut.f) == [7, 9] for i in insts)
    hosts, devs = zip(*[to_dev(i.entries, torch.float32) for i in insts])
    cuts = [cqc.CutMap.from_workload(i.cut) for i in insts]

    def run_batch():
        b = cqc.Batch([list(d) for d in devs], cuts, precision="fp32")
        with cqc.trace() as tr:
            b.run()
            torch.cuda.synchronize()
        return b, tr.result
    b0, kt0 = run_batch()
    assert "contract_strip_queue" in kt0, list(kt0)
    with open(tune_env, "w") as fh:
        fh.write("0 1 1 7 9 2 0 2 0 1.000\n")
    cqc.tune_reset()
    b1, kt1 = run_batch()
    assert "contract_small_queue" in kt1 and "contract_strip_queue" not in kt1, list(kt1)
    for k, inst in enumerate(insts):
        p1, _ = cqc.reconstruct_fd(list(devs[k]), cuts[k], precision="fp32")
        torch.cuda.synchronize()
        assert torch.equal(b1.outs[k], p1), k
        assert _check(b1.outs[k], hosts[k], inst.cut) <= 1e-6
        assert _check(b0.outs[k], hosts[k], inst.cut) <= 1e-6
