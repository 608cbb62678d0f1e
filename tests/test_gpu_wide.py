"""GPU parity of the LDS-staged wide contraction kernel (FP32 and BF16X6 forms)
on the shapes that reach it: long term sums (three or more shared cut labels)
over operands at least 128 columns wide with at least 2^22 outputs per step
(fewer run the register kernel in FP32: the same cases then check that one),
and any shape in the BF16X6 form.

Cases cover more live labels than one 256-label compaction chunk, chunks left
partial by early termination, scattered (bit-deposit) output orders, chained
contractions whose intermediate tensor is written by the wide kernel, and FP64
output from FP32 arithmetic.  Tolerances as in test_gpu_fd.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fd, metrics
from tests.gpu_util import to_dev, oracle_inputs, abs_bound, elementwise_ok, sum_terms, U32, REL_L1

pytestmark = pytest.mark.gpu
cqc = pytest.importorskip("paper_2012_02333_amd")

PRECS = ["fp32", "bf16x6", "bf16x3"]


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _check(cut, ents, prec, xs=None, out_dtype=None):
    host, dev = to_dev(ents, torch.float32)
    p, mass = cqc.reconstruct_fd(dev, cqc.CutMap.from_workload(cut), precision=prec, out_dtype=out_dtype)
    e64 = oracle_inputs(host)
    if xs is None:
        got = p.double().cpu().numpy()
    else:
        got = p[torch.from_numpy(xs).to("cuda")].double().cpu().numpy()
    ref = fd.reconstruct(e64, cut, xs)
    err = metrics.rel_l1(got, ref)
    kap = metrics.kappa(e64, cut, np.abs(ref).sum()) if xs is None else 1.0
    print(f"{prec}: rel_l1={err:.3e} kappa={kap:.2f}")
    # FP32 and BF16X6: the flat 1e-6 bar (kappa is a diagnostic); BF16X3's
    # bar is its dropped part, at most 2^-15 = 3.05e-5 of T_x, hence
    # kappa-scaled
    bar = REL_L1[prec] * (max(1.0, kap) if prec == "bf16x3" else 1.0)
    assert err <= bar
    ok, info = elementwise_ok(got, ref, abs_bound(e64, cut, xs), U32, sum_terms(prec, 4 ** cut.n_cuts))
    assert ok, info
    if xs is None:
        assert abs(float(mass.cpu()) - ref.sum()) <= bar * np.abs(ref).sum()
    return p


@pytest.mark.parametrize("prec", PRECS)
def test_wide_many_labels_with_dead_rows(prec):
    """Five shared cuts: 1024 labels in four compaction chunks; dead rows in
    both operands leave chunks whose live count is not a multiple of 32."""
    _gpu()
    cut = W.CutMap(16, [8, 8], [0] * 5, [1] * 5, list(range(16)))
    zr = ((0, 5), (0, 6), (0, 300), (0, 1023), (1, 0), (1, 17), (1, 511), (1, 512))
    ents = W.random_entries(cut, seed=41, zero_rows=zr)
    _check(cut, ents, prec)


@pytest.mark.parametrize("prec", PRECS)
def test_wide_scattered_output(prec):
    """Bit-deposit output order (subcircuit bits interleaved in the global index)."""
    _gpu()
    rng = np.random.default_rng(7)
    perm = [int(q) for q in rng.permutation(16)]
    cut = W.CutMap(16, [8, 8], [0, 0, 0], [1, 1, 1], perm)
    _check(cut, W.random_entries(cut, seed=42), prec)


@pytest.mark.parametrize("prec", PRECS)
def test_wide_chain_intermediate(prec):
    """Three subcircuits, three cuts per boundary: the first contraction writes
    a batched intermediate (64 batches of 128 x 128) that the last one reads."""
    _gpu()
    cut = W.CutMap(21, [7, 7, 7], [0, 0, 0, 1, 1, 1], [1, 1, 1, 2, 2, 2], list(range(21)))
    xs = W.sample_outputs(21, 4096, seed=43)
    _check(cut, W.random_entries(cut, seed=43), prec, xs=xs)


def test_wide_fp64_output():
    _gpu()
    cut = W.CutMap(16, [8, 8], [0, 0, 0], [1, 1, 1], list(range(16)))
    p = _check(cut, W.random_entries(cut, seed=44), "fp32", out_dtype=torch.float64)
    assert p.dtype == torch.float64


@pytest.mark.parametrize("prec", PRECS)
def test_wide_bitwise_repeatable(prec):
    _gpu()
    cut = W.CutMap(16, [8, 8], [0] * 4, [1] * 4, list(range(16)))
    host, dev = to_dev(W.random_entries(cut, seed=45), torch.float32)
    c = cqc.CutMap.from_workload(cut)
    a, ma = cqc.reconstruct_fd(dev, c, precision=prec)
    b, mb = cqc.reconstruct_fd(dev, c, precision=prec)
    assert torch.equal(a, b) and torch.equal(ma, mb)


def test_bf16x6_split_is_exact_enough():
    """Values whose FP32 significand needs all 24 bits (and a power-of-two
    spread of magnitudes) keep FP32 accuracy through the three-part split."""
    _gpu()
    cut = W.CutMap(10, [5, 5], [0, 0, 0], [1, 1, 1], list(range(10)))
    rng = np.random.default_rng(46)
    ents = []
    for c in range(2):
        E = (1.0 + rng.random((64, 32))) * np.exp2(rng.integers(-30, 30, size=(64, 32)))
        E *= rng.choice([-1.0, 1.0], size=E.shape)
        ents.append(E.astype(np.float32).astype(np.float64))
    host, dev = to_dev(ents, torch.float32)
    p, _ = cqc.reconstruct_fd(dev, cqc.CutMap.from_workload(cut), precision="bf16x6")
    e64 = oracle_inputs(host)
    ref = fd.reconstruct(e64, cut)
    ok, info = elementwise_ok(p.double().cpu().numpy(), ref, abs_bound(e64, cut), U32, sum_terms("bf16x6", 64))
    assert ok, info


def _wide_ran(kt, final=True):
    return any(k.startswith("wide_f32_final" if final else "wide_f32_inter") for k in kt)


def test_wide_fp32_pair_at_2p22_outputs():
    """Two 11-qubit subcircuits, three cuts: 2^22 outputs reach the FP32 wide
    kernel; sampled outputs against the oracle, plus the FP64 mass."""
    _gpu()
    cut = W.CutMap(22, [11, 11], [0, 0, 0], [1, 1, 1], list(range(22)))
    host, dev = to_dev(W.random_entries(cut, seed=47), torch.float32)
    with cqc.trace() as tr:
        p, mass = cqc.reconstruct_fd(dev, cqc.CutMap.from_workload(cut), precision="fp32")
        torch.cuda.synchronize()
    assert _wide_ran(tr.result), tr.result
    xs = W.sample_outputs(22, 4096, seed=47)
    got = p[torch.from_numpy(xs).to("cuda")].double().cpu().numpy()
    e64 = oracle_inputs(host)
    ref = fd.reconstruct(e64, cut, xs)
    assert metrics.rel_l1(got, ref) <= 1e-6
    ok, info = elementwise_ok(got, ref, abs_bound(e64, cut, xs), U32, sum_terms("fp32", 64))
    assert ok, info


def test_wide_fp32_chain_intermediate_and_final():
    """Three 8-qubit subcircuits, three cuts per boundary: the intermediate
    (64 batches of 256 x 256) and the final contraction (2^24 outputs) both run
    on the FP32 wide kernel; sampled outputs against the oracle."""
    _gpu()
    cut = W.CutMap(24, [8, 8, 8], [0, 0, 0, 1, 1, 1], [1, 1, 1, 2, 2, 2], list(range(24)))
    host, dev = to_dev(W.random_entries(cut, seed=48), torch.float32)
    with cqc.trace() as tr:
        p, mass = cqc.reconstruct_fd(dev, cqc.CutMap.from_workload(cut), precision="fp32")
        torch.cuda.synchronize()
    assert _wide_ran(tr.result) and _wide_ran(tr.result, final=False), tr.result
    xs = W.sample_outputs(24, 4096, seed=48)
    got = p[torch.from_numpy(xs).to("cuda")].double().cpu().numpy()
    e64 = oracle_inputs(host)
    ref = fd.reconstruct(e64, cut, xs)
    assert metrics.rel_l1(got, ref) <= 1e-6
    ok, info = elementwise_ok(got, ref, abs_bound(e64, cut, xs), U32, sum_terms("fp32", 64 + 64))
    assert ok, info
