"""The two-part split-BF16 form (BF16X3: a = a0 + a1, products a_i b_j with
i + j <= 1) against the FP64 oracle, and its place between BF16X6 and FP32.

Bars, derived from the split: the remainder after two parts is at most
2^-17 |a| and the second part at most 2^-8 |a|, so the dropped product a1 b1
and the remainders leave at most 2^-15 = 512 u of |a b| per product (bounds
checked on the host in test_split_bound); elementwise |p - ref| <=
4 (3 t + 130) u T_x (gpu_util.sum_terms) and relative L1 <= 3.1e-5 kappa.  Steps with at most 16 terms run FP32 under BF16X3 as under
BF16X6, so the cases here have three or more shared cuts where it matters.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fd, metrics
from tests.gpu_util import to_dev, oracle_inputs, abs_bound, elementwise_ok, sum_terms, U32, REL_L1

pytestmark = pytest.mark.gpu
cqc = pytest.importorskip("paper_2012_02333_amd")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _inner_terms(wcut):
    _, macs = cqc.cost(cqc.CutMap.from_workload(wcut))
    return max(4, int(round(macs / 2 ** wcut.n)))


@pytest.mark.parametrize("shape", [((3, 2, 3), (3, 3), 4), ((6, 6), (3,), 6), ((5, 5), (4,), 4),
                                   ((4, 4, 4), (3, 2), 6)])
def test_bf16x3_simulated_circuits(shape):
    _gpu()
    own, bridges, layers = shape
    inst = W.make_instance(own, bridges, layers, seed=102)
    host, dev = to_dev(inst.entries, torch.float32)
    p, mass = cqc.reconstruct_fd(dev, cqc.CutMap.from_workload(inst.cut), precision="bf16x3")
    got = p.double().cpu().numpy()
    e64 = oracle_inputs(host)
    ref = fd.reconstruct(e64, inst.cut)
    kap = metrics.kappa(e64, inst.cut, np.abs(ref).sum())
    err = metrics.rel_l1(got, ref)
    print(f"{shape} bf16x3: rel_l1={err:.3e} kappa={kap:.2f}")
    assert err <= REL_L1["bf16x3"] * max(1.0, kap)
    ok, info = elementwise_ok(got, ref, abs_bound(e64, inst.cut), U32, sum_terms("bf16x3", _inner_terms(inst.cut)))
    assert ok, info
    assert abs(float(mass.cpu()) - ref.sum()) <= REL_L1["bf16x3"] * max(1.0, kap) * np.abs(ref).sum()


def test_bf16x3_runs_the_two_part_kernel_and_sits_between():
    """Five shared cuts (1024 terms): BF16X3 runs its own wide kernel, is less
    accurate than BF16X6 and FP32 (its split keeps 16 of 24 significand bits)
    and still inside its bar."""
    _gpu()
    cut = W.CutMap(16, [8, 8], [0] * 5, [1] * 5, list(range(16)))
    ents = W.random_entries(cut, seed=47)
    host, dev = to_dev(ents, torch.float32)
    c = cqc.CutMap.from_workload(cut)
    e64 = oracle_inputs(host)
    ref = fd.reconstruct(e64, cut)
    errs = {}
    for prec in ("fp32", "bf16x6", "bf16x3"):
        with cqc.trace() as tr:
            p, _ = cqc.reconstruct_fd(dev, c, precision=prec)
            torch.cuda.synchronize()
        errs[prec] = metrics.rel_l1(p.double().cpu().numpy(), ref)
        if prec == "bf16x3":
            assert any(k.startswith("wide_bf16x3") for k in tr.result), list(tr.result)
            assert not any(k.startswith("wide_bf16x6") for k in tr.result)
    kap = metrics.kappa(e64, cut, np.abs(ref).sum())
    print(errs, kap)
    assert errs["bf16x3"] > 4 * max(errs["bf16x6"], errs["fp32"])
    assert errs["bf16x3"] <= REL_L1["bf16x3"] * max(1.0, kap)


def test_bf16x3_c3_sampled():
    """n=30, K=6: sampled outputs against the oracle's per-output definition."""
    _gpu()
    inst = W.config_instance("c3")
    host, dev = to_dev(inst.entries, torch.float32)
    p, mass = cqc.reconstruct_fd(dev, cqc.CutMap.from_workload(inst.cut), precision="bf16x3")
    xs = W.sample_outputs(inst.n, 4096, seed=34)
    got = p[torch.from_numpy(xs).to("cuda")].cpu().numpy().astype(np.float64)
    e64 = oracle_inputs(host)
    ref = fd.reconstruct(e64, inst.cut, xs)
    T = abs_bound(e64, inst.cut, xs)
    err = metrics.rel_l1(got, ref)
    print(f"c3 bf16x3 sampled rel_l1={err:.3e} kappa_sample={T.sum() / np.abs(ref).sum():.2f}")
    assert err <= REL_L1["bf16x3"] * max(1.0, T.sum() / np.abs(ref).sum())
    ok, info = elementwise_ok(got, ref, T, U32, sum_terms("bf16x3", 64 + 64))
    assert ok, info
    del p


def test_bf16x3_dd_and_adjoint_fallback():
    """DD accepts BF16X3 (bins within its bar); the adjoint has no split form
    and refuses it, while the autograd wrapper differentiates in FP32."""
    _gpu()
    from oracle import dd
    inst = W.make_instance((4, 4, 4), (3, 2), 6, seed=103)
    host, dev = to_dev(inst.entries, torch.float32)
    cut = cqc.CutMap.from_workload(inst.cut)
    bins, recs = cqc.reconstruct_dd(dev, cut, 5, 3, precision="bf16x3")
    e64 = oracle_inputs(host)
    ref = dd.reconstruct(e64, inst.cut, 5, 3, chooser=lambda records, expanded: tuple(recs[len(records)]["parent"]))
    for r, o in enumerate(ref):
        merged = dd.merge_entries(e64, inst.cut, o["role"])
        T = dd.bins_from_merged([np.abs(m) for m in merged], inst.cut, o["role"])
        got = bins[r, :len(o["bins"])].cpu().numpy()
        assert metrics.rel_l1(got, o["bins"]) <= REL_L1["bf16x3"] * max(1.0, T.sum() / np.abs(o["bins"]).sum())
    g = torch.ones(2 ** inst.n, dtype=torch.float32, device="cuda")
    with pytest.raises(cqc.CqcError) as e:
        cqc.reconstruct_backward(dev, cut, g, precision="bf16x3")
    assert e.value.code == 3
    leaves = [E.clone().requires_grad_(True) for E in dev]
    p = cqc.ReconstructFD.apply(cut, "bf16x3", *leaves)
    p.sum().backward()
    ref_g = cqc.reconstruct_backward([E.detach() for E in leaves], cut, torch.ones_like(p), precision="fp32")
    for a, b in zip(leaves, ref_g):
        assert torch.equal(a.grad, b)
