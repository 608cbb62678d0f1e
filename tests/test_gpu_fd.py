"""GPU parity of the full-definition path against the FP64 oracle.

Tolerances: relative L1 <= 1e-6 for the FP32 and BF16X6 forms (the target
accuracy), <= 1e-12 for the FP64 form; in addition every element must lie
within the rounding bound 4 (t + 2) u T_x of any summation order of the t terms
it adds (t counts the six partial products per term of the BF16X6 form), with
T_x = 2^-K sum_l prod_c |E_c| computed by the oracle.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fd, metrics
from tests.gpu_util import to_dev, oracle_inputs, abs_bound, elementwise_ok, sum_terms, U32, U64

pytestmark = pytest.mark.gpu

cqc = pytest.importorskip("paper_2012_02333_amd")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_mfma_lane_layout():
    _gpu()
    f, d, b = cqc.selftest_mfma()
    i = np.arange(16)[:, None]
    j = np.arange(16)[None, :]
    ref = sum((i + 16 * k) * (1 + k + 4 * j) for k in range(4)).astype(np.float64)
    assert np.array_equal(f.numpy().astype(np.float64), ref)
    assert np.array_equal(d.numpy(), ref)
    A = (np.arange(16)[:, None] + 3 * np.arange(32)[None, :]) % 7 - 3
    B = (2 * np.arange(32)[:, None] + np.arange(16)[None, :]) % 5 - 2
    assert np.array_equal(b.numpy().astype(np.float64), (A @ B).astype(np.float64))


def _run(entries_np, wcut, dtype, prec, out_dtype=None):
    host, dev = to_dev(entries_np, dtype)
    cut = cqc.CutMap.from_workload(wcut)
    p, mass = cqc.reconstruct_fd(dev, cut, precision=prec, out_dtype=out_dtype)
    torch.cuda.synchronize()
    return host, p.cpu().numpy().astype(np.float64), float(mass.cpu())


def _inner_terms(wcut):
    cut = cqc.CutMap.from_workload(wcut)
    _, macs = cqc.cost(cut)
    return max(4, int(round(macs / 2 ** wcut.n)))


@pytest.mark.parametrize("prec,dtype,tol,unit", [("fp64", torch.float64, 1e-12, U64),
                                                 ("fp32", torch.float32, 1e-6, U32),
                                                 ("bf16x6", torch.float32, 1e-6, U32)])
@pytest.mark.parametrize("shape", [((4, 3), (1,), 4), ((5, 5), (2,), 6), ((3, 2, 3), (3, 3), 4),
                                   ((3, 3, 3), (2, 2), 6), ((2, 3, 3, 2), (1, 2, 2), 4),
                                   ((6, 6), (3,), 6), ((7, 7), (2,), 4)])
def test_fd_simulated_circuits(shape, prec, dtype, tol, unit):
    _gpu()
    own, bridges, layers = shape
    inst = W.make_instance(own, bridges, layers, seed=101)
    host, p, mass = _run(inst.entries, inst.cut, dtype, prec)
    e64 = oracle_inputs(host)
    ref = fd.reconstruct(e64, inst.cut)
    err = metrics.rel_l1(p, ref)
    print(f"{shape} {prec}: rel_l1={err:.3e}")
    assert err <= tol
    ok, info = elementwise_ok(p, ref, abs_bound(e64, inst.cut), unit, sum_terms(prec, _inner_terms(inst.cut)))
    assert ok, info
    assert abs(mass - ref.sum()) <= 1e-6 * np.abs(ref).sum()


@pytest.mark.parametrize("prec,dtype,unit", [("fp64", torch.float64, U64), ("fp32", torch.float32, U32),
                                             ("bf16x6", torch.float32, U32)])
@pytest.mark.parametrize("case", ["perm", "kron2", "kron3", "single", "triangle", "ragged",
                                  "zero_rows", "k0_f0"])
def test_fd_random_structures(case, prec, dtype, unit):
    _gpu()
    C = W.CutMap
    if case == "perm":          # outputs scattered over the global order
        cut = C(9, [4, 5], [0, 0], [1, 1], [5, 0, 3, 8, 1, 2, 4, 7, 6])
    elif case == "kron2":       # disconnected: plain Kronecker product
        cut = C(7, [3, 4], [], [], list(range(7)))
    elif case == "kron3":
        cut = C(9, [2, 3, 4], [0], [1], list(range(9)))
    elif case == "single":
        cut = C(6, [6], [], [], [3, 1, 0, 5, 2, 4])
    elif case == "triangle":    # cyclic subcircuit graph, reversed edge directions
        cut = C(12, [4, 4, 4], [0, 1, 2, 0], [1, 2, 0, 1], list(range(12)))
    elif case == "ragged":      # tiny and odd tile shapes: 1, 2, 8 wide operands
        cut = C(11, [1, 2, 8], [0, 1, 1, 2], [1, 2, 2, 0], list(range(11)))
    elif case == "zero_rows":   # early termination: some rows exactly zero
        cut = C(10, [5, 5], [0, 0, 0], [1, 1, 1], list(range(10)))
    else:                       # a subcircuit with no output qubit
        cut = C(8, [0, 8], [0, 0], [1, 1], list(range(8)))
    zr = ((0, 3), (0, 17), (1, 40), (1, 0)) if case == "zero_rows" else ()
    seed = ["perm", "kron2", "kron3", "single", "triangle", "ragged", "zero_rows", "k0_f0"].index(case)
    ents = W.random_entries(cut, seed=100 + seed, zero_rows=zr)
    host, p, mass = _run(ents, cut, dtype, prec)
    e64 = oracle_inputs(host)
    ref = fd.reconstruct(e64, cut)
    T = abs_bound(e64, cut)
    ok, info = elementwise_ok(p, ref, T, unit, sum_terms(prec, 4 ** cut.n_cuts))
    assert ok, (case, info)
    # the flat bar of the precision; kappa (up to 13 here) is printed as a
    # diagnostic of how much cancellation the random signed entries carry
    tol = 1e-12 if prec == "fp64" else 1e-6
    err, kap = metrics.rel_l1(p, ref), metrics.kappa(e64, cut, np.abs(ref).sum())
    print(f"{case} {prec}: rel_l1={err:.3e} kappa={kap:.2f}")
    assert err <= tol


def test_fd_c1_plain_fp64():
    _gpu()
    inst = W.config_instance("c1")
    host, p, mass = _run(inst.entries, inst.cut, torch.float64, "fp64")
    ref = fd.reconstruct(inst.entries, inst.cut)
    assert metrics.rel_l1(p, ref) <= 1e-13
    assert abs(mass - 1.0) <= 1e-13


@pytest.mark.parametrize("prec,dtype,tol", [("fp32", torch.float32, 1e-6), ("fp64", torch.float64, 1e-12),
                                            ("bf16x6", torch.float32, 1e-6)])
def test_fd_c2_full_vector(prec, dtype, tol):
    """n=24, K=2, two 13-qubit subcircuits: the headline shape, all 2^24 outputs."""
    _gpu()
    inst = W.config_instance("c2")
    host, p, mass = _run(inst.entries, inst.cut, dtype, prec)
    e64 = oracle_inputs(host)
    from oracle import native
    ref = native.reconstruct(e64, inst.cut)
    err = metrics.rel_l1(p, ref)
    print(f"c2 {prec}: rel_l1={err:.3e} mass={mass!r}")
    assert err <= tol
    T = native.reconstruct([np.abs(E) for E in e64], inst.cut)
    ok, info = elementwise_ok(p, ref, T, U64 if prec == "fp64" else U32, sum_terms(prec, 16))
    assert ok, info
    # the mass is the FP64 sum of the written outputs
    assert abs(mass - p.sum()) <= 1e-12 * np.abs(p).sum()
    # FP32/FP64 roundings are unbiased and cancel in the sum; the BF16 matrix
    # cores' are not, so there only the L1 bound holds
    assert abs(mass - ref.sum()) <= (tol * np.abs(ref).sum() if prec == "bf16x6" else 1e-9)


@pytest.mark.parametrize("prec", ["fp32", "bf16x6"])
def test_fd_c3_sampled(prec):
    """n=30, K=6, three subcircuits (2^30 outputs): sampled outputs against the
    oracle's per-output definition, plus the FP64 mass."""
    _gpu()
    inst = W.config_instance("c3")
    host, dev = to_dev(inst.entries, torch.float32)
    cut = cqc.CutMap.from_workload(inst.cut)
    p, mass = cqc.reconstruct_fd(dev, cut, precision=prec)
    xs = W.sample_outputs(inst.n, 4096, seed=33)
    got = p[torch.from_numpy(xs).to("cuda")].cpu().numpy().astype(np.float64)
    e64 = oracle_inputs(host)
    ref = fd.reconstruct(e64, inst.cut, xs)
    err = metrics.rel_l1(got, ref)
    print(f"c3 {prec} sampled rel_l1={err:.3e} mass={float(mass.cpu())!r}")
    assert err <= 1e-6
    assert abs(float(mass.cpu()) - 1.0) <= 1e-5
    ok, info = elementwise_ok(got, ref, abs_bound(e64, inst.cut, xs), U32, sum_terms(prec, 64 + 64))
    assert ok, info
    del p


@pytest.mark.parametrize("prec", ["fp32", "bf16x6"])
def test_fd_c3_full_vector(prec):
    """n=30, K=6, three subcircuits: all 2^30 outputs against the blocked FP64
    oracle, 16 blocks of 2^26 (each a contiguous range of the global vector),
    so the relative L1 error is the whole vector's, with every element inside
    its rounding bound."""
    _gpu()
    from oracle import blocked
    inst = W.config_instance("c3")
    host, dev = to_dev(inst.entries, torch.float32)
    cut = cqc.CutMap.from_workload(inst.cut)
    p, mass = cqc.reconstruct_fd(dev, cut, precision=prec)
    torch.cuda.synchronize()
    e64 = oracle_inputs(host)
    a64 = [np.abs(E) for E in e64]
    top = 4
    span = 2 ** (inst.n - top)
    num = den = 0.0
    worst = 0.0
    for b in range(2 ** top):
        got = p[b * span:(b + 1) * span].cpu().numpy().astype(np.float64)
        ref = blocked.reconstruct_block(e64, inst.cut, top, b)
        T = blocked.reconstruct_block(a64, inst.cut, top, b)
        err = np.abs(got - ref)
        num += float(err.sum())
        den += float(np.abs(ref).sum())
        tol = 4.0 * (sum_terms(prec, 64 + 64) + 2) * U32 * T
        worst = max(worst, float(np.max(err / tol)))
    rel = num / den
    print(f"c3 {prec} full-vector rel_l1={rel:.3e} worst err/bound={worst:.3f} mass={float(mass.cpu())!r}")
    assert rel <= 1e-6
    assert worst <= 1.0
    assert abs(float(mass.cpu()) - 1.0) <= 1e-5
    del p


def test_fd_bitwise_repeatable():
    _gpu()
    inst = W.make_instance((6, 6), (3,), 6, seed=5)
    host, dev = to_dev(inst.entries, torch.float32)
    cut = cqc.CutMap.from_workload(inst.cut)
    a, ma = cqc.reconstruct_fd(dev, cut, precision="fp32")
    b, mb = cqc.reconstruct_fd(dev, cut, precision="fp32")
    assert torch.equal(a, b) and torch.equal(ma, mb)


@pytest.mark.parametrize("in_dt,out_dt,prec", [(torch.float32, torch.float64, "fp64"),
                                              (torch.float64, torch.float32, "fp32"),
                                              (torch.float32, torch.float64, "fp32")])
def test_fd_mixed_dtypes(in_dt, out_dt, prec):
    _gpu()
    inst = W.make_instance((5, 5), (2,), 6, seed=9)
    host, dev = to_dev(inst.entries, in_dt)
    cut = cqc.CutMap.from_workload(inst.cut)
    p, mass = cqc.reconstruct_fd(dev, cut, precision=prec, out_dtype=out_dt)
    assert p.dtype == out_dt
    ref = fd.reconstruct(oracle_inputs(host), inst.cut)
    assert metrics.rel_l1(p.cpu().numpy().astype(np.float64), ref) <= 1e-6


@pytest.mark.parametrize("prec,shape", [("fp32", ((6, 6), (2,), 6)), ("fp64", ((4, 4), (3,), 6)),
                                        ("bf16x6", ((6, 6), (3,), 6)), ("fp32", ((4, 4), (3,), 6))])
def test_fd_mass_fresh_across_calls(prec, shape):
    """The FP64 mass is the ordered sum of per-tile partials that the last
    contraction writes, added by a separate final pass: the same prepared call,
    run again after the entries are scaled by 2 in place, must report exactly
    twice the mass (outputs scale exactly by 2, and the partials are added in
    the same order), so no partial or total survives from the previous run."""
    _gpu()
    own, bridges, layers = shape
    inst = W.make_instance(own, bridges, layers, seed=21)
    dt = torch.float64 if prec == "fp64" else torch.float32
    host, dev = to_dev(inst.entries, dt)
    cut = cqc.CutMap.from_workload(inst.cut)
    call = cqc.FDCall(dev, cut, precision=prec)
    masses = []
    for rep in range(3):
        call.run()
        torch.cuda.synchronize()
        p = call.outs[0].double().cpu().numpy()
        m = float(call.mass[0].cpu())
        assert abs(m - p.sum()) <= 1e-12 * np.abs(p).sum(), (rep, m, p.sum())
        masses.append(m)
        dev[0].mul_(2.0)
    assert masses[1] == 2.0 * masses[0] and masses[2] == 2.0 * masses[1], masses


def _traced_fd(dev, cut, **kw):
    with cqc.trace() as tr:
        p, mass = cqc.reconstruct_fd(dev, cut, **kw)
        torch.cuda.synchronize()
    return p, mass, tr.result


@pytest.mark.parametrize("out_dt", [torch.float32, torch.float64])
def test_fd_small_k_two_tile_strips(out_dt):
    """Two 9-qubit subcircuits, two cuts (16 terms over 512 x 512 outputs):
    with FP32 output the FP32 small-term contraction runs as two-tile strips
    (Y operands loaded once per strip); FP32 and FP64 outputs, element by
    element."""
    _gpu()
    cut = W.CutMap(18, [9, 9], [0, 0], [1, 1], list(range(18)))
    host, dev = to_dev(W.random_entries(cut, seed=61), torch.float32)
    p, mass, kt = _traced_fd(dev, cqc.CutMap.from_workload(cut), precision="fp32", out_dtype=out_dt)
    # FP64 output keeps the one-tile kernel (its stores are not staged)
    assert ("contract_small_strip_64x256" in kt) == (out_dt == torch.float32), kt
    e64 = oracle_inputs(host)
    ref = fd.reconstruct(e64, cut)
    got = p.double().cpu().numpy()
    assert metrics.rel_l1(got, ref) <= 1e-6
    ok, info = elementwise_ok(got, ref, abs_bound(e64, cut), U32, sum_terms("fp32", 16))
    assert ok, info
    assert abs(float(mass.cpu()) - ref.sum()) <= 1e-6 * np.abs(ref).sum()


def test_fd_small_k_strip_chain():
    """Three 8-qubit subcircuits in a chain, two cuts per boundary: both
    contractions have 16 terms; the first writes a batched intermediate
    (16 batches of 256 x 256) through the two-tile strips."""
    _gpu()
    cut = W.CutMap(24, [8, 8, 8], [0, 0, 1, 1], [1, 1, 2, 2], list(range(24)))
    host, dev = to_dev(W.random_entries(cut, seed=62), torch.float32)
    p, mass, kt = _traced_fd(dev, cqc.CutMap.from_workload(cut), precision="fp32")
    assert "contract_small_strip_64x256" in kt, kt
    xs = W.sample_outputs(24, 4096, seed=62)
    got = p[torch.from_numpy(xs).to("cuda")].double().cpu().numpy()
    e64 = oracle_inputs(host)
    ref = fd.reconstruct(e64, cut, xs)
    assert metrics.rel_l1(got, ref) <= 1e-6
    ok, info = elementwise_ok(got, ref, abs_bound(e64, cut, xs), U32, sum_terms("fp32", 16 + 16))
    assert ok, info
