"""On-device entry construction (cqc_build_entries) against the oracle's
entries_from_variants on the same stacked variant distributions.

Bar: FP64 in and out within 1e-13 of the oracle's largest |term| sum;
FP32 output within one FP32 rounding of the FP64 result (the kernel adds in
FP64 and rounds once).  Inputs: simulated variants of bridged chains (where
the result must also equal the operator-route entries and, reconstructed, the
uncut circuit's state-vector distribution) and seeded finite-shot or
synthetic variants with interleaved cut orders and the largest supported cut
counts.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import variants, fd, metrics, statevector as sv

pytestmark = pytest.mark.gpu
cqc = pytest.importorskip("paper_2012_02333_amd")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _check(V, kinds, in_dt, out_dt):
    Vd = torch.from_numpy(V).to(device="cuda", dtype=in_dt).contiguous()
    (E,) = cqc.build_entries([(Vd, kinds)], out_dtype=out_dt)
    torch.cuda.synchronize()
    ref = variants.entries_from_variants(Vd.double().cpu().numpy(), kinds)
    got = E.double().cpu().numpy()
    scale = np.max(np.abs(ref)) + 1.0
    if out_dt == torch.float64:
        assert np.max(np.abs(got - ref)) <= 1e-13 * scale
    else:
        # one rounding to FP32 of the FP64 sum
        assert np.all(np.abs(got - ref) <= 2.0 ** -24 * np.abs(ref) + 1e-13 * scale)
    return got, ref


@pytest.mark.parametrize("own,bridges,layers", [((3, 3), (2,), 6), ((3, 2, 3), (2, 1), 4), ((2, 3, 2), (3, 2), 4)])
def test_simulated_variants_chain_end_to_end(own, bridges, layers):
    """Simulated variants of every subcircuit -> entries on the GPU (FP64):
    equal to the oracle, to the independent operator-route entries, and
    reconstructed on the GPU equal to the uncut circuit's distribution."""
    _gpu()
    circ = W.bridged_chain(own, bridges, layers, seed=17)
    cut = circ.cut_map()
    subs = circ.subcircuits()
    jobs, Vs = [], []
    for sub in subs:
        V = variants.variant_tensor(circ, sub)
        kinds = [0] * len(sub.q_in) + [1] * len(sub.q_out)
        jobs.append((torch.from_numpy(V).cuda(), kinds))
        Vs.append((V, kinds))
    Es = cqc.build_entries(jobs)
    torch.cuda.synchronize()
    gen = W.circuit_entries(circ)
    for E, (V, kinds), g in zip(Es, Vs, gen):
        got = E.cpu().numpy()
        assert np.max(np.abs(got - variants.entries_from_variants(V, kinds))) < 1e-13
        assert np.max(np.abs(got - g)) < 1e-12
    p, mass = cqc.reconstruct_fd(Es, cqc.CutMap.from_workload(cut), precision="fp64")
    truth = sv.uncut_distribution(circ)
    assert metrics.rel_l1(p.cpu().numpy(), truth) < 1e-12


@pytest.mark.parametrize("kinds", [[1], [0], [1, 0], [0, 1, 1], [1, 0, 1, 0], [0, 0, 0, 1, 1],
                                   [1, 0, 1, 1, 1], []])
@pytest.mark.parametrize("in_dt,out_dt", [(torch.float64, torch.float64), (torch.float32, torch.float32),
                                          (torch.float32, torch.float64), (torch.float64, torch.float32)])
def test_shot_and_synthetic_variants(kinds, in_dt, out_dt):
    """Finite-shot (seeded multinomial) variants in any cut order, up to three
    incoming and up to four outgoing cuts, every dtype pair; no cut at all
    copies the distribution."""
    _gpu()
    k_in, k_out = kinds.count(0), kinds.count(1)
    f = 5 if k_in + k_out >= 5 else 7
    V = W.random_variants(k_in, k_out, f, seed=30 + len(kinds))
    Vs = W.sample_variant_shots(V, 5000, seed=31 + len(kinds))
    got, ref = _check(Vs, kinds, in_dt, out_dt)
    if not kinds:   # a copy, rounded once when the output is narrower
        want = ref[0].astype(np.float32).astype(np.float64) if out_dt == torch.float32 else ref[0]
        assert np.array_equal(got[0], want)


def test_wide_output_many_blocks():
    """2^16 output columns, one incoming and two outgoing cuts (the grid-stride
    loop covers several passes)."""
    _gpu()
    V = W.random_variants(1, 2, 16, seed=44)
    _check(V, [1, 0, 1], torch.float32, torch.float32)


def test_outs_are_filled_in_place():
    """Given output tensors, build_entries writes into them (no new
    allocation) with the same result as a fresh call."""
    _gpu()
    V = torch.from_numpy(W.random_variants(1, 1, 8, seed=50)).cuda()
    (E1,) = cqc.build_entries([(V, [0, 1])])
    E2 = torch.full_like(E1, 7.0)
    (E3,) = cqc.build_entries([(V, [0, 1])], outs=[E2])
    torch.cuda.synchronize()
    assert E3.data_ptr() == E2.data_ptr()
    assert torch.equal(E2, E1)


def test_unaligned_fp32_variants():
    """FP32 variants at a 4-byte (not 16-byte) aligned address take the scalar
    path and give the same entries."""
    _gpu()
    V = W.random_variants(1, 2, 6, seed=51).astype(np.float32).astype(np.float64)
    Vd = torch.from_numpy(V).to(device="cuda", dtype=torch.float32).contiguous()
    buf = torch.empty(Vd.numel() + 1, dtype=torch.float32, device="cuda")
    Vu = buf[1:].view(Vd.shape)
    Vu.copy_(Vd)
    assert Vu.data_ptr() % 16 != 0
    (Ea,) = cqc.build_entries([(Vd, [1, 0, 1])])
    (Eu,) = cqc.build_entries([(Vu, [1, 0, 1])])
    torch.cuda.synchronize()
    assert torch.equal(Ea, Eu)


@pytest.mark.parametrize("kinds", [[1], [0], [1, 0, 1], [0, 0, 1, 1], [0, 1, 1, 1, 1]])
def test_eigen_form_matches_oracle(kinds):
    """Eigen-form entries (Eq. 2) from finite-shot variants, FP64, against the
    oracle's eigen form."""
    _gpu()
    k_in, k_out = kinds.count(0), kinds.count(1)
    V = W.sample_variant_shots(W.random_variants(k_in, k_out, 5, seed=60 + len(kinds)), 3000, seed=61)
    Vd = torch.from_numpy(V).cuda()
    (E,) = cqc.build_entries([(Vd, kinds)], form="eigen")
    torch.cuda.synchronize()
    ref = variants.entries_from_variants(V, kinds, "eigen")
    assert np.max(np.abs(E.cpu().numpy() - ref)) <= 1e-13 * (np.max(np.abs(ref)) + 1.0)


def test_eigen_form_end_to_end_and_smaller_kappa():
    """A chain with six cuts: eigen-form entries built on the GPU reconstruct
    the uncut distribution (FP64), their condition number kappa (the term sum
    of |products| over sum |p|) is below the Pauli form's, and both FP32
    reconstructions meet the 1e-6 bar."""
    _gpu()
    circ = W.bridged_chain((3, 2, 3), (3, 3), 6, seed=23)
    cut = circ.cut_map()
    jobs = []
    for sub in circ.subcircuits():
        jobs.append((torch.from_numpy(variants.variant_tensor(circ, sub)).cuda(),
                     [0] * len(sub.q_in) + [1] * len(sub.q_out)))
    truth = sv.uncut_distribution(circ)
    kap = {}
    for form in ("pauli", "eigen"):
        Es = cqc.build_entries(jobs, form=form)
        p64, _ = cqc.reconstruct_fd(Es, cqc.CutMap.from_workload(cut), precision="fp64")
        assert metrics.rel_l1(p64.cpu().numpy(), truth) < 1e-12, form
        E32 = [E.float() for E in Es]
        p32, _ = cqc.reconstruct_fd(E32, cqc.CutMap.from_workload(cut), precision="fp32")
        assert metrics.rel_l1(p32.double().cpu().numpy(), truth) < 1e-6, form
        kap[form] = metrics.kappa([E.cpu().numpy() for E in Es], cut, np.abs(truth).sum())
    assert kap["eigen"] < kap["pauli"], kap
