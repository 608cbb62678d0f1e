"""Pins of the blocked full-vector oracle (pairwise contraction over output
blocks): it must equal the per-output FD definition and brute-force state
vectors of the uncut circuit (exactness of cutting, Section 3.2.3) for every
block split, cut topology and output order."""
import numpy as np
import pytest

import workloads as W
from oracle import blocked, fd, metrics, statevector as sv


def _close(p, ref, ents, cut, sl=slice(None)):
    """|p - ref| within 1e-13 of T_x = 2^-K sum_l prod_c |E_c| (the scale of
    the rounding of any summation order) at every output of the slice."""
    T = fd.reconstruct([np.abs(E) for E in ents], cut)[sl]
    return np.max(np.abs(p - ref) / np.maximum(T, 1e-300)) < 1e-13


@pytest.mark.parametrize("own,bridges,layers", [((4, 3), (1,), 4), ((3, 2, 3), (3, 3), 4),
                                                ((2, 3, 3, 2), (1, 2, 2), 4), ((6, 6), (3,), 6)])
def test_blocked_equals_uncut_state_vector(own, bridges, layers):
    inst = W.make_instance(own, bridges, layers, seed=31)
    truth = sv.uncut_distribution(inst.circuit)
    for top in (0, 1, 3):
        p = np.concatenate([v for _, v in blocked.blocks(inst.entries, inst.cut, top)])
        assert metrics.rel_l1(p, truth) < 1e-12
        assert abs(p.sum() - 1.0) < 1e-12


@pytest.mark.parametrize("top", [0, 2, 5])
def test_blocked_equals_definition_general_topology(top):
    # cuts between non-adjacent subcircuits, a subcircuit reached by no cut of
    # its predecessor, and an output order scattered over the global qubits
    cut = W.CutMap(n=11, f=[3, 2, 3, 3], edge_up=[0, 2, 0, 1, 3], edge_down=[2, 1, 3, 3, 2],
                   out_qubit=[7, 2, 10, 5, 0, 3, 9, 1, 8, 4, 6])
    ents = W.random_entries(cut, seed=5)
    ref = fd.reconstruct(ents, cut)
    p = np.concatenate([v for _, v in blocked.blocks(ents, cut, top)])
    assert _close(p, ref, ents, cut)


def test_blocked_block_is_a_contiguous_range():
    inst = W.make_instance((3, 3, 3), (2, 2), 4, seed=4)
    ref = fd.reconstruct(inst.entries, inst.cut)
    n = inst.n
    for b in (0, 5, 15):
        v = blocked.reconstruct_block(inst.entries, inst.cut, 4, b)
        sl = slice(b * 2 ** (n - 4), (b + 1) * 2 ** (n - 4))
        assert _close(v, ref[sl], inst.entries, inst.cut, sl)


def test_blocked_no_cut_is_kron_and_gemm():
    cut = W.CutMap(n=7, f=[3, 4], edge_up=[], edge_down=[], out_qubit=list(range(7)))
    A, B = W.random_entries(cut, seed=1)
    assert np.max(np.abs(blocked.reconstruct([A, B], cut) - np.kron(A[0], B[0]))) < 1e-16
    K = 3
    cut = W.CutMap(n=9, f=[4, 5], edge_up=[0] * K, edge_down=[1] * K, out_qubit=list(range(9)))
    A, B = W.random_entries(cut, seed=2)
    ref = ((2.0 ** -K) * (A.T @ B)).reshape(-1)
    assert np.max(np.abs(blocked.reconstruct([A, B], cut) - ref)) < 1e-16 * 4 ** K


def test_blocked_rejects_bad_block():
    cut = W.CutMap(n=4, f=[2, 2], edge_up=[0], edge_down=[1], out_qubit=[0, 1, 2, 3])
    ents = W.random_entries(cut, seed=1)
    with pytest.raises(ValueError):
        blocked.reconstruct_block(ents, cut, 2, 4)
