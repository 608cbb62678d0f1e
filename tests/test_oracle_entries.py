"""Pins of the entry tensors: the paper's physical route against an independent
operator route, row-sum invariants, and the worked example of Section 3.2."""
import numpy as np
import pytest

import workloads as W
from oracle import variants, fd, statevector as sv

SHAPES = [((4, 3), (1,), 4), ((2, 2), (1,), 4), ((3, 3), (2,), 6),
          ((3, 2, 3), (2, 2), 6), ((2, 2, 2, 2), (1, 2, 1), 4), ((3, 1, 3), (3, 2), 4)]


@pytest.mark.parametrize("own,bridges,layers", SHAPES)
def test_paper_route_equals_operator_route(own, bridges, layers):
    circ = W.bridged_chain(own, bridges, layers, seed=11)
    gen = W.circuit_entries(circ)
    orc = variants.circuit_entries(circ)
    for a, b in zip(gen, orc):
        assert a.shape == b.shape
        assert np.max(np.abs(a - b)) < 1e-13


@pytest.mark.parametrize("own,bridges,layers", SHAPES[:4])
def test_row_sum_invariants(own, bridges, layers):
    circ = W.bridged_chain(own, bridges, layers, seed=5)
    ents = variants.circuit_entries(circ)
    subs = circ.subcircuits()
    # root (no incoming cut): the all-I row is a marginal distribution, sums to 1
    assert abs(ents[0][0].sum() - 1.0) < 1e-13
    # leaf (no outgoing cut): Tr(sigma) = 2^k for all-I, 0 for any other label
    leaf = ents[-1]
    k = len(subs[-1].q_in)
    sums = leaf.sum(axis=1)
    assert abs(sums[0] - 2 ** k) < 1e-12
    assert np.max(np.abs(sums[1:])) < 1e-12


def test_eigen_form_equals_pauli_form():
    circ = W.bridged_chain((3, 2, 3), (2, 1), 6, seed=21)
    cut = circ.cut_map()
    p_pauli = fd.reconstruct(variants.circuit_entries(circ, "pauli"), cut)
    p_eigen = fd.reconstruct(variants.circuit_entries(circ, "eigen"), cut)
    assert np.max(np.abs(p_pauli - p_eigen)) < 1e-14


def test_worked_example_section_3_2():
    """5-qubit circuit, one cut on q2 into two 3-qubit subcircuits (Figure 4 shape).

    p(|01010>) = 1/2 sum_i p_{1,i} p_{2,i} with the p_{1,i}, p_{2,i} exactly as
    printed in Section 3.2.2 (eigen form), from the variant distributions.
    """
    circ = W.bridged_chain((2, 2), (1,), 4, seed=33)
    s1, s2 = circ.subcircuits()
    assert s1.d == 3 and s2.d == 3
    # subcircuit 1: outputs q0 q1, measured cut qubit last; p(|01b> | M)
    d1 = {b: variants.variant_distribution(circ, s1, (), (b,)) for b in ("Z", "X", "Y")}
    x1 = 0b01
    pI0, pI1 = d1["Z"][x1, 0], d1["Z"][x1, 1]        # M=I and M=Z share the circuit
    pZ0, pZ1 = pI0, pI1
    pX0, pX1 = d1["X"][x1, 0], d1["X"][x1, 1]
    pY0, pY1 = d1["Y"][x1, 0], d1["Y"][x1, 1]
    p11 = pI0 + pI1 + pZ0 - pZ1
    p12 = pI0 + pI1 - pZ0 + pZ1
    p13 = pX0 - pX1
    p14 = pY0 - pY1
    # subcircuit 2: outputs q2 (initialised) q3 q4; relevant state |010>
    x2 = 0b010
    q = {i: variants.variant_distribution(circ, s2, (i,), ())[x2, 0] for i in range(4)}
    p21 = q[0]
    p22 = q[1]
    p23 = 2 * q[2] - q[0] - q[1]
    p24 = 2 * q[3] - q[0] - q[1]
    recon = 0.5 * (p11 * p21 + p12 * p22 + p13 * p23 + p14 * p24)
    truth = sv.uncut_distribution(circ)[0b01010]
    assert abs(recon - truth) < 1e-15
    assert abs(fd.reconstruct(variants.circuit_entries(circ), circ.cut_map(), [0b01010])[0] - truth) < 1e-15


def test_cut_map_shapes():
    circ = W.bridged_chain((9, 6, 9), (3, 3), 10, seed=3)
    cut = circ.cut_map()
    assert cut.n == 30 and cut.n_cuts == 6
    assert cut.f == [9, 9, 12]
    assert [cut.entry_shape(c) for c in range(3)] == [(64, 512), (4096, 512), (64, 4096)]
    assert sorted(cut.out_qubit) == list(range(30))
    assert [s.d for s in circ.subcircuits()] == [12, 12, 12]
