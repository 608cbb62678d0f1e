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


# ---- entries from stacked variant distributions (the input of on-device
# entry construction)

@pytest.mark.parametrize("own,bridges,layers", SHAPES[:5])
def test_entries_from_variants_equal_paper_route(own, bridges, layers):
    """From the stacked simulated variants, with the chain's cut order (incoming
    cuts before outgoing ones), the entries equal the paper route (itself
    pinned to the independent operator route above)."""
    circ = W.bridged_chain(own, bridges, layers, seed=13)
    for sub in circ.subcircuits():
        V = variants.variant_tensor(circ, sub)
        kinds = [0] * len(sub.q_in) + [1] * len(sub.q_out)
        E = variants.entries_from_variants(V, kinds)
        ref = variants.subcircuit_entries(circ, sub)
        assert E.shape == ref.shape
        assert np.max(np.abs(E - ref)) < 1e-13


def test_entries_from_variants_row_sums_any_distribution():
    """For any normalised variant distributions (finite shots included): a row
    whose outgoing labels are all I sums to 2^k_in if every incoming label is
    I and to 0 otherwise (the I, Z, X, Y initialisation weights sum to 2, 0,
    0, 0)."""
    V = W.random_variants(2, 2, 4, seed=3)
    Vs = W.sample_variant_shots(V, 1000, seed=4)
    for VV in (V, Vs):
        E = variants.entries_from_variants(VV, [0, 1, 0, 1])
        for row in range(E.shape[0]):
            d = [(row >> (2 * (3 - t))) & 3 for t in range(4)]   # labels of cuts 0..3
            if d[1] == 0 and d[3] == 0:
                want = 4.0 if d[0] == 0 and d[2] == 0 else 0.0
                assert abs(E[row].sum() - want) < 1e-12, (row, d)


def test_entries_from_variants_cut_order_permutes_rows():
    """Listing the same cuts in another id order permutes the label digits of
    the rows and nothing else."""
    V = W.random_variants(1, 2, 3, seed=6)
    a = variants.entries_from_variants(V, [0, 1, 1]).reshape(4, 4, 4, -1)   # (in, out0, out1)
    b = variants.entries_from_variants(V, [1, 0, 1]).reshape(4, 4, 4, -1)   # (out0, in, out1)
    assert np.array_equal(np.transpose(a, (1, 0, 2, 3)), b)


def test_entries_from_variants_single_cut_by_hand():
    """One measured cut (k_out = 1) and no incoming cut: rows I, X, Y, Z are
    p0 + p1 in the computational basis, p0 - p1 in the X and Y bases, and
    p0 - p1 in the computational basis (Eq. 3 written out)."""
    V = W.random_variants(0, 1, 2, seed=8)   # [1][3][4][2]
    E = variants.entries_from_variants(V, [1])
    comp, xb, yb = V[0, 0], V[0, 1], V[0, 2]
    assert np.allclose(E[0], comp[:, 0] + comp[:, 1], atol=0, rtol=0)
    assert np.allclose(E[1], xb[:, 0] - xb[:, 1], atol=0, rtol=0)
    assert np.allclose(E[2], yb[:, 0] - yb[:, 1], atol=0, rtol=0)
    assert np.allclose(E[3], comp[:, 0] - comp[:, 1], atol=0, rtol=0)


@pytest.mark.parametrize("own,bridges,layers", SHAPES[:4])
def test_entries_from_variants_eigen_equal_paper_route(own, bridges, layers):
    """Eigen form (Eq. 2) from the stacked variants equals the eigen-form paper
    route, which reconstructs the same distribution as the Pauli form."""
    circ = W.bridged_chain(own, bridges, layers, seed=19)
    ents = []
    for sub in circ.subcircuits():
        V = variants.variant_tensor(circ, sub)
        kinds = [0] * len(sub.q_in) + [1] * len(sub.q_out)
        E = variants.entries_from_variants(V, kinds, "eigen")
        assert np.max(np.abs(E - variants.subcircuit_entries(circ, sub, "eigen"))) < 1e-13
        ents.append(E)
    cut = circ.cut_map()
    assert np.max(np.abs(fd.reconstruct(ents, cut) - sv.uncut_distribution(circ))) < 1e-13


def test_eigen_weights_by_hand():
    """One measured cut, eigen form: rows A1..A4 are 2 p0, 2 p1 in the
    computational basis, p0 - p1 in the X and in the Y basis."""
    V = W.random_variants(0, 1, 2, seed=9)
    E = variants.entries_from_variants(V, [1], "eigen")
    comp, xb, yb = V[0, 0], V[0, 1], V[0, 2]
    assert np.array_equal(E[0], 2 * comp[:, 0])
    assert np.array_equal(E[1], 2 * comp[:, 1])
    assert np.array_equal(E[2], xb[:, 0] - xb[:, 1])
    assert np.array_equal(E[3], yb[:, 0] - yb[:, 1])
