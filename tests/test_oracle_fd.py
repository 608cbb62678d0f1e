"""Pins of the FD oracle: brute-force state vectors (exactness of cutting,
Section 3.2.3), special cases that reduce to library routines, permuted output
orders, the C twin, and the Eq. 14 cost model."""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import fd, native, statevector as sv, metrics

BRUTE = [((4, 3), (1,), 4), ((5, 5), (2,), 6), ((3, 2, 3), (3, 3), 4),
         ((3, 3, 3), (2, 2), 6), ((2, 3, 3, 2), (1, 2, 2), 4), ((6, 6), (3,), 6),
         ((4, 3, 4), (2, 1), 8), ((7, 7), (2,), 4)]


@pytest.mark.parametrize("own,bridges,layers", BRUTE)
def test_fd_equals_uncut_state_vector(own, bridges, layers):
    inst = W.make_instance(own, bridges, layers, seed=101)
    p = fd.reconstruct(inst.entries, inst.cut)
    truth = sv.uncut_distribution(inst.circuit)
    assert metrics.rel_l1(p, truth) < 1e-12
    assert abs(p.sum() - 1.0) < 1e-12


def test_fd_bit_order_asymmetric_circuit():
    # all angles zero, X on qubit 0 only: the output is |10...0> exactly
    circ = W.bridged_chain((3, 3), (1,), 4, seed=0, x_gates=((0, 0),))
    circ.angles[:] = 0.0
    cut = circ.cut_map()
    p = fd.reconstruct(W.circuit_entries(circ), cut)
    assert abs(p[2 ** (cut.n - 1)] - 1.0) < 1e-14
    assert abs(p.sum() - 1.0) < 1e-14


def test_no_cut_reduces_to_kron():
    cut = W.CutMap(n=7, f=[3, 4], edge_up=[], edge_down=[], out_qubit=list(range(7)))
    A, B = W.random_entries(cut, seed=1)
    p = fd.reconstruct([A, B], cut)
    assert np.max(np.abs(p - np.kron(A[0], B[0]))) < 1e-15
    cut3 = W.CutMap(n=6, f=[2, 1, 3], edge_up=[], edge_down=[], out_qubit=list(range(6)))
    E = W.random_entries(cut3, seed=2)
    p3 = fd.reconstruct(E, cut3)
    assert np.max(np.abs(p3 - np.kron(np.kron(E[0][0], E[1][0]), E[2][0]))) < 1e-15


@pytest.mark.parametrize("K", [1, 2, 3, 4])
def test_two_subcircuits_is_a_gemm(K):
    cut = W.CutMap(n=9, f=[4, 5], edge_up=[0] * K, edge_down=[1] * K, out_qubit=list(range(9)))
    A, B = W.random_entries(cut, seed=K)
    p = fd.reconstruct([A, B], cut)
    ref = (2.0 ** -K) * (A.T @ B)
    assert np.max(np.abs(p - ref.reshape(-1))) < 1e-15 * 4 ** K


def test_permuted_output_order():
    # same tensors, outputs scattered over the global order: p is the transposed tensor
    base = W.CutMap(n=7, f=[3, 4], edge_up=[0, 0], edge_down=[1, 1], out_qubit=list(range(7)))
    ents = W.random_entries(base, seed=4)
    p_base = fd.reconstruct(ents, base).reshape((2,) * 7)
    perm = [5, 0, 3, 6, 1, 2, 4]          # local bit j (concatenated) -> global qubit perm[j]
    cut = W.CutMap(n=7, f=[3, 4], edge_up=[0, 0], edge_down=[1, 1], out_qubit=perm)
    p = fd.reconstruct(ents, cut).reshape((2,) * 7)
    # p[b_perm[0], ..] = p_base[b_0, ..]: global axis perm[j] carries base axis j
    inv = np.argsort(perm)
    assert np.max(np.abs(p - np.transpose(p_base, inv))) < 1e-16


def test_reversed_edge_direction_and_digit_order():
    # edge direction does not change the arithmetic; digit order follows cut id
    cut_a = W.CutMap(n=6, f=[2, 2, 2], edge_up=[0, 1, 2], edge_down=[1, 2, 0], out_qubit=list(range(6)))
    ents = W.random_entries(cut_a, seed=9)
    p = fd.reconstruct(ents, cut_a)
    # brute force over labels by hand
    ref = np.zeros(64)
    for x in range(64):
        x0, x1, x2 = x >> 4, (x >> 2) & 3, x & 3
        s = 0.0
        for l0, l1, l2 in itertools.product(range(4), repeat=3):
            # sub 0 touches cuts 0, 2; sub 1 cuts 0, 1; sub 2 cuts 1, 2
            s += ents[0][l0 * 4 + l2][x0] * ents[1][l0 * 4 + l1][x1] * ents[2][l1 * 4 + l2][x2]
        ref[x] = s / 8.0
    assert np.max(np.abs(p - ref)) < 1e-16


@pytest.mark.parametrize("own,bridges,layers", [((4, 3), (1,), 4), ((3, 2, 3), (2, 2), 6)])
def test_c_twin_matches_python(own, bridges, layers):
    inst = W.make_instance(own, bridges, layers, seed=8)
    p = fd.reconstruct(inst.entries, inst.cut)
    pc = native.reconstruct(inst.entries, inst.cut)
    assert np.array_equal(p, pc)          # same sequential order, same FP64 ops
    xs = W.sample_outputs(inst.n, 50, seed=3)
    assert np.array_equal(native.reconstruct(inst.entries, inst.cut, xs), p[xs])


def test_c_twin_random_permuted():
    cut = W.CutMap(n=8, f=[3, 2, 3], edge_up=[0, 1, 0], edge_down=[1, 2, 2],
                   out_qubit=[7, 2, 5, 0, 3, 6, 1, 4])
    ents = W.random_entries(cut, seed=12)
    assert np.array_equal(fd.reconstruct(ents, cut), native.reconstruct(ents, cut))


def test_sampled_equals_full():
    inst = W.make_instance((3, 3, 3), (2, 2), 4, seed=17)
    p = fd.reconstruct(inst.entries, inst.cut)
    xs = W.sample_outputs(inst.n, 100, seed=1)
    assert np.array_equal(fd.reconstruct(inst.entries, inst.cut, xs), p[xs])


def test_eq14_cost_model():
    # L = 4^K sum_{c=2}^{nC} prod_{i<=c} 2^{f_i}
    assert fd.cost_eq14([4, 4], 1) == 4 * 2 ** 8
    assert fd.cost_eq14([9, 9, 12], 6) == 4 ** 6 * (2 ** 18 + 2 ** 30)
    assert fd.cost_eq14([5], 0) == 0
    # greedy smallest-first never costs more than the given order
    f = [12, 9, 9]
    g = [f[c] for c in fd.greedy_order(f)]
    assert g == [9, 9, 12]
    assert fd.cost_eq14(g, 6) <= fd.cost_eq14(f, 6)
    assert fd.cost_eq14(f, 6) / fd.cost_eq14(g, 6) <= 2.0   # "up to 50%" saving


def test_metrics_closed_forms():
    a = np.array([0.5, 0.5, 0.0])
    b = np.array([0.25, 0.75, 0.0])
    assert metrics.chi2(a, a) == 0.0
    assert abs(metrics.chi2(a, b) - (0.0625 / 0.75 + 0.0625 / 1.25)) < 1e-16
    assert abs(metrics.rel_l1(a, b) - 0.5) < 1e-16
    # kappa = 1 when every term is non-negative
    cut = W.CutMap(n=4, f=[2, 2], edge_up=[0], edge_down=[1], out_qubit=[0, 1, 2, 3])
    ents = [np.abs(E) for E in W.random_entries(cut, seed=3)]
    p = fd.reconstruct(ents, cut)
    assert abs(metrics.kappa(ents, cut, np.abs(p).sum()) - 1.0) < 1e-14


def test_rel_l2_closed_forms():
    ref = np.array([3.0, 4.0])
    assert abs(metrics.rel_l2(ref + np.array([0.3, -0.4]), ref) - 0.1) < 1e-15
    assert abs(metrics.rel_l2(ref * (1 + 1e-3), ref) - 1e-3) < 1e-15
    # normalised by the second argument, not the first
    assert abs(metrics.rel_l2(np.array([6.0, 8.0]), ref) - 1.0) < 1e-15
    assert abs(metrics.rel_l2(ref, np.array([6.0, 8.0])) - 0.5) < 1e-15
    # an orthogonal perturbation adds in quadrature
    assert abs(metrics.rel_l2(np.array([1.0, 1e-5, 0.0]), np.array([1.0, 0.0, 0.0])) - 1e-5) < 1e-20
    # a zero reference reports the plain norm
    assert metrics.rel_l2(np.array([3.0, 4.0]), np.zeros(2)) == 5.0


def test_kappa_signed_hand_case():
    # one cut between two one-qubit subcircuits, signed integer entries:
    # |A| row sums (3, 3, 1, 4), |B| row sums (2, 3, 5, 1): numerator 24 / 2 = 12;
    # p = A^T B / 2 = (-1, 4.5, -2, 1.5), sum |p| = 9, so kappa = 4/3
    cut = W.CutMap(n=2, f=[1, 1], edge_up=[0], edge_down=[1], out_qubit=[0, 1])
    A = np.array([[1.0, -2.0], [3.0, 0.0], [0.0, -1.0], [2.0, 2.0]])
    B = np.array([[1.0, 1.0], [-1.0, 2.0], [2.0, -3.0], [0.0, 1.0]])
    p = fd.reconstruct([A, B], cut)
    assert np.array_equal(p, [-1.0, 4.5, -2.0, 1.5])
    assert abs(metrics.kappa([A, B], cut, np.abs(p).sum()) - 4.0 / 3.0) < 1e-15


def test_kappa_equals_brute_force_abs_term_sum():
    # kappa * sum|p| = sum_x sum_l |term(l, x)|, term by term over a signed
    # three-subcircuit chain with a permuted output order
    cut = W.CutMap(n=6, f=[2, 2, 2], edge_up=[0, 1, 0], edge_down=[1, 2, 2],
                   out_qubit=[4, 1, 5, 0, 2, 3])
    ents = W.random_entries(cut, seed=21)
    p = fd.reconstruct(ents, cut)
    tot = 0.0
    for x in range(2 ** cut.n):
        xc = [int(fd.local_index(cut, c, np.array([x]))[0]) for c in range(3)]
        for l in range(4 ** cut.n_cuts):
            d = fd.label_digits(l, cut.n_cuts)
            t = 1.0
            for c in range(3):
                t *= ents[c][fd.row_of(cut, c, d)][xc[c]]
            tot += abs(t)
    tot *= 2.0 ** -cut.n_cuts
    k = metrics.kappa(ents, cut, np.abs(p).sum())
    assert abs(k * np.abs(p).sum() - tot) < 1e-13 * tot
    assert k > 1.5          # signed entries cancel: the abs() matters here


def test_c_twin_chi2():
    """The C/OpenMP chi-square twin: the closed form on a hand case (zero-sum
    terms skipped), and the numpy oracle to rounding on a large random pair
    for several thread counts."""
    a = np.array([0.5, 0.5, 0.0, 0.0])
    b = np.array([0.25, 0.75, 0.0, 0.0])
    assert abs(native.chi2(a, b) - (0.0625 / 0.75 + 0.0625 / 1.25)) < 1e-16
    rng = np.random.default_rng(5)
    x, y = rng.random(100003), rng.random(100003)
    x[::7] = 0.0
    y[::7] = 0.0
    ref = metrics.chi2(x, y)
    for t in (1, 3, 8):
        assert abs(native.chi2(x, y, threads=t) - ref) <= 1e-12 * ref
