"""Pins of the adjoint oracle: multilinearity makes directional derivatives
exact, so the dot-product identity and linear-loss finite differences hold to
rounding; n_C = 2 reduces to two matrix products; cross-entropy gradients match
FP64 central differences."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, fd


def _replace(ents, c, D):
    out = list(ents)
    out[c] = D
    return out


@pytest.mark.parametrize("own,bridges,layers", [((3, 3), (2,), 4), ((2, 3, 2), (2, 1), 4)])
def test_dot_product_identity(own, bridges, layers):
    inst = W.make_instance(own, bridges, layers, seed=3)
    rng = np.random.default_rng(1)
    G = rng.standard_normal(2 ** inst.n)
    grads = adjoint.vjp(inst.entries, inst.cut, G)
    for c, E in enumerate(inst.entries):
        D = rng.standard_normal(E.shape)
        # p is linear in E_c: J_c D = p(E_1..D..E_nC)
        jd = fd.reconstruct(_replace(inst.entries, c, D), inst.cut)
        lhs = float(G @ jd)
        rhs = float(np.sum(grads[c] * D))
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_two_subcircuit_closed_form():
    K = 3
    cut = W.CutMap(n=7, f=[3, 4], edge_up=[0] * K, edge_down=[1] * K, out_qubit=list(range(7)))
    A, B = W.random_entries(cut, seed=5)
    G = np.random.default_rng(2).standard_normal((8, 16))
    gA, gB = adjoint.vjp([A, B], cut, G.reshape(-1))
    assert np.max(np.abs(gA - (2.0 ** -K) * (B @ G.T))) < 1e-15
    assert np.max(np.abs(gB - (2.0 ** -K) * (A @ G))) < 1e-15


def test_cross_entropy_finite_differences():
    inst = W.make_instance((3, 2, 3), (1, 1), 4, seed=8)
    t = W.dirichlet_target(inst.n, seed=1000)
    p = fd.reconstruct(inst.entries, inst.cut)
    G = adjoint.cross_entropy_grad(p, t)
    grads = adjoint.vjp(inst.entries, inst.cut, G)
    rng = np.random.default_rng(4)
    for c, E in enumerate(inst.entries):
        h = 1e-6 * np.max(np.abs(E))
        for _ in range(5):
            r, x = int(rng.integers(E.shape[0])), int(rng.integers(E.shape[1]))
            Ep, Em = E.copy(), E.copy()
            Ep[r, x] += h
            Em[r, x] -= h
            lp = adjoint.cross_entropy(fd.reconstruct(_replace(inst.entries, c, Ep), inst.cut), t)
            lm = adjoint.cross_entropy(fd.reconstruct(_replace(inst.entries, c, Em), inst.cut), t)
            num = (lp - lm) / (2 * h)
            assert abs(num - grads[c][r, x]) <= 1e-6 * max(1.0, abs(num))


def test_cross_entropy_floor():
    p = np.array([0.5, 0.0, -1e-3, 0.5])
    t = np.array([0.25, 0.25, 0.25, 0.25])
    g = adjoint.cross_entropy_grad(p, t)
    assert np.array_equal(g, [-0.5, 0.0, 0.0, -0.5])
    assert abs(adjoint.cross_entropy(p, t) - (-0.5 * np.log(0.5) - 0.5 * np.log(1e-30))) < 1e-12


@pytest.mark.parametrize("own,bridges,layers", [((3, 3), (2,), 4), ((2, 3, 2), (2, 1), 4),
                                                ((2, 2, 2, 2), (1, 1, 1), 4)])
def test_vjp_at_equals_vjp(own, bridges, layers):
    inst = W.make_instance(own, bridges, layers, seed=6)
    G = np.random.default_rng(3).standard_normal(2 ** inst.n)
    grads = adjoint.vjp(inst.entries, inst.cut, G)
    rng = np.random.default_rng(9)
    for c, E in enumerate(inst.entries):
        elems = [(int(rng.integers(E.shape[0])), int(rng.integers(E.shape[1]))) for _ in range(12)]
        got = adjoint.vjp_at(inst.entries, inst.cut, G, c, elems)
        ref = np.array([grads[c][r, y] for r, y in elems])
        scale = np.max(np.abs(grads[c]))
        assert np.max(np.abs(got - ref)) <= 1e-13 * scale


def test_vjp_at_closed_form_permuted_order():
    # n_C = 2: dE_A = 2^-K B G^T and dE_B = 2^-K A G, with G laid out in the
    # local (x_A, x_B) order after undoing a scattered global output order
    K = 2
    perm = [3, 0, 5, 1, 4, 2]
    cut = W.CutMap(n=6, f=[2, 4], edge_up=[0] * K, edge_down=[1] * K, out_qubit=perm)
    A, B = W.random_entries(cut, seed=7)
    G = np.random.default_rng(8).standard_normal(2 ** 6)
    # local index (x_A, x_B) -> global index
    loc = np.arange(64)
    glob = np.zeros(64, dtype=np.int64)
    for j, q in enumerate(perm):
        glob |= ((loc >> (5 - j)) & 1) << (5 - q)
    Gl = G[glob].reshape(4, 16)
    gA = (2.0 ** -K) * (B @ Gl.T)
    gB = (2.0 ** -K) * (A @ Gl)
    elems_a = [(r, y) for r in range(16) for y in range(4)]
    elems_b = [(r, y) for r in (0, 5, 15) for y in range(16)]
    assert np.max(np.abs(adjoint.vjp_at([A, B], cut, G, 0, elems_a) - [gA[r, y] for r, y in elems_a])) < 1e-15
    assert np.max(np.abs(adjoint.vjp_at([A, B], cut, G, 1, elems_b) - [gB[r, y] for r, y in elems_b])) < 1e-15
