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
