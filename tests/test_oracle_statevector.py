"""Pins of the oracle's state-vector simulator against closed forms."""
import numpy as np
import pytest

from oracle import statevector as sv


def test_u3_unitary_and_special_values():
    rng = np.random.default_rng(0)
    for _ in range(20):
        U = sv.u3(*rng.uniform(0, 2 * np.pi, 3))
        assert np.allclose(U.conj().T @ U, np.eye(2), atol=1e-14)
    # U3(pi, 0, pi) = X ; U3(pi/2, 0, pi) = H ; U3(0, 0, lam) = diag(1, e^{i lam})
    assert np.allclose(sv.u3(np.pi, 0, np.pi), sv.X, atol=1e-15)
    assert np.allclose(sv.u3(np.pi / 2, 0, np.pi), sv.H, atol=1e-15)
    assert np.allclose(sv.u3(0, 0, 0.3), np.diag([1, np.exp(0.3j)]), atol=1e-15)


def test_gate_identities():
    Z = np.diag([1.0, -1.0]).astype(complex)
    assert np.allclose(sv.S @ sv.S, Z)
    assert np.allclose(sv.H @ sv.X @ sv.H, Z)
    assert np.allclose(sv.S @ sv.SDG, np.eye(2))


def test_bit_order_q0_is_msb():
    n = 5
    psi = sv.apply_1q(sv.zero_state(n), sv.X, 0)
    p = sv.probabilities(psi)
    assert p[2 ** (n - 1)] == 1.0
    psi = sv.apply_1q(sv.zero_state(n), sv.X, n - 1)
    assert sv.probabilities(psi)[1] == 1.0


def test_bell_state_via_cz():
    # H(q0); H(q1) CZ H(q1) = CNOT(q0 -> q1): (|00> + |11>)/sqrt2
    psi = sv.zero_state(2)
    psi = sv.apply_1q(psi, sv.H, 0)
    psi = sv.apply_1q(psi, sv.H, 1)
    psi = sv.apply_cz(psi, 0, 1)
    psi = sv.apply_1q(psi, sv.H, 1)
    assert np.allclose(sv.probabilities(psi), [0.5, 0, 0, 0.5], atol=1e-15)


@pytest.mark.parametrize("n", [3, 6, 9])
def test_norm_preserved(n):
    rng = np.random.default_rng(n)
    psi = sv.zero_state(n)
    for _ in range(30):
        q = int(rng.integers(n))
        psi = sv.apply_1q(psi, sv.u3(*rng.uniform(0, 2 * np.pi, 3)), q)
        a, b = rng.choice(n, 2, replace=False)
        psi = sv.apply_cz(psi, int(a), int(b))
    assert abs(sv.probabilities(psi).sum() - 1.0) < 1e-13
