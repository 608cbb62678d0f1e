"""Plain FP64 (complex128) state-vector simulator: the ground truth of Section 2.

Qubit q is axis q of a (2,)*n array, so the flattened index of |b_0 ... b_{n-1}>
is sum_q b_q 2^(n-1-q): qubit 0 is the most significant bit, as in the
|q_0, ..., q_{n-1}> notation of Section 3.2.
"""
from __future__ import annotations

import numpy as np

SQ2 = 1.0 / np.sqrt(2.0)
H = np.array([[SQ2, SQ2], [SQ2, -SQ2]], dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
S = np.array([[1, 0], [0, 1j]], dtype=np.complex128)
SDG = np.array([[1, 0], [0, -1j]], dtype=np.complex128)


def u3(theta, phi, lam):
    """OpenQASM U3(theta, phi, lambda)."""
    return np.array([
        [np.cos(theta / 2), -np.exp(1j * lam) * np.sin(theta / 2)],
        [np.exp(1j * phi) * np.sin(theta / 2), np.exp(1j * (phi + lam)) * np.cos(theta / 2)],
    ], dtype=np.complex128)


def zero_state(n):
    psi = np.zeros((2,) * n, dtype=np.complex128)
    psi[(0,) * n] = 1.0
    return psi


def apply_1q(psi, gate, q):
    """psi'[.., a, ..] = sum_b gate[a, b] psi[.., b, ..] on axis q."""
    out = np.tensordot(gate, psi, axes=([1], [q]))
    return np.moveaxis(out, 0, q)


def apply_cz(psi, a, b):
    psi = psi.copy()
    idx = [slice(None)] * psi.ndim
    idx[a] = 1
    idx[b] = 1
    psi[tuple(idx)] = -psi[tuple(idx)]
    return psi


def run_gates(psi, gates, qmap):
    """Apply ("u3", q, th, ph, la, ...), ("x", q, ...), ("cz", a, b, ...) with qubit map."""
    for g in gates:
        if g[0] == "u3":
            psi = apply_1q(psi, u3(g[2], g[3], g[4]), qmap[g[1]])
        elif g[0] == "x":
            psi = apply_1q(psi, X, qmap[g[1]])
        elif g[0] == "cz":
            psi = apply_cz(psi, qmap[g[1]], qmap[g[2]])
        else:
            raise ValueError(g[0])
    return psi


def probabilities(psi):
    return (np.abs(psi) ** 2).reshape(-1)


def uncut_distribution(circ):
    """|U|0>|^2 of the whole (uncut) circuit, the exactness target of Section 3.2.3."""
    n = circ.n
    psi = run_gates(zero_state(n), circ.gate_list(), {q: q for q in range(n)})
    return probabilities(psi)
