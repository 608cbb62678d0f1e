"""Subcircuit entry tensors of a bridged-chain circuit, by ideal operator simulation.

This is the stand-in for running the subcircuit variants on a quantum device
and reading out their exact (infinite-shot) statistics.  It produces, for every
subcircuit c, the tensor

    E_c[(l_in, l_out), x_c] = Tr[ (|x_c><x_c| (x) tau_{l_out}) U_c (|0><0|_own (x) sigma_{l_in}) U_c^dagger ]

where sigma_{l_in} is the tensor product of Pauli matrices on the incoming cut
qubits (the downstream side of each cut) and tau_{l_out} the one on the
outgoing cut qubits (the upstream side), labels I=0, X=1, Y=2, Z=3.  By the
Pauli expansion of a 2x2 operator (Eq. 1 of the paper) these are the entry
tensors whose 2^-K-scaled Kronecker term sum equals the uncut distribution.

Route taken here (deliberately different from the paper's physical route of
basis-change circuits, eigenstate initialisations and the +-1 shot attribution
of Eq. 3): simulate the 2^k computational-basis initialisations of the incoming
qubits, form the Gram tensor <V_j|(|x><x| (x) |o><o'|)|V_i>, and contract it with
the Pauli matrices.  No part of the reconstruction (the term sum) lives here.
"""
from __future__ import annotations

import numpy as np

from .circuits import BridgedChain

_PAULI = np.array([
    [[1, 0], [0, 1]],
    [[0, 1], [1, 0]],
    [[0, -1j], [1j, 0]],
    [[1, 0], [0, -1]],
], dtype=np.complex128)


def _pauli_strings(k):
    """(4^k, 2^k, 2^k): tensor products, first factor = most significant qubit/digit."""
    out = np.ones((1, 1, 1), dtype=np.complex128)
    for _ in range(k):
        out = np.einsum("aij,bkl->abikjl", out, _PAULI).reshape(
            out.shape[0] * 4, out.shape[1] * 2, out.shape[2] * 2)
    return out


def _u3(theta, phi, lam):
    c, s = np.cos(theta / 2.0), np.sin(theta / 2.0)
    return np.array([[c, -np.exp(1j * lam) * s],
                     [np.exp(1j * phi) * s, np.exp(1j * (phi + lam)) * c]],
                    dtype=np.complex128)


def _apply_1q(state, mat, axis):
    # state: (B, 2, 2, ..., 2); axis counts from 1
    st = np.moveaxis(state, axis, -1)
    st = st @ mat.T
    return np.moveaxis(st, -1, axis)


def _apply_cz(state, a, b):
    idx = [slice(None)] * state.ndim
    idx[a] = 1
    idx[b] = 1
    state[tuple(idx)] *= -1.0
    return state


def simulate_basis_inputs(circ: BridgedChain, sub):
    """Amplitudes V[i, x, o] of U_c |i>_in |0>_own |0>_out for all 2^k_in basis states i."""
    loc = sub.local_qubits
    pos = {q: p for p, q in enumerate(loc)}
    d = len(loc)
    k_in = len(sub.q_in)
    b = 2 ** k_in
    state = np.zeros((b,) + (2,) * d, dtype=np.complex128)
    for i in range(b):
        bits = [(i >> (k_in - 1 - t)) & 1 for t in range(k_in)]
        idx = (i,) + tuple(bits) + (0,) * (d - k_in)
        state[idx] = 1.0
    for g in circ.subcircuit_gates(sub):
        if g[0] == "u3":
            state = _apply_1q(state, _u3(g[2], g[3], g[4]), 1 + pos[g[1]])
        elif g[0] == "x":
            state = _apply_1q(state, _PAULI[1], 1 + pos[g[1]])
        elif g[0] == "cz":
            state = _apply_cz(state, 1 + pos[g[1]], 1 + pos[g[2]])
    f = sub.f
    return state.reshape(b, 2 ** f, 2 ** len(sub.q_out))


def subcircuit_entries(circ: BridgedChain, sub, dtype=np.float64):
    """Entry tensor E_c of shape (4^k_c, 2^f_c), rows = (incoming labels, outgoing labels)."""
    V = simulate_basis_inputs(circ, sub)
    k_in, k_out = len(sub.q_in), len(sub.q_out)
    sig = _pauli_strings(k_in)
    tau = _pauli_strings(k_out)
    # E[s, t, x] = sum sig[s,i,j] tau[t,o,p] conj(V[j,x,o]) V[i,x,p]
    tmp = np.einsum("jxo,top->jtxp", V.conj(), tau, optimize=True)
    tmp = np.einsum("jtxp,ixp->jitx", tmp, V, optimize=True)
    E = np.einsum("sij,jitx->stx", sig, tmp, optimize=True)
    E = E.real.reshape(4 ** k_in * 4 ** k_out, 2 ** sub.f)
    return np.ascontiguousarray(E.astype(dtype))


def circuit_entries(circ: BridgedChain, dtype=np.float64):
    return [subcircuit_entries(circ, s, dtype) for s in circ.subcircuits()]
