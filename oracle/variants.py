"""Subcircuit entry tensors by the paper's physical route (Sections 3.1, 3.2).

For a cut wire between an upstream vertex u and a downstream vertex v
(Figure 3), the upstream subcircuit is run with the cut qubit measured in the
I, X, Y or Z basis (I and Z are the same physical circuit) and the downstream
subcircuit with the cut qubit initialised in |0>, |1>, |+> or |+i>.

Upstream, each shot is attributed with a +-1 factor from the measured cut
qubit (Eq. 3): basis I counts both outcomes with +1; any other basis counts
outcome 0 with +1 and outcome 1 with -1.  The basis changes are: X = H before
measuring, Y = S^dagger then H, outcome 0 <-> the +1 eigenstate.

Downstream, the terms p_{2,i} combine initialisations (Section 3.2.2):
  Pauli form (Eq. 1):   I -> q(|0>) + q(|1>),       Z -> q(|0>) - q(|1>),
                        X -> 2q(|+>) - q(|0>) - q(|1>),
                        Y -> 2q(|+i>) - q(|0>) - q(|1>)
  eigen form (Eq. 2):   A1 -> q(|0>), A2 -> q(|1>), A3, A4 as X, Y above,
                        with the upstream partners Tr(AI)+Tr(AZ), Tr(AI)-Tr(AZ),
                        Tr(AX), Tr(AY).
Each cut contributes one label digit; several cuts multiply.  The row of E_c is
the base-4 number of the labels of the cuts incident to c in ascending cut id,
first cut = most significant digit; in Pauli form I=0, X=1, Y=2, Z=3, in eigen
form A1..A4 = 0..3.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import statevector as sv

# measurement basis per upstream Pauli label (I and Z share the physical circuit)
_BASIS_OF_LABEL = {0: "Z", 1: "X", 2: "Y", 3: "Z"}
# init states: 0 -> |0>, 1 -> |1>, 2 -> |+>, 3 -> |+i>
_INIT_GATES = {0: [], 1: [sv.X], 2: [sv.H], 3: [sv.H, sv.S]}
_BASIS_GATES = {"Z": [], "X": [sv.H], "Y": [sv.SDG, sv.H]}

# Downstream combination coefficients over (|0>, |1>, |+>, |+i>) per label.
_DOWN_PAULI = {0: (1, 1, 0, 0), 3: (1, -1, 0, 0), 1: (-1, -1, 2, 0), 2: (-1, -1, 0, 2)}
_DOWN_EIGEN = {0: (1, 0, 0, 0), 1: (0, 1, 0, 0), 2: (-1, -1, 2, 0), 3: (-1, -1, 0, 2)}


def variant_distribution(circ, sub, inits, bases):
    """Probabilities over the subcircuit's d qubits for one variant.

    inits: per incoming qubit, init index 0..3; bases: per outgoing qubit,
    "Z" | "X" | "Y".  Returned shape (2^f, 2^k_out): outputs (incoming, own in
    local order) by outgoing measurement outcomes.
    """
    loc = sub.local_qubits
    qmap = {q: p for p, q in enumerate(loc)}
    psi = sv.zero_state(len(loc))
    for q, init in zip(sub.q_in, inits):
        for g in _INIT_GATES[init]:
            psi = sv.apply_1q(psi, g, qmap[q])
    psi = sv.run_gates(psi, circ.subcircuit_gates(sub), qmap)
    for q, b in zip(sub.q_out, bases):
        for g in _BASIS_GATES[b]:
            psi = sv.apply_1q(psi, g, qmap[q])
    return sv.probabilities(psi).reshape(2 ** sub.f, 2 ** len(sub.q_out))


def attribute(prob, labels):
    """Eq. 3: weight each outgoing outcome by prod_t lambda(label_t, outcome_t)."""
    k = len(labels)
    out = np.zeros(prob.shape[0])
    for o in range(2 ** k):
        w = 1.0
        for t, lab in enumerate(labels):
            bit = (o >> (k - 1 - t)) & 1
            if lab != 0 and bit == 1:
                w = -w
        out = out + w * prob[:, o]
    return out


def _upstream_pauli(dist_by_basis, labels):
    bases = tuple(_BASIS_OF_LABEL[l] for l in labels)
    return attribute(dist_by_basis[bases], labels)


def _upstream_eigen(dist_by_basis, labels):
    # A1: Tr(AI)+Tr(AZ), A2: Tr(AI)-Tr(AZ), A3: Tr(AX), A4: Tr(AY); expand per cut.
    expansion = {0: [(0, 1.0), (3, 1.0)], 1: [(0, 1.0), (3, -1.0)], 2: [(1, 1.0)], 3: [(2, 1.0)]}
    total = None
    for combo in itertools.product(*[expansion[l] for l in labels]):
        pl = tuple(c[0] for c in combo)
        coef = float(np.prod([c[1] for c in combo])) if combo else 1.0
        val = coef * _upstream_pauli(dist_by_basis, pl)
        total = val if total is None else total + val
    if total is None:
        total = _upstream_pauli(dist_by_basis, ())
    return total


def subcircuit_entries(circ, sub, form="pauli"):
    """E_c of shape (4^k_c, 2^f_c) by running all 4^k_in x 3^k_out variants."""
    k_in, k_out = len(sub.q_in), len(sub.q_out)
    down = _DOWN_PAULI if form == "pauli" else _DOWN_EIGEN
    upstream = _upstream_pauli if form == "pauli" else _upstream_eigen
    rows = np.zeros((4 ** k_in, 4 ** k_out, 2 ** sub.f))
    for inits in itertools.product(range(4), repeat=k_in):
        dists = {}
        for bases in itertools.product(("Z", "X", "Y"), repeat=k_out):
            dists[bases] = variant_distribution(circ, sub, inits, bases)
        for l_out_idx, l_out in enumerate(itertools.product(range(4), repeat=k_out)):
            up = upstream(dists, l_out)
            for l_in_idx, l_in in enumerate(itertools.product(range(4), repeat=k_in)):
                coef = 1.0
                for lab, init in zip(l_in, inits):
                    coef *= down[lab][init]
                if coef != 0.0:
                    rows[l_in_idx, l_out_idx] += coef * up
    return rows.reshape(4 ** k_in * 4 ** k_out, 2 ** sub.f)


def circuit_entries(circ, form="pauli"):
    return [subcircuit_entries(circ, s, form) for s in circ.subcircuits()]


def variant_tensor(circ, sub):
    """Every variant distribution of a subcircuit stacked as
    [4^k_in][3^k_out][2^f][2^k_out]: initialisation combination (per incoming
    cut 0 |0>, 1 |1>, 2 |+>, 3 |+i>, first cut the most significant base-4
    digit), measurement-basis combination (per outgoing cut 0 computational,
    1 X, 2 Y, first cut the most significant base-3 digit), output bits, then
    the measured cut bits (first outgoing cut the most significant bit)."""
    k_in, k_out = len(sub.q_in), len(sub.q_out)
    V = np.zeros((4 ** k_in, 3 ** k_out, 2 ** sub.f, 2 ** k_out))
    for ii, inits in enumerate(itertools.product(range(4), repeat=k_in)):
        for bi, bases in enumerate(itertools.product(("Z", "X", "Y"), repeat=k_out)):
            V[ii, bi] = variant_distribution(circ, sub, inits, bases)
    return V


# Per outgoing-cut label: the measurement basis it reads (0 computational,
# 1 X, 2 Y) and the weights of measured bit 0 and 1.  Pauli form: Eq. 3.
# Eigen form (Eq. 2): A1 = Tr(AI) + Tr(AZ), A2 = Tr(AI) - Tr(AZ) in the
# computational basis, A3, A4 as X, Y.
_UP_BASIS = {"pauli": {0: 0, 1: 1, 2: 2, 3: 0}, "eigen": {0: 0, 1: 0, 2: 1, 3: 2}}
_UP_WEIGHT = {"pauli": {0: (1, 1), 1: (1, -1), 2: (1, -1), 3: (1, -1)},
              "eigen": {0: (2, 0), 1: (0, 2), 2: (1, -1), 3: (1, -1)}}


def entries_from_variants(V, cut_kind, form="pauli"):
    """Entry tensor from stacked variant distributions (Sections 3.1-3.2): for
    every label assignment, the outgoing cuts' labels pick the measurement
    bases and weight the measured bits (Eq. 3 in Pauli form); the incoming
    cuts' labels combine the initialisations by the p_{2,i} rule (Eq. 1, or
    Eq. 2 in eigen form).

    V: [4^k_in][3^k_out][2^f][2^k_out] as variant_tensor.  cut_kind: per
    incident cut in ascending cut id, 0 if initialised here (incoming), 1 if
    measured here (outgoing); the i-th incoming / outgoing cut of that list is
    the i-th digit of V's initialisation / basis axes.  Row of E = base-4
    number of the labels (I=0, X=1, Y=2, Z=3) in cut_kind's order, first most
    significant.
    """
    cut_kind = list(cut_kind)
    k_in, k_out = cut_kind.count(0), cut_kind.count(1)
    assert V.shape[0] == 4 ** k_in and V.shape[1] == 3 ** k_out and V.shape[3] == 2 ** k_out
    basis_digit, weight = _UP_BASIS[form], _UP_WEIGHT[form]
    down = _DOWN_PAULI if form == "pauli" else _DOWN_EIGEN
    E = np.zeros((4 ** (k_in + k_out), V.shape[2]))
    for row, labels in enumerate(itertools.product(range(4), repeat=k_in + k_out)):
        l_in = [l for l, kd in zip(labels, cut_kind) if kd == 0]
        l_out = [l for l, kd in zip(labels, cut_kind) if kd == 1]
        bi = 0
        for l in l_out:
            bi = 3 * bi + basis_digit[l]
        # weight of each measured bit string: product over the outgoing cuts
        w = np.ones(2 ** k_out)
        for o in range(2 ** k_out):
            for t, lab in enumerate(l_out):
                w[o] *= weight[lab][(o >> (k_out - 1 - t)) & 1]
        for ii, inits in enumerate(itertools.product(range(4), repeat=k_in)):
            coef = 1.0
            for lab, init in zip(l_in, inits):
                coef *= down[lab][init]
            if coef != 0.0:
                E[row] += coef * (V[ii, bi] @ w)
    return E
