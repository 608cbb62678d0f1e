"""Seeded "bridged linear chain" random circuits and their cut structure.

A circuit is a chain of qubits laid out as
    own(S_0), bridges_1, own(S_1), bridges_2, ..., own(S_{m-1}).
Every layer applies a U3 gate (angles uniform in [0, 2*pi)) to every qubit and
then CZ on each chain edge whose two qubits have the same owner in that half of
the circuit.  Own qubits of S_j belong to S_j throughout; a bridge between S_j
and S_{j+1} belongs to S_j in the first half (layers < L/2) and to S_{j+1} in
the second half.  Cutting every bridge wire between layer L/2-1 and L/2 (0-based)
therefore splits the circuit exactly into m subcircuits (one wire cut per bridge
qubit, upstream = S_j, downstream = S_{j+1}), which is the situation of the
paper's wire-cutting procedure (Section 3, Figure 3).

This module only describes circuits; it contains no reconstruction arithmetic.
Global qubit q is bit (n-1-q) of an output index (q_0 is the most significant
bit), matching the |q_0 ... q_{n-1}> notation of Section 3.2.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Subcircuit:
    index: int
    q_in: tuple      # incoming bridge qubits (initialised by the cut), ascending
    q_own: tuple     # qubits owned throughout, ascending
    q_out: tuple     # outgoing bridge qubits (measured by the cut), ascending

    @property
    def local_qubits(self):
        """Local simulation order: incoming, own, outgoing (chain order)."""
        return self.q_in + self.q_own + self.q_out

    @property
    def outputs(self):
        """Qubits of this subcircuit that are outputs of the uncut circuit."""
        return self.q_in + self.q_own

    @property
    def f(self):
        return len(self.q_in) + len(self.q_own)

    @property
    def d(self):
        return len(self.q_in) + len(self.q_own) + len(self.q_out)


@dataclass
class CutMap:
    """Cut description in the form the reconstruction library takes.

    f[c]          output qubits of subcircuit c
    edge_up[e]    upstream (measured) subcircuit of cut e
    edge_down[e]  downstream (initialised) subcircuit of cut e
    out_qubit     concatenated over c: local output bit j of c (j = 0 is the
                  most significant bit of x_c) -> global qubit id
    Rows of E_c enumerate the labels of the cuts incident to c in ascending
    cut id, first cut = most significant base-4 digit, I=0, X=1, Y=2, Z=3.
    """
    n: int
    f: list
    edge_up: list
    edge_down: list
    out_qubit: list

    @property
    def n_sub(self):
        return len(self.f)

    @property
    def n_cuts(self):
        return len(self.edge_up)

    def incident(self, c):
        return [e for e in range(self.n_cuts)
                if self.edge_up[e] == c or self.edge_down[e] == c]

    def k(self, c):
        return len(self.incident(c))

    def entry_shape(self, c):
        return (4 ** self.k(c), 2 ** self.f[c])

    def out_qubits_of(self, c):
        s = sum(self.f[:c])
        return list(self.out_qubit[s:s + self.f[c]])


@dataclass
class BridgedChain:
    own: tuple
    bridges: tuple
    layers: int
    angles: np.ndarray = field(repr=False)   # (L, n, 3): theta, phi, lambda
    x_gates: tuple = ()                       # optional extra X gates: (layer, qubit)

    @property
    def n(self):
        return int(sum(self.own) + sum(self.bridges))

    @property
    def m(self):
        return len(self.own)

    def _segments(self):
        own_ranges, bridge_ranges = [], []
        q = 0
        for j in range(self.m):
            own_ranges.append(tuple(range(q, q + self.own[j])))
            q += self.own[j]
            if j < self.m - 1:
                bridge_ranges.append(tuple(range(q, q + self.bridges[j])))
                q += self.bridges[j]
        return own_ranges, bridge_ranges

    def owner(self, q, half):
        own_ranges, bridge_ranges = self._segments()
        for j, r in enumerate(own_ranges):
            if q in r:
                return j
        for j, r in enumerate(bridge_ranges):
            if q in r:
                return j if half == 0 else j + 1
        raise ValueError(q)

    def half_of(self, layer):
        return 0 if layer < self.layers // 2 else 1

    def cz_edges(self, half):
        return [(q, q + 1) for q in range(self.n - 1)
                if self.owner(q, half) == self.owner(q + 1, half)]

    def subcircuits(self):
        own_ranges, bridge_ranges = self._segments()
        subs = []
        for j in range(self.m):
            q_in = bridge_ranges[j - 1] if j > 0 else ()
            q_out = bridge_ranges[j] if j < self.m - 1 else ()
            subs.append(Subcircuit(j, tuple(q_in), own_ranges[j], tuple(q_out)))
        return subs

    def cut_qubits(self):
        _, bridge_ranges = self._segments()
        return [q for r in bridge_ranges for q in r]

    def cut_map(self):
        subs = self.subcircuits()
        edge_up, edge_down = [], []
        _, bridge_ranges = self._segments()
        for j, r in enumerate(bridge_ranges):
            for _q in r:
                edge_up.append(j)
                edge_down.append(j + 1)
        out_qubit = [q for s in subs for q in s.outputs]
        return CutMap(self.n, [s.f for s in subs], edge_up, edge_down, out_qubit)

    def gate_list(self):
        """The uncut circuit as an ordered gate list.

        ("u3", q, theta, phi, lam), ("cz", q, q+1), ("x", q).  Each gate carries
        the layer and half it belongs to as the last two fields.
        """
        gates = []
        for t in range(self.layers):
            h = self.half_of(t)
            for q in range(self.n):
                th, ph, la = self.angles[t, q]
                gates.append(("u3", q, float(th), float(ph), float(la), t, h))
            for (layer, q) in self.x_gates:
                if layer == t:
                    gates.append(("x", q, t, h))
            for (a, b) in self.cz_edges(h):
                gates.append(("cz", a, b, t, h))
        return gates

    def subcircuit_gates(self, sub: Subcircuit):
        """Gates of the uncut circuit that belong to subcircuit `sub`."""
        out = []
        for g in self.gate_list():
            h = g[-1]
            qs = g[1:3] if g[0] == "cz" else (g[1],)
            if all(self.owner(q, h) == sub.index for q in qs):
                out.append(g)
        return out


def bridged_chain(own, bridges, layers, seed, x_gates=()):
    """Seeded circuit: angles drawn layer-major, then qubit, then (theta, phi, lambda)."""
    own = tuple(int(v) for v in own)
    bridges = tuple(int(v) for v in bridges)
    if len(bridges) != len(own) - 1:
        raise ValueError("need one bridge count per boundary")
    if layers % 2:
        raise ValueError("layers must be even (the cut sits at the middle)")
    n = sum(own) + sum(bridges)
    rng = np.random.default_rng(seed)
    angles = rng.uniform(0.0, 2.0 * np.pi, size=(layers, n, 3))
    return BridgedChain(own, bridges, layers, angles, tuple(x_gates))
