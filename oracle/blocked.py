"""Full FD vectors in bounded memory: pairwise contraction over output blocks (FP64).

TEST INFRASTRUCTURE ONLY (like the rest of this package): it exists to give
full-vector references at sizes where the per-output definition in fd.py is
too slow (a 2^30-output vector with 4096 terms).

The FD build (Section 3.2.3 for one cut, Section 3.3 for K cuts) is

    p(x) = 2^-K * sum_{l in {I,X,Y,Z}^K} prod_c E_c[ row_c(l), x_c ].

Every cut label appears in exactly two factors of each product: those of its
upstream and its downstream subcircuit.  By distributivity the sum over a label
can therefore be taken as soon as both of those factors have been multiplied
together.  This module multiplies the subcircuits together in index order
(0, 1, 2, ...), keeping the labels of cuts that still lead to a subcircuit not
yet included as open indices, and sums each label when its second subcircuit
joins: one FP64 matrix product per subcircuit, over the shared labels.  This is
the progressive Kronecker build that Eq. 14 counts, with each label summed as
early as it can be (the greedy contraction idea of Section 4.2).

Outputs are produced block by block: block b fixes the top `top_bits` global
qubits to the bits of b (qubit 0 is the most significant bit of x), so block b
is the contiguous range [b * 2^(n - top_bits), (b + 1) * 2^(n - top_bits)) of
the global vector, and each factor only contributes its columns whose fixed
bits match.  Blocks are independent, so memory stays at one block.

The result equals fd.reconstruct up to FP64 rounding (the order of the label
sum differs); tests pin it to fd.reconstruct and to brute-force state vectors
for n <= 16.
"""
from __future__ import annotations

import numpy as np


def _columns(E, qs, fixed):
    """Columns of E whose bits on fixed qubits match; they stay in ascending
    order, so the kept column index enumerates the remaining bits in local order."""
    f = len(qs)
    cols = np.arange(2 ** f, dtype=np.int64)
    keep = np.ones(2 ** f, dtype=bool)
    for j, q in enumerate(qs):
        if q in fixed:
            keep &= ((cols >> (f - 1 - j)) & 1) == fixed[q]
    return E[:, keep], [q for q in qs if q not in fixed]


def reconstruct_block(entries, cut, top_bits, block):
    """p at global indices block * 2^(n - top_bits) + j, j = 0 .. 2^(n - top_bits) - 1 (FP64)."""
    n, K = cut.n, cut.n_cuts
    if not 0 <= top_bits <= n or not 0 <= block < 2 ** top_bits:
        raise ValueError("bad block")
    fixed = {q: (block >> (top_bits - 1 - q)) & 1 for q in range(top_bits)}
    open_cuts, bits, P = None, [], None
    for c in range(cut.n_sub):
        E = np.asarray(entries[c], dtype=np.float64)
        Ec, qs = _columns(E, cut.out_qubits_of(c), fixed)
        inc = cut.incident(c)
        Y = Ec.shape[1]
        if P is None:
            open_cuts, bits, P = inc, qs, Ec.reshape((4,) * len(inc) + (Y,))
            continue
        X = P.shape[-1]
        shared = [e for e in open_cuts if e in inc]
        a = [e for e in open_cuts if e not in shared]
        b = [e for e in inc if e not in shared]
        # P as [a labels][shared labels][X], E_c as [shared labels][b labels][Y]
        Pt = np.transpose(P, [open_cuts.index(e) for e in a + shared] + [len(open_cuts)])
        Pt = Pt.reshape(4 ** len(a), 4 ** len(shared), X)
        Et = np.transpose(Ec.reshape((4,) * len(inc) + (Y,)),
                          [inc.index(e) for e in shared + b] + [len(inc)])
        Et = Et.reshape(4 ** len(shared), 4 ** len(b) * Y)
        # sum over the shared labels: one matrix product
        R = np.transpose(Pt, (0, 2, 1)).reshape(4 ** len(a) * X, 4 ** len(shared)) @ Et
        R = R.reshape(4 ** len(a), X, 4 ** len(b), Y).transpose(0, 2, 1, 3)
        new_open = a + b
        R = R.reshape((4,) * len(new_open) + (X * Y,))
        order = sorted(new_open)
        P = np.transpose(R, [new_open.index(e) for e in order] + [len(new_open)])
        open_cuts, bits = order, bits + qs
    if open_cuts:
        raise ValueError("a cut does not join two distinct subcircuits")
    v = P.reshape(-1) * (2.0 ** -K)
    # bits holds the global qubit of every axis of v (most significant first);
    # put the axes in ascending global qubit order
    if len(bits) == 0:
        return v
    t = v.reshape((2,) * len(bits))
    return np.ascontiguousarray(np.transpose(t, np.argsort(bits))).reshape(-1)


def blocks(entries, cut, top_bits):
    """Yield (block, p_block) for every block of the global vector, in order."""
    for b in range(2 ** top_bits):
        yield b, reconstruct_block(entries, cut, top_bits, b)


def reconstruct(entries, cut):
    """The whole 2^n vector (one block)."""
    return reconstruct_block(entries, cut, 0, 0)
