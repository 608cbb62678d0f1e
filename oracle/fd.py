"""Full-definition (FD) build by its plain definition.

For one cut, p(x) = 1/2 * sum_{i=1..4} p_{1,i} p_{2,i} (Section 3.2.3); with K
cuts every measurement-initialisation combination is evaluated, giving 4^K
Kronecker products (Section 3.3), each factor contributing 1/2 per cut:

    p(x) = 2^-K * sum_{l in {I,X,Y,Z}^K} prod_c E_c[ row_c(l), x_c ]

where row_c(l) is the base-4 number of the labels of the cuts incident to c
(ascending cut id, first = most significant digit) and x_c the bits of x on
c's output qubits (local bit 0 = most significant).  The sum over l is taken
sequentially in ascending l (cut 0 = most significant digit) in FP64, with no
reordering and no pruning.
"""
from __future__ import annotations

import numpy as np


def incident(cut, c):
    return [e for e in range(cut.n_cuts) if cut.edge_up[e] == c or cut.edge_down[e] == c]


def label_digits(l, K):
    """Labels of all K cuts for term index l (cut 0 = most significant digit)."""
    return [(l >> (2 * (K - 1 - e))) & 3 for e in range(K)]


def row_of(cut, c, digits):
    r = 0
    for e in incident(cut, c):
        r = r * 4 + digits[e]
    return r


def local_index(cut, c, xs):
    """x_c for every global index in xs (int64 array)."""
    n = cut.n
    qs = cut.out_qubits_of(c)
    xc = np.zeros_like(xs)
    for q in qs:
        xc = (xc << 1) | ((xs >> (n - 1 - q)) & 1)
    return xc


def reconstruct(entries, cut, xs=None):
    """p at the global indices xs (default: all 2^n), FP64."""
    n, K = cut.n, cut.n_cuts
    if xs is None:
        xs = np.arange(2 ** n, dtype=np.int64)
    xs = np.asarray(xs, dtype=np.int64)
    ents = [np.asarray(E, dtype=np.float64) for E in entries]
    xc = [local_index(cut, c, xs) for c in range(cut.n_sub)]
    acc = np.zeros(xs.shape[0], dtype=np.float64)
    for l in range(4 ** K):
        d = label_digits(l, K)
        term = np.ones(xs.shape[0], dtype=np.float64)
        for c in range(cut.n_sub):
            term = term * ents[c][row_of(cut, c, d)][xc[c]]
        acc = acc + term
    return acc * (2.0 ** -K)


def cost_eq14(f_in_order, K):
    """Eq. 14: L = 4^K * sum_{c=2}^{n_C} prod_{i=1}^{c} 2^{f_i} (multiplications of the build)."""
    total = 0
    for c in range(2, len(f_in_order) + 1):
        prod = 1
        for i in range(c):
            prod *= 2 ** f_in_order[i]
        total += prod
    return (4 ** K) * total


def greedy_order(f):
    """Greedy subcircuit order of Section 4.2: smallest subcircuits first."""
    return sorted(range(len(f)), key=lambda c: (f[c], c))
