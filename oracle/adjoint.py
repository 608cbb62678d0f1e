"""Gradient of a loss on the reconstructed distribution w.r.t. every entry tensor.

p(x) = 2^-K sum_l prod_c E_c[row_c(l), x_c] is linear in each E_c, so with
G = dL/dp the vector-Jacobian product is, by its plain definition,

    dL/dE_c[r, y] = 2^-K * sum_{l : row_c(l) = r}  sum_{x : x_c = y}  G[x] * prod_{c' != c} E_{c'}[row_{c'}(l), x_{c'}]

evaluated term by term (ascending l, then ascending x) in FP64.  The paper has
no gradients; this is the adjoint of its FD build (Section 3.2.3, Section 3.3).
"""
from __future__ import annotations

import numpy as np

from . import fd as _fd

CE_FLOOR = 1e-30


def vjp(entries, cut, G):
    n, K = cut.n, cut.n_cuts
    xs = np.arange(2 ** n, dtype=np.int64)
    ents = [np.asarray(E, dtype=np.float64) for E in entries]
    G = np.asarray(G, dtype=np.float64)
    xc = [_fd.local_index(cut, c, xs) for c in range(cut.n_sub)]
    grads = [np.zeros_like(E) for E in ents]
    for l in range(4 ** K):
        d = _fd.label_digits(l, K)
        rows = [_fd.row_of(cut, c, d) for c in range(cut.n_sub)]
        for c in range(cut.n_sub):
            others = np.ones(2 ** n)
            for c2 in range(cut.n_sub):
                if c2 != c:
                    others = others * ents[c2][rows[c2]][xc[c2]]
            contrib = G * others
            grads[c][rows[c]] += np.bincount(xc[c], weights=contrib, minlength=2 ** cut.f[c])
    return [g * (2.0 ** -K) for g in grads]


def cross_entropy(p, t):
    """L = -sum_x t_x log max(p_x, 1e-30), FP64."""
    p = np.asarray(p, dtype=np.float64)
    return float(-np.sum(np.asarray(t, dtype=np.float64) * np.log(np.maximum(p, CE_FLOOR))))


def cross_entropy_grad(p, t):
    """dL/dp: -t/p where p > 1e-30, else 0 (the floor is flat there)."""
    p = np.asarray(p, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    g = np.zeros_like(p)
    live = p > CE_FLOOR
    g[live] = -t[live] / p[live]
    return g


def vjp_at(entries, cut, G, c, elems):
    """dL/dE_c[r, y] at the (r, y) pairs in `elems`, by the same plain definition
    as vjp: for each pair, the labels l with row_c(l) = r in ascending order,
    and for each l the outputs x with x_c = y (the other qubits enumerated in
    ascending global order) weighted by G[x] and the other factors.

    Costs 4^(K - k_c) * 2^(n - f_c) products per element, so single entries of
    large instances (n = 24) can be checked without the full vjp.
    """
    n, K = cut.n, cut.n_cuts
    ents = [np.asarray(E, dtype=np.float64) for E in entries]
    G = np.asarray(G, dtype=np.float64)
    qs = cut.out_qubits_of(c)
    others = [q for q in range(n) if q not in qs]
    j = np.arange(2 ** len(others), dtype=np.int64)
    free = np.zeros_like(j)
    for t, q in enumerate(others):
        free |= ((j >> (len(others) - 1 - t)) & 1) << (n - 1 - q)
    out = np.empty(len(elems), dtype=np.float64)
    for i, (r, y) in enumerate(elems):
        fixed = 0
        for t, q in enumerate(qs):
            fixed |= ((int(y) >> (len(qs) - 1 - t)) & 1) << (n - 1 - q)
        xs = free | fixed
        g = G[xs]
        xcs = [_fd.local_index(cut, c2, xs) for c2 in range(cut.n_sub)]
        acc = 0.0
        for l in range(4 ** K):
            d = _fd.label_digits(l, K)
            if _fd.row_of(cut, c, d) != int(r):
                continue
            prod = g.copy()
            for c2 in range(cut.n_sub):
                if c2 != c:
                    prod = prod * ents[c2][_fd.row_of(cut, c2, d)][xcs[c2]]
            acc += float(np.sum(prod))
        out[i] = acc * (2.0 ** -K)
    return out
