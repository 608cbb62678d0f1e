"""Seeded workload recipes for the reconstruction path.

C1  FD, plain FP64:   own (4,3), bridges (1),  L=4  -> n=8,  K=1, f=(4,4)
C2  FD, GEMM form:    own (11,11), bridges (2), L=8 -> n=24, K=2, f=(11,13)
C3  FD, chain:        own (9,6,9), bridges (3,3), L=10 -> n=30, K=6, f=(9,9,12)
C4  DD:               own (9,7,7,9), bridges (3,2,3), L=10 -> n=40, K=8,
                      f=(9,10,9,12), 2^20 active bins, 5 recursions
C5  batched+adjoint:  256 instances, n ~ U{12..24}, K ~ U{1..4}, 2-3 subcircuits,
                      L=8, Dirichlet(1) cross-entropy targets

Entries come from noiseless simulation of the subcircuits (entries.py); targets
and output samples are plain seeded random numbers.  Nothing here reconstructs.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .circuits import bridged_chain, BridgedChain, CutMap
from .entries import circuit_entries


@dataclass
class Instance:
    name: str
    circuit: BridgedChain
    cut: CutMap
    entries: list  # FP64 numpy arrays

    @property
    def n(self):
        return self.cut.n

    @property
    def K(self):
        return self.cut.n_cuts


RECIPES = {
    "c1": dict(own=(4, 3), bridges=(1,), layers=4, seed=1),
    "c2": dict(own=(11, 11), bridges=(2,), layers=8, seed=2),
    "c3": dict(own=(9, 6, 9), bridges=(3, 3), layers=10, seed=3),
    "c4": dict(own=(9, 7, 7, 9), bridges=(3, 2, 3), layers=10, seed=4),
}

DD_C4 = dict(n_active=20, n_recursions=5)

# DD at the paper's large-circuit scale (Section 6.2, Figure 10: one recursion
# of 2^35 bins for circuits of up to 100 qubits): a 100-qubit chain of five
# 20-qubit subcircuits, two cuts per boundary (K = 8).  No simulation produces
# 100-qubit entries, so they are seeded signed random values of the right
# shapes (not uniform distributions, whose bins would all be equal).
DD_SCALE = dict(n=100, f=(20, 20, 20, 20, 20), cuts_per_boundary=2, n_active=35, n_recursions=1, seed=35)


def make_instance(own, bridges, layers, seed, name="custom", x_gates=()):
    circ = bridged_chain(own, bridges, layers, seed, x_gates=x_gates)
    return Instance(name, circ, circ.cut_map(), circuit_entries(circ))


def config_instance(name):
    return make_instance(name=name, **RECIPES[name])


def _split_even(total, parts, minimum):
    base = [minimum] * parts
    rest = total - minimum * parts
    for i in range(rest):
        base[i % parts] += 1
    return base


def batch_recipes(count=256, seed=5, n_lo=12, n_hi=24, k_lo=1, k_hi=4, layers=8):
    """Shapes of the batched workload: n ~ U{n_lo..n_hi}, K ~ U{k_lo..k_hi}, n_C ~ U{2,3}."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(n_lo, n_hi + 1))
        K = int(rng.integers(k_lo, k_hi + 1))
        nc = int(rng.integers(2, 4))
        if K == 1:
            nc = 2
        bridges = _split_even(K, nc - 1, 1)
        own = _split_even(n - K, nc, 1)
        out.append(dict(own=tuple(own), bridges=tuple(bridges), layers=layers,
                        seed=10_000 + i))
    return out


def batch_instances(count=256, seed=5, **kw):
    return [make_instance(name=f"b{i}", **r)
            for i, r in enumerate(batch_recipes(count, seed, **kw))]


def dirichlet_target(n, seed):
    """Dirichlet(1) target over 2^n outcomes: normalised Exp(1) draws (FP64)."""
    rng = np.random.default_rng(seed)
    e = rng.exponential(1.0, size=2 ** n)
    return e / e.sum()


def sample_outputs(n, count, seed):
    """Seeded sample of distinct output indices in [0, 2^n), sorted."""
    rng = np.random.default_rng(seed)
    if 2 ** n <= count:
        return np.arange(2 ** n, dtype=np.int64)
    s = set()
    while len(s) < count:
        s.update(int(v) for v in rng.integers(0, 2 ** n, size=count - len(s)))
    return np.array(sorted(s), dtype=np.int64)


def dd_scale_instance(seed=None):
    """The DD_SCALE cut and its FP32 entries (uniform in [-1, 1) times 2^-f_c),
    drawn directly in FP32: about 3 GiB."""
    r = DD_SCALE
    m = len(r["f"])
    up = [c for c in range(m - 1) for _ in range(r["cuts_per_boundary"])]
    down = [c + 1 for c in up]
    cut = CutMap(r["n"], list(r["f"]), up, down, list(range(r["n"])))
    rng = np.random.default_rng(r["seed"] if seed is None else seed)
    ents = []
    for c in range(cut.n_sub):
        rows, w = cut.entry_shape(c)
        E = rng.random((rows, w), dtype=np.float32)
        E *= np.float32(2.0)
        E -= np.float32(1.0)
        E *= np.float32(2.0 ** -cut.f[c])
        ents.append(E)
    return cut, ents


def random_entries(cut: CutMap, seed, zero_rows=(), scale=None):
    """Unstructured signed entries of the right shapes (no simulation behind them).

    zero_rows: iterable of (c, row) forced to exactly zero, to exercise early
    termination.  Values are uniform in [-1, 1) times 2^-f_c unless scale given.
    """
    rng = np.random.default_rng(seed)
    ents = []
    for c in range(cut.n_sub):
        r, w = cut.entry_shape(c)
        s = 2.0 ** -cut.f[c] if scale is None else scale
        ents.append(rng.uniform(-1.0, 1.0, size=(r, w)) * s)
    for (c, row) in zero_rows:
        ents[c][row, :] = 0.0
    return ents


def sample_variant_shots(V, shots, seed):
    """Finite-shot variant distributions: every variant's distribution over
    (output bits, measured cut bits) of V [4^k_in][3^k_out][2^f][2^k_out]
    replaced by seeded multinomial counts / shots."""
    rng = np.random.default_rng(seed)
    out = np.empty_like(V)
    for i in range(V.shape[0]):
        for j in range(V.shape[1]):
            p = np.clip(V[i, j].ravel(), 0.0, None)
            p = p / p.sum()
            out[i, j] = (rng.multinomial(shots, p) / shots).reshape(V.shape[2:])
    return out


def random_variants(k_in, k_out, f, seed):
    """Seeded synthetic variant distributions [4^k_in][3^k_out][2^f][2^k_out]:
    each variant a normalised Exp(1) draw over its 2^(f + k_out) outcomes."""
    rng = np.random.default_rng(seed)
    V = rng.exponential(1.0, size=(4 ** k_in, 3 ** k_out, 2 ** f, 2 ** k_out))
    return V / V.sum(axis=(2, 3), keepdims=True)
