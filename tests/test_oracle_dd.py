"""Pins of the DD oracle (Algorithm 1): bins equal brute-force marginals,
refinements conserve mass, a deterministic circuit is located with mass 1 in n
recursions of one active qubit (the 4-qubit BV walk-through of Section 6.2)."""
import numpy as np
import pytest

import workloads as W
from oracle import dd, fd, statevector as sv


def _marginal(p, n, role):
    """Brute-force bin masses for a role vector (ACTIVE / MERGED / 0 / 1)."""
    active = [q for q in range(n) if role[q] == dd.ACTIVE]
    xs = np.arange(2 ** n)
    keep = np.ones(2 ** n, dtype=bool)
    for q in range(n):
        if role[q] in (0, 1):
            keep &= ((xs >> (n - 1 - q)) & 1) == role[q]
    idx = np.zeros(2 ** n, dtype=np.int64)
    for q in active:
        idx = (idx << 1) | ((xs >> (n - 1 - q)) & 1)
    return np.bincount(idx[keep], weights=p[keep], minlength=2 ** len(active))


@pytest.mark.parametrize("own,bridges,layers,a", [((4, 3), (1,), 4, 3), ((3, 2, 3), (2, 2), 6, 4),
                                                 ((4, 4, 4), (1, 2), 4, 5)])
def test_every_recursion_equals_marginal(own, bridges, layers, a):
    inst = W.make_instance(own, bridges, layers, seed=42)
    p = sv.uncut_distribution(inst.circuit)
    recs = dd.reconstruct(inst.entries, inst.cut, n_active=a, n_recursions=4)
    assert len(recs) == 4
    for rec in recs:
        ref = _marginal(p, inst.n, rec["role"])
        assert np.max(np.abs(rec["bins"] - ref)) < 1e-13
    assert abs(recs[0]["bins"].sum() - 1.0) < 1e-13


def test_refinement_conserves_parent_mass():
    inst = W.make_instance((4, 4, 4), (2, 1), 6, seed=7)
    recs = dd.reconstruct(inst.entries, inst.cut, n_active=3, n_recursions=6)
    for rec in recs[1:]:
        pr, pb = rec["parent"]
        assert abs(rec["bins"].sum() - recs[pr]["bins"][pb]) < 1e-13


def test_heaviest_rule_and_first_active():
    inst = W.make_instance((3, 3), (2,), 4, seed=3)
    p = sv.uncut_distribution(inst.circuit)
    n = inst.n
    recs = dd.reconstruct(inst.entries, inst.cut, n_active=2, n_recursions=3,
                          first_active=[5, 1])
    assert recs[0]["active"] == [1, 5]
    b0 = recs[0]["bins"]
    # recursion 2 refines the heaviest recursion-1 bin
    assert recs[1]["parent"] == (0, int(np.argmax(b0)))
    # recursion 2's active qubits: first two un-zoomed qubits in output order
    assert recs[1]["active"] == [0, 2]
    assert abs(recs[1]["bins"].sum() - b0.max()) < 1e-13
    # bins are marginals
    for rec in recs:
        assert np.max(np.abs(rec["bins"] - _marginal(p, n, rec["role"]))) < 1e-13


def test_deterministic_circuit_located_in_n_recursions():
    # angles zero + X gates: the uncut output is one basis state
    own, bridges = (2, 2), (1,)
    target = [1, 0, 1, 1, 0]
    xg = tuple((0, q) for q, b in enumerate(target) if b)
    circ = W.bridged_chain(own, bridges, 4, seed=0, x_gates=xg)
    circ.angles[:] = 0.0
    ents = W.circuit_entries(circ)
    cut = circ.cut_map()
    recs = dd.reconstruct(ents, cut, n_active=1, n_recursions=cut.n)
    assert len(recs) == cut.n
    for r, rec in enumerate(recs):
        # one active qubit per recursion: bins (0, 1) or (1, 0) exactly
        assert sorted(np.round(rec["bins"], 12).tolist()) == [0.0, 1.0]
        assert rec["active"] == [r]
        assert int(np.argmax(rec["bins"])) == target[r]
    final = recs[-1]
    zoom = dict(final["zoom"])
    zoom[final["active"][0]] = int(np.argmax(final["bins"]))
    assert [zoom[q] for q in range(cut.n)] == target


def test_all_active_is_fd():
    inst = W.make_instance((3, 3), (1,), 4, seed=5)
    recs = dd.reconstruct(inst.entries, inst.cut, n_active=inst.n, n_recursions=2)
    assert len(recs) == 1                   # nothing merged: no bin can be refined
    assert np.max(np.abs(recs[0]["bins"] - fd.reconstruct(inst.entries, inst.cut))) < 1e-15


def test_sampled_bins_match_full():
    inst = W.make_instance((3, 2, 3), (2, 1), 4, seed=9)
    recs = dd.reconstruct(inst.entries, inst.cut, n_active=4, n_recursions=2)
    rec = recs[1]
    merged = dd.merge_entries(inst.entries, inst.cut, rec["role"])
    betas = [0, 3, 7, 15]
    assert np.array_equal(dd.bins_from_merged(merged, inst.cut, rec["role"], betas),
                          rec["bins"][betas])


# ---- search strategies, pinned to brute-force marginals of the uncut state
# vector walked in the order the strategy names (a recursive pre-order walk
# for DFS, a level-order walk for BFS), not to the oracle's own selection code

def _prefix_masses(p, n, k):
    """Mass of every value of the first k qubits (index = their bits)."""
    return p.reshape(2 ** k, 2 ** (n - k)).sum(axis=1)


def _preorder(p, n, a, limit):
    """Zoom tree in depth-first pre-order, children heaviest first: the list
    of zoomed prefixes (bit strings of the first d*a qubits) of each visited
    recursion.  Default active sets are the next a qubits in order."""
    order = []

    def visit(prefix):
        if len(order) == limit:
            return
        order.append(prefix)
        k = len(prefix) + a
        if k >= n:                              # nothing merged: a leaf
            return
        child = _prefix_masses(p, n, k).reshape(2 ** len(prefix), 2 ** a)
        row = child[int(prefix, 2) if prefix else 0]
        for b in sorted(range(2 ** a), key=lambda b: (-row[b], b)):
            visit(prefix + format(b, f"0{a}b"))
    visit("")
    return order


def _zoom_prefix(rec, n):
    z = rec["zoom"]
    return "".join(str(z[q]) for q in range(len(z)))


def test_dfs_is_preorder_walk():
    inst = W.make_instance((3, 2), (2,), 6, seed=21)          # n = 7, a = 2: depth 3 is a leaf
    p = sv.uncut_distribution(inst.circuit)
    R = 14
    recs = dd.reconstruct(inst.entries, inst.cut, 2, R, strategy="dfs")
    assert [_zoom_prefix(r, inst.n) for r in recs] == _preorder(p, inst.n, 2, R)
    for rec in recs:
        assert np.max(np.abs(rec["bins"] - _marginal(p, inst.n, rec["role"]))) < 1e-13


def test_dfs_multi_bin_round():
    """per_round = 3: the first round expands the three heaviest first-recursion
    bins; the next round goes down under the heaviest of them, taking its
    children heaviest first."""
    inst = W.make_instance((3, 2), (2,), 6, seed=22)
    p = sv.uncut_distribution(inst.circuit)
    recs = dd.reconstruct(inst.entries, inst.cut, 2, 6, strategy="dfs", per_round=3)
    top = sorted(range(4), key=lambda b: (-_prefix_masses(p, inst.n, 2)[b], b))
    assert [r["parent"] for r in recs[1:4]] == [(0, b) for b in top[:3]]
    m4 = _prefix_masses(p, inst.n, 4).reshape(4, 4)[top[0]]
    kids = sorted(range(4), key=lambda b: (-m4[b], b))
    assert [r["parent"] for r in recs[4:6]] == [(1, kids[0]), (1, kids[1])]


@pytest.mark.parametrize("per_round", [1, 3, 7])
def test_bfs_is_level_order(per_round):
    """BFS: all first-recursion bins heaviest first, then the heaviest depth-2
    bins over every depth-1 recursion; the same for every per_round."""
    inst = W.make_instance((2, 2), (2,), 6, seed=23)          # n = 6, a = 2
    p = sv.uncut_distribution(inst.circuit)
    n, R = inst.n, 1 + 4 + 6
    recs = dd.reconstruct(inst.entries, inst.cut, 2, R, strategy="bfs", per_round=per_round)
    assert len(recs) == R
    m2, m4 = _prefix_masses(p, n, 2), _prefix_masses(p, n, 4)
    lvl1 = sorted(range(4), key=lambda b: (-m2[b], b))
    assert [_zoom_prefix(r, n) for r in recs[1:5]] == [format(b, "02b") for b in lvl1]
    # depth 2: six heaviest 4-bit prefixes (ties: lower recursion, then bin)
    rec_of = {b: 1 + lvl1.index(b) for b in range(4)}
    lvl2 = sorted(range(16), key=lambda x: (-m4[x], rec_of[x >> 2], x & 3))[:6]
    assert [_zoom_prefix(r, n) for r in recs[5:]] == [format(x, "04b") for x in lvl2]
    for rec in recs:
        assert np.max(np.abs(rec["bins"] - _marginal(p, n, rec["role"]))) < 1e-13


def test_heaviest_multi_bin_round():
    """per_round = 2 under the heaviest rule: the first round takes the two
    heaviest first-recursion bins; later picks see every recursion."""
    inst = W.make_instance((3, 2), (2,), 6, seed=24)
    p = sv.uncut_distribution(inst.circuit)
    n = inst.n
    recs = dd.reconstruct(inst.entries, inst.cut, 2, 5, per_round=2)
    m2 = _prefix_masses(p, n, 2)
    top = sorted(range(4), key=lambda b: (-m2[b], b))
    assert [r["parent"] for r in recs[1:3]] == [(0, top[0]), (0, top[1])]
    # the second expansion round: the two heaviest of {the remaining first-recursion bins} and
    # {the depth-2 bins under top[0], top[1]}, all as brute-force masses
    m4 = _prefix_masses(p, n, 4)
    pool = [(m2[b], 0, b) for b in top[2:]] + [(m4[4 * top[j] + b], 1 + j, b) for j in range(2) for b in range(4)]
    pool.sort(key=lambda t: (-t[0], t[1], t[2]))
    assert [r["parent"] for r in recs[3:5]] == [(t[1], t[2]) for t in pool[:2]]


@pytest.mark.parametrize("strategy", ["dfs", "bfs"])
def test_strategies_locate_deterministic_state(strategy):
    own, bridges = (2, 2), (1,)
    target = [0, 1, 1, 0, 1]
    circ = W.bridged_chain(own, bridges, 4, seed=0, x_gates=tuple((0, q) for q, b in enumerate(target) if b))
    circ.angles[:] = 0.0
    cut = circ.cut_map()
    recs = dd.reconstruct(W.circuit_entries(circ), cut, 1, cut.n, strategy=strategy)
    if strategy == "dfs":                       # straight down the one non-zero path
        assert len(recs) == cut.n
        for r, rec in enumerate(recs):
            assert rec["active"] == [r] and int(np.argmax(rec["bins"])) == target[r]
    else:                                       # level order: both bins of every level
        assert [r["depth"] for r in recs[:3]] == [0, 1, 1]
        assert recs[1]["parent"] == (0, target[0])
    assert abs(recs[0]["bins"].sum() - 1.0) < 1e-13


def test_unknown_strategy():
    inst = W.make_instance((2, 2), (1,), 4, seed=1)
    with pytest.raises(ValueError):
        dd.reconstruct(inst.entries, inst.cut, 2, 2, strategy="random")


@pytest.mark.parametrize("case", ["recursion1", "zoomed", "permuted"])
def test_c_twin_dd_merge_and_bins_bitwise(case):
    """The C/OpenMP twin of the DD merge and bins (used for CPU timing) equals
    the Python oracle bit for bit: same additions in the same order."""
    from oracle import native
    if case == "permuted":
        cut = W.CutMap(n=10, f=[4, 3, 3], edge_up=[0, 1, 0], edge_down=[1, 2, 2],
                       out_qubit=[7, 2, 9, 0, 5, 3, 8, 1, 4, 6])
        ents = W.random_entries(cut, seed=44)
    else:
        inst = W.make_instance((3, 2, 3), (2, 2), 4, seed=45)
        cut, ents = inst.cut, inst.entries
    n = cut.n
    role = [dd.MERGED] * n
    if case == "recursion1":
        for q in range(4):
            role[q] = dd.ACTIVE
    else:
        for q, v in ((0, 1), (3, 0), (5, 1)):
            role[q] = v
        for q in (1, 2, 6, 8):
            role[q] = dd.ACTIVE
    m_py = dd.merge_entries(ents, cut, role)
    m_c = native.dd_merge(ents, cut, role, threads=4)
    for a, b in zip(m_py, m_c):
        assert np.array_equal(a, b)
    b_py = dd.bins_from_merged(m_py, cut, role)
    assert np.array_equal(native.dd_bins(m_c, cut, role, threads=3), b_py)
    sel = np.array([0, 3, 7, 15], dtype=np.int64)
    assert np.array_equal(native.dd_bins(m_c, cut, role, sel), b_py[sel])
