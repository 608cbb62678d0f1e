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
