"""GPU parity of dynamic definition (Algorithm 1) against the FP64 oracle.

Bins: relative L1 <= 1e-12 (FP64 form) or <= 1e-6 (FP32 form) per recursion,
plus the element-wise rounding bound.  Where two bin masses tie within the
FP32 error, either choice is correct (reading of the bin rule), so the oracle
follows the GPU's choice of parent and the choice itself is checked to be the
heaviest unexpanded bin of the GPU's own masses.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import dd, fd, metrics
from tests.gpu_util import to_dev, oracle_inputs, U32, U64

pytestmark = pytest.mark.gpu
cqc = pytest.importorskip("paper_2012_02333_amd")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run(entries_np, wcut, a, R, prec, dtype, first=None):
    host, dev = to_dev(entries_np, dtype)
    cut = cqc.CutMap.from_workload(wcut)
    bins, recs = cqc.reconstruct_dd(dev, cut, a, R, first_active=first, precision=prec)
    torch.cuda.synchronize()
    return host, bins.cpu().numpy(), recs


def _follow(gpu_recs):
    def chooser(records, expanded):
        r = len(records)
        if r >= len(gpu_recs):
            return None
        return tuple(gpu_recs[r]["parent"])
    return chooser


def _check_heaviest(bins, recs):
    """Each parent is the heaviest unexpanded bin (GPU masses), ties to lowest (rec, bin)."""
    expanded = set()
    for r in range(1, len(recs)):
        best, best_key = None, None
        for k in range(r):
            if all(v != -1 for v in recs[k]["role"]):
                continue                                  # no merged qubit
            nb = 2 ** recs[k]["n_active"]
            for i in range(nb):
                if (k, i) in expanded:
                    continue
                key = (-bins[k, i], k, i)
                if best_key is None or key < best_key:
                    best, best_key = (k, i), key
        assert tuple(recs[r]["parent"]) == best, (r, recs[r]["parent"], best)
        expanded.add(best)


@pytest.mark.parametrize("prec,dtype,tol", [("fp64", torch.float64, 1e-12), ("fp32", torch.float32, 1e-6),
                                            ("bf16x6", torch.float32, 1e-6)])
@pytest.mark.parametrize("shape,a,R", [(((4, 3), (1,), 4), 3, 4), (((3, 2, 3), (2, 2), 6), 4, 6),
                                       (((4, 4, 4), (1, 2), 4), 5, 5), (((3, 3), (2,), 4), 2, 12)])
def test_dd_matches_oracle(shape, a, R, prec, dtype, tol):
    _gpu()
    own, bridges, layers = shape
    inst = W.make_instance(own, bridges, layers, seed=42)
    host, bins, recs = _run(inst.entries, inst.cut, a, R, prec, dtype)
    e64 = oracle_inputs(host)
    ref = dd.reconstruct(e64, inst.cut, a, R, chooser=_follow(recs))
    assert len(ref) == len(recs)
    _check_heaviest(bins, recs)
    for r, (g, o) in enumerate(zip(recs, ref)):
        assert g["role"] == o["role"], r
        nb = 2 ** g["n_active"]
        got = bins[r, :nb]
        err = metrics.rel_l1(got, o["bins"])
        assert err <= tol, (r, err)
        assert abs(g["mass"] - o["bins"].sum()) <= tol * np.abs(o["bins"]).sum() + 1e-15
        if r > 0:
            pr, pb = g["parent"]
            assert abs(got.sum() - bins[pr, pb]) <= 10 * tol * max(1e-300, abs(bins[pr, pb])) + 1e-14


@pytest.mark.parametrize("prec,dtype", [("fp64", torch.float64), ("fp32", torch.float32)])
def test_dd_locates_deterministic_state(prec, dtype):
    _gpu()
    target = [1, 0, 1, 1, 0, 1, 1]
    circ = W.bridged_chain((3, 2), (2,), 4, seed=0, x_gates=tuple((0, q) for q, b in enumerate(target) if b))
    circ.angles[:] = 0.0
    cut = circ.cut_map()
    host, bins, recs = _run(W.circuit_entries(circ), cut, 1, cut.n, prec, dtype)
    assert len(recs) == cut.n
    for r, rec in enumerate(recs):
        assert rec["active"] == [r]
        assert np.allclose(bins[r, :2], [1 - target[r], target[r]], atol=1e-6)
    assert abs(recs[0]["mass"] - 1.0) < 1e-6


def test_dd_first_active_and_refill():
    """Explicit first active set; many recursions so that the candidate list of
    the first recursion is consumed and refilled."""
    _gpu()
    inst = W.make_instance((4, 4), (2,), 4, seed=7)
    first = [9, 2, 5, 0]
    host, bins, recs = _run(inst.entries, inst.cut, 4, 20, "fp64", torch.float64, first=first)
    assert recs[0]["active"] == sorted(first)
    assert sum(1 for r in recs if r["parent"][0] == 0) > 8      # first list consumed, refilled
    ref = dd.reconstruct(oracle_inputs(host), inst.cut, 4, 20, first_active=first)
    assert [tuple(r["parent"]) for r in recs] == [r["parent"] for r in ref]
    for r, o in enumerate(ref):
        assert np.max(np.abs(bins[r, :len(o["bins"])] - o["bins"])) < 1e-14


def test_dd_c4_n40():
    """n=40, K=8, four 12-qubit subcircuits, 2^20 active bins, 5 recursions (FP32
    term sum, FP64 bins): sampled bins against the oracle's per-bin definition,
    recursion-1 total mass 1, refinements conserve their parent's mass."""
    _gpu()
    inst = W.config_instance("c4")
    a, R = W.DD_C4["n_active"], W.DD_C4["n_recursions"]
    host, bins, recs = _run(inst.entries, inst.cut, a, R, "fp32", torch.float32)
    assert len(recs) == R
    _check_heaviest(bins, recs)
    e64 = oracle_inputs(host)
    assert abs(recs[0]["mass"] - 1.0) < 1e-5
    for r, g in enumerate(recs):
        role = g["role"]
        merged = dd.merge_entries(e64, inst.cut, role)
        nb = 2 ** g["n_active"]
        betas = np.unique(np.concatenate([W.sample_outputs(g["n_active"], 48, seed=r), [int(np.argmax(bins[r, :nb]))]]))
        ref = dd.bins_from_merged(merged, inst.cut, role, betas)
        got = bins[r, betas]
        T = dd.bins_from_merged([np.abs(m) for m in merged], inst.cut, role, betas)
        assert np.all(np.abs(got - ref) <= 4 * (256 + 2) * U32 * T + 1e-300), r
        assert metrics.rel_l1(got, ref) <= 1e-6
        if r > 0:
            pr, pb = g["parent"]
            assert abs(bins[r, :nb].sum() - bins[pr, pb]) <= 1e-5 * abs(bins[pr, pb])


def test_dd_bad_arguments():
    _gpu()
    inst = W.make_instance((3, 3), (1,), 4, seed=1)
    host, dev = to_dev(inst.entries, torch.float32)
    cut = cqc.CutMap.from_workload(inst.cut)
    with pytest.raises(cqc.CqcError) as e:
        cqc.reconstruct_dd(dev, cut, 0, 2)
    assert e.value.code == 1
    with pytest.raises(cqc.CqcError) as e:
        cqc.reconstruct_dd(dev, cut, 2, 2, first_active=[1, 1])
    assert e.value.code == 1


# ---- search strategies and multi-bin rounds

def _replay_picks(bins, recs, strategy, per_round):
    """The parents the strategy's rule gives on the GPU's own bin masses, with
    the round structure of the call (picks from the recursions that existed
    when the round began)."""
    fake = [dict(bins=bins[r, :2 ** g["n_active"]], has_merged=any(v == -1 for v in g["role"]),
                 depth=g["depth"], round=0) for r, g in enumerate(recs)]
    choose = dd.CHOOSERS[strategy]
    expanded, parents = set(), [(-1, -1)]
    made, start, left, restrict, rnd = 1, 1, 0, None, 0
    while made < len(recs):
        if left == 0:
            start, left, restrict, rnd = made, per_round, None, rnd + 1
        pick = choose(fake[:start], expanded, restrict)
        if pick is None and made > start:
            start, left, restrict, rnd = made, per_round, None, rnd + 1
            pick = choose(fake[:start], expanded, None)
        fake[made]["round"] = rnd
        assert pick is not None
        left -= 1
        if restrict is None and strategy != "heaviest":
            restrict = ("depth", fake[pick[0]]["depth"]) if strategy == "bfs" else ("rec", pick[0])
        expanded.add(pick)
        parents.append(pick)
        made += 1
    return parents


@pytest.mark.parametrize("strategy", ["heaviest", "dfs", "bfs"])
@pytest.mark.parametrize("per_round", [1, 4])
@pytest.mark.parametrize("prec,dtype,tol", [("fp64", torch.float64, 1e-12), ("fp32", torch.float32, 1e-6)])
def test_dd_strategies_match_oracle(strategy, per_round, prec, dtype, tol):
    _gpu()
    inst = W.make_instance((3, 2, 3), (2, 2), 6, seed=31)        # n = 12, a = 3: depth 3 has no merged qubit
    a, R = 3, 13
    host, dev = to_dev(inst.entries, dtype)
    cut = cqc.CutMap.from_workload(inst.cut)
    bins, recs = cqc.reconstruct_dd(dev, cut, a, R, precision=prec, strategy=strategy, bins_per_round=per_round)
    bins = bins.cpu().numpy()
    assert len(recs) == R
    assert [tuple(r["parent"]) for r in recs] == _replay_picks(bins, recs, strategy, per_round)
    e64 = oracle_inputs(host)
    ref = dd.reconstruct(e64, inst.cut, a, R, chooser=_follow(recs))
    for r, (g, o) in enumerate(zip(recs, ref)):
        assert g["role"] == o["role"] and g["depth"] == o["depth"], r
        nb = 2 ** g["n_active"]
        assert metrics.rel_l1(bins[r, :nb], o["bins"]) <= tol, r
        assert abs(g["mass"] - o["bins"].sum()) <= tol * np.abs(o["bins"]).sum() + 1e-15
    if prec == "fp64":     # no near-ties at this seed: the oracle's own choices agree
        free = dd.reconstruct(e64, inst.cut, a, R, strategy=strategy, per_round=per_round)
        assert [tuple(r["parent"]) for r in recs] == [r["parent"] for r in free]


def test_dd_bfs_rounds_do_not_change_records():
    """BFS: every depth's recursions exist before its first bin is expanded, so
    one bin per round and five per round give bitwise the same bins."""
    _gpu()
    inst = W.make_instance((4, 4), (2,), 4, seed=32)
    host, dev = to_dev(inst.entries, torch.float32)
    cut = cqc.CutMap.from_workload(inst.cut)
    b1, r1 = cqc.reconstruct_dd(dev, cut, 3, 20, strategy="bfs", bins_per_round=1)
    b5, r5 = cqc.reconstruct_dd(dev, cut, 3, 20, strategy="bfs", bins_per_round=5)
    assert [r["parent"] for r in r1] == [r["parent"] for r in r5]
    assert torch.equal(b1, b5)
    assert [r["depth"] for r in r1[:9]] == [0] + [1] * 8          # all of recursion 1's bins first


def test_dd_dfs_locates_deterministic_state():
    """One active qubit, two bins per round: every round expands both bins of
    the heaviest newest recursion, so the state is pinned one qubit per round."""
    _gpu()
    target = [0, 1, 1, 0, 1, 0, 1]
    circ = W.bridged_chain((3, 2), (2,), 4, seed=0, x_gates=tuple((0, q) for q, b in enumerate(target) if b))
    circ.angles[:] = 0.0
    cut = circ.cut_map()
    n = cut.n
    host, dev = to_dev(W.circuit_entries(circ), torch.float32)
    bins, recs = cqc.reconstruct_dd(dev, cqc.CutMap.from_workload(cut), 1, 1 + 2 * (n - 1), strategy="dfs",
                                    bins_per_round=2)
    bins = bins.cpu().numpy()
    heavy = [g for g in recs if g["mass"] > 0.5]
    assert len(heavy) == n
    last = max(heavy, key=lambda g: g["depth"])
    assert last["depth"] == n - 1
    assert [last["role"][q] for q in range(n - 1)] == target[:n - 1]
    assert int(np.argmax(bins[recs.index(last), :2])) == target[n - 1]


def test_dd_strategy_arguments():
    _gpu()
    inst = W.make_instance((3, 3), (1,), 4, seed=1)
    host, dev = to_dev(inst.entries, torch.float32)
    cut = cqc.CutMap.from_workload(inst.cut)
    with pytest.raises(ValueError):
        cqc.reconstruct_dd(dev, cut, 2, 2, strategy="random")
    with pytest.raises(cqc.CqcError) as e:
        cqc.reconstruct_dd(dev, cut, 2, 2, bins_per_round=65)
    assert e.value.code == 1


@pytest.mark.parametrize("strategy,per_round", [("heaviest", 1), ("heaviest", 4), ("dfs", 1), ("dfs", 4),
                                                ("bfs", 1)])
@pytest.mark.parametrize("prec,dtype", [("fp64", torch.float64), ("fp32", torch.float32)])
def test_dd_exact_ties_go_to_lowest_index(strategy, per_round, prec, dtype):
    """A uniform distribution (only the all-identity row is non-zero, every
    entry 1): all 4096 first-recursion bins tie exactly, so every ranking -
    within a thread, across a wave, across blocks and after a refill of the
    candidate list - must order them by index, and the records are exactly
    the oracle's own, bins included."""
    _gpu()
    cut = W.CutMap(16, [8, 8], [0], [1], list(range(16)))
    ents = [np.zeros((4, 256)), np.zeros((4, 256))]
    ents[0][0] = 1.0
    ents[1][0] = 1.0
    a, R = 12, 12                      # eleven picks: more than one top-8 list
    host, dev = to_dev(ents, dtype)
    bins, recs = cqc.reconstruct_dd(dev, cqc.CutMap.from_workload(cut), a, R, precision=prec,
                                    strategy=strategy, bins_per_round=per_round)
    bins = bins.cpu().numpy()
    ref = dd.reconstruct(oracle_inputs(host), cut, a, R, strategy=strategy, per_round=per_round)
    assert [tuple(r["parent"]) for r in recs] == [r["parent"] for r in ref]
    assert [tuple(r["parent"]) for r in recs][1:4] == [(0, 0), (0, 1), (0, 2)]
    for r, (g, o) in enumerate(zip(recs, ref)):
        assert g["role"] == o["role"], r
        nb = 2 ** g["n_active"]
        assert np.array_equal(bins[r, :nb], o["bins"]), r
        assert g["mass"] == o["bins"].sum(), r


def test_dd_concurrent_queries_on_two_streams():
    """Two host threads run DD queries at once, each on its own stream: the
    shared plan cache and the pool of page-locked read-back buffers serve both,
    and every query returns the records of a query run alone."""
    import threading
    _gpu()
    inst = W.make_instance((3, 2, 3), (2, 2), 6, seed=31)
    host, dev = to_dev(inst.entries, torch.float32)
    cut = cqc.CutMap.from_workload(inst.cut)
    ref_bins, ref_recs = cqc.reconstruct_dd(dev, cut, 3, 9, precision="fp32", bins_per_round=2)
    ref_bins = ref_bins.cpu()
    results, errors = [[], []], []

    def worker(k):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for _ in range(6):
                    b, r = cqc.reconstruct_dd(dev, cut, 3, 9, precision="fp32", bins_per_round=2)
                    s.synchronize()
                    results[k].append((b.cpu(), r))
        except Exception as e:          # reported below, in the main thread
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for k in range(2):
        assert len(results[k]) == 6
        for b, r in results[k]:
            assert torch.equal(b, ref_bins)
            assert [(g["parent"], g["mass"]) for g in r] == [(g["parent"], g["mass"]) for g in ref_recs]
