"""Dynamic definition (Algorithm 1, Section 4.3), plain FP64.

Each recursion labels every output qubit active, merged or zoomed:
  * first recursion: the chosen active qubits (default: the first a qubits in
    output order); nothing zoomed.
  * later recursions: the bin with the largest probability sum is chosen from
    all bins reconstructed so far; its recursion's zoomed qubits stay zoomed
    and its active qubits become zoomed, fixed to the bits of the bin index.
    The next a un-zoomed qubits in output order become active.
  * every remaining qubit is merged.
Subcircuit outputs are then grouped over their merged qubits (summed) with the
zoomed qubits held at their fixed values, and the 2^#active bins are
reconstructed from the merged entries by the FD definition (2^-K times the
sum over all label assignments of the products of merged entries).

Readings where the algorithm is silent:
  * candidate bins are those not yet expanded whose recursion still has merged
    qubits (a bin with no merged qubit is a single state and cannot be refined);
    ties go to the lowest (recursion, bin index).
  * bin index bits follow the active qubits in ascending qubit id, first = most
    significant bit; zoomed values are stored per qubit.
  * the loop stops early when no candidate bin is left.

Search strategies (Section 4.3 describes a depth-first search for sparse
outputs and a breadth-first one for dense outputs without fixing the rule;
the readings here):
  * "heaviest": Algorithm 1 as written - the heaviest candidate over all
    recursions so far.
  * "dfs": the candidates of the most recent recursion that still has any,
    heaviest first; a recursion without merged qubits (a single state) sends
    the search back to the latest recursion with candidates left.  With
    several bins per round, "most recent" means the latest round, and within
    it the earliest (heaviest) pick, so the search continues under the
    heaviest bin it just expanded.
  * "bfs": the candidates of the shallowest zoom depth that still has any,
    heaviest first across the recursions of that depth (ties: lowest
    recursion, then bin).
  * per_round > 1 expands several bins per round from the candidates of the
    recursions that existed when the round began (the multi-bin expansion):
    the best per_round of them in the strategy's order, restricted to the
    first pick's depth (bfs) or recursion (dfs).  For bfs every depth's
    recursions exist before its first bin is expanded, so bfs gives the same
    records for every per_round.
"""
from __future__ import annotations

import numpy as np

from . import fd as _fd

ACTIVE, MERGED = -2, -1


def merge_entries(entries, cut, role):
    """E'_c[r, a_c] = sum over merged local bits of E_c[r, x_c], zoomed bits fixed.

    role[q] in {ACTIVE, MERGED, 0, 1}.  Columns of E'_c enumerate c's active
    bits in local order (first = most significant).
    """
    out = []
    for c in range(cut.n_sub):
        E = np.asarray(entries[c], dtype=np.float64)
        qs = cut.out_qubits_of(c)
        f = len(qs)
        act = [j for j, q in enumerate(qs) if role[q] == ACTIVE]
        cols = np.arange(2 ** f, dtype=np.int64)
        keep = np.ones(2 ** f, dtype=bool)
        for j, q in enumerate(qs):
            if role[q] in (0, 1):
                keep &= ((cols >> (f - 1 - j)) & 1) == role[q]
        a_idx = np.zeros(2 ** f, dtype=np.int64)
        for j in act:
            a_idx = (a_idx << 1) | ((cols >> (f - 1 - j)) & 1)
        Em = np.zeros((E.shape[0], 2 ** len(act)))
        for x in np.nonzero(keep)[0]:          # ascending x_c: fixed summation order
            Em[:, a_idx[x]] += E[:, x]
        out.append(Em)
    return out


def bins_from_merged(merged, cut, role, betas=None):
    """2^#active bins (or the bins at indices `betas`): FD definition over the
    active qubits on merged entries."""
    K = cut.n_cuts
    active = [q for q in range(cut.n) if role[q] == ACTIVE]
    a = len(active)
    beta = (np.arange(2 ** a, dtype=np.int64) if betas is None
            else np.asarray(betas, dtype=np.int64))
    ac = []
    for c in range(cut.n_sub):
        qs = [q for q in cut.out_qubits_of(c) if role[q] == ACTIVE]
        idx = np.zeros_like(beta)
        for q in qs:
            pos = active.index(q)
            idx = (idx << 1) | ((beta >> (a - 1 - pos)) & 1)
        ac.append(idx)
    acc = np.zeros(beta.shape[0])
    for l in range(4 ** K):
        d = _fd.label_digits(l, K)
        term = np.ones(beta.shape[0])
        for c in range(cut.n_sub):
            term = term * merged[c][_fd.row_of(cut, c, d)][ac[c]]
        acc = acc + term
    return acc * (2.0 ** -K)


def reconstruct(entries, cut, n_active, n_recursions, first_active=None, chooser=None,
                strategy="heaviest", per_round=1):
    """Run Algorithm 1.  Returns a list of records (dicts).

    chooser(records, expanded) may override the bin choice (used by parity tests
    to follow the GPU's choice where two masses tie within rounding); default is
    the strategy's rule, applied to the recursions that existed when the round
    began.
    """
    if strategy not in CHOOSERS:
        raise ValueError(f"unknown strategy {strategy!r}")
    n = cut.n
    records, expanded = [], set()
    round_start, round_left, restrict, rnd = 0, 0, None, 0
    for r in range(n_recursions):
        if r == 0:
            active = list(first_active) if first_active is not None else list(range(min(n_active, n)))
            zoom = {}
            parent = (-1, -1)
        else:
            if round_left == 0:
                round_start, round_left, restrict, rnd = len(records), max(1, per_round), None, rnd + 1
            if chooser is not None:
                pick = chooser(records, expanded)
            else:
                pick = CHOOSERS[strategy](records[:round_start], expanded, restrict)
                if pick is None and len(records) > round_start:
                    # the round's candidates ran dry: a new round also sees the
                    # recursions this one made
                    round_start, round_left, restrict, rnd = len(records), max(1, per_round), None, rnd + 1
                    pick = CHOOSERS[strategy](records[:round_start], expanded, None)
            if pick is None:
                break
            round_left -= 1
            if restrict is None:
                restrict = _restriction(strategy, records, pick)
            pr, pb = pick
            expanded.add(pick)
            prev = records[pr]
            zoom = dict(prev["zoom"])
            pa = prev["active"]
            for t, q in enumerate(pa):
                zoom[q] = (pb >> (len(pa) - 1 - t)) & 1
            free = [q for q in range(n) if q not in zoom]
            active = free[:n_active]
            parent = (pr, pb)
        role = [MERGED] * n
        for q, v in zoom.items():
            role[q] = v
        for q in active:
            role[q] = ACTIVE
        merged = merge_entries(entries, cut, role)
        bins = bins_from_merged(merged, cut, role)
        depth = 0 if parent[0] < 0 else records[parent[0]]["depth"] + 1
        records.append(dict(parent=parent, role=role, zoom=zoom, active=sorted(active), depth=depth,
                            round=rnd, bins=bins, has_merged=any(v == MERGED for v in role)))
    return records


def _restriction(strategy, records, pick):
    """What the remaining picks of a round are limited to."""
    if strategy == "bfs":
        return ("depth", records[pick[0]]["depth"])
    if strategy == "dfs":
        return ("rec", pick[0])
    return None


def _candidates(records, expanded):
    """(recursion, bin, mass) of every unexpanded bin of a recursion that
    still has merged qubits."""
    out = []
    for r, rec in enumerate(records):
        if not rec["has_merged"]:
            continue
        for i, v in enumerate(rec["bins"]):
            if (r, i) not in expanded:
                out.append((r, i, float(v)))
    return out


def _mass_key(v):
    return np.inf if np.isnan(v) else -v          # NaN ranks last


def choose_dfs(records, expanded, restrict=None):
    """Heaviest candidate of the most recent recursion that has one: the
    latest round, and in it the earliest pick."""
    cands = _candidates(records, expanded)
    if restrict is not None:
        cands = [c for c in cands if c[0] == restrict[1]]
    if not cands:
        return None
    last = max(records[c[0]]["round"] for c in cands)
    rec = min(c[0] for c in cands if records[c[0]]["round"] == last)
    r, i, _ = min((c for c in cands if c[0] == rec), key=lambda c: (_mass_key(c[2]), c[1]))
    return (r, i)


def choose_bfs(records, expanded, restrict=None):
    """Heaviest candidate of the shallowest depth that has one."""
    cands = _candidates(records, expanded)
    if restrict is not None:
        cands = [c for c in cands if records[c[0]]["depth"] == restrict[1]]
    if not cands:
        return None
    top = min(records[c[0]]["depth"] for c in cands)
    r, i, _ = min((c for c in cands if records[c[0]]["depth"] == top),
                  key=lambda c: (_mass_key(c[2]), c[0], c[1]))
    return (r, i)


def choose_heaviest(records, expanded, restrict=None):
    """Largest bin mass among unexpanded bins of recursions with merged qubits;
    ties -> lowest (recursion, bin)."""
    best, best_val = None, None
    for r, rec in enumerate(records):
        if not rec["has_merged"]:
            continue
        b = np.array(rec["bins"], dtype=np.float64)
        for (er, eb) in expanded:
            if er == r:
                b[eb] = -np.inf
        i = int(np.argmax(b))                # first maximum = lowest index
        if b[i] == -np.inf:
            continue
        if best_val is None or b[i] > best_val:   # strict: earlier recursion wins ties
            best, best_val = (r, i), b[i]
    return best


CHOOSERS = {"heaviest": choose_heaviest, "dfs": choose_dfs, "bfs": choose_bfs}
