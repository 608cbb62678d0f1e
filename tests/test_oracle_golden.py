"""Golden values stated in the paper, reproduced by the oracle."""
import os

import numpy as np

import workloads as W
from oracle import dd

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read(name):
    rows, extra = [], {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0].isdigit():
                rows.append([int(v) for v in parts])
            else:
                extra[parts[0]] = parts[1]
    return rows, extra


def test_fig7_dd_walkthrough():
    rows, extra = _read("fig7_dd_walkthrough.txt")
    # 4 qubits, output |1111> only; subcircuits of 3 qubits: own (1, 1), 2 bridge cuts
    circ = W.bridged_chain((1, 1), (2,), 4, seed=0, x_gates=tuple((0, q) for q in range(4)))
    circ.angles[:] = 0.0
    assert max(s.d for s in circ.subcircuits()) == 3
    recs = dd.reconstruct(W.circuit_entries(circ), circ.cut_map(), n_active=1, n_recursions=4)
    assert len(recs) == len(rows)
    for rec, (r, q, m0, m1) in zip(recs, rows):
        assert rec["active"] == [q]
        assert np.allclose(rec["bins"], [m0, m1], atol=1e-14)
    last = recs[-1]
    state = dict(last["zoom"])
    state[last["active"][0]] = int(np.argmax(last["bins"]))
    assert "".join(str(state[q]) for q in range(4)) == extra["solution"]
