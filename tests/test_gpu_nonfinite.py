"""Non-finite entries: NaN and Inf propagate to exactly the outputs whose term
sum contains them, and the FP64 mass reports them; early termination of an
all-zero factor row skips the terms that row multiplies, including a NaN
factor they would have met (the behaviour the C ABI documents: with finite
entries pruning changes nothing, with Inf/NaN the skipped product would have
been NaN)."""
import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu
cqc = pytest.importorskip("paper_2012_02333_amd")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run(cut, ents, prec):
    dt = torch.float64 if prec == "fp64" else torch.float32
    _, dev = to_dev(ents, dt)
    p, mass = cqc.reconstruct_fd(dev, cqc.CutMap.from_workload(cut), precision=prec)
    torch.cuda.synchronize()
    return p.double().cpu().numpy().reshape(2 ** cut.f[0], 2 ** cut.f[1]), float(mass.cpu())


@pytest.mark.parametrize("prec", ["fp32", "fp64", "bf16x6"])
@pytest.mark.parametrize("bad", [np.nan, np.inf])
@pytest.mark.parametrize("ncuts", [2, 3])
def test_nonfinite_entry_reaches_exactly_its_outputs(prec, bad, ncuts):
    """Two subcircuits, outputs blocked as [x_A][x_B]: a non-finite
    E_A[r][y] enters every term of every output with x_A = y (row r is live,
    and E_B's rows are non-zero), and no other output."""
    _gpu()
    cut = W.CutMap(16, [8, 8], [0] * ncuts, [1] * ncuts, list(range(16)))
    ents = W.random_entries(cut, seed=71)
    y = 37
    ents[0][5, y] = bad
    p, mass = _run(cut, ents, prec)
    assert not np.isfinite(p[y]).any()
    others = np.delete(p, y, axis=0)
    assert np.isfinite(others).all()
    assert not np.isfinite(mass)
    if bad != bad:                      # NaN stays NaN
        assert np.isnan(p[y]).all()


@pytest.mark.parametrize("prec", ["fp32", "bf16x6"])
def test_pruned_zero_row_skips_a_nan_factor(prec):
    """Three shared cuts (64 terms, the step prunes): E_B's row 9 is all zero,
    so term 9 is skipped and the NaN in E_A's row 9 never reaches an output,
    where the unpruned product NaN * 0 would have been NaN everywhere in that
    column.  A NaN in a live row still propagates."""
    _gpu()
    cut = W.CutMap(22, [11, 11], [0, 0, 0], [1, 1, 1], list(range(22)))
    ents = W.random_entries(cut, seed=72, zero_rows=((1, 9),))
    ents[0][9, 100] = np.nan
    p, mass = _run(cut, ents, prec)
    assert np.isfinite(p).all() and np.isfinite(mass)
    ents[0][10, 200] = np.nan          # row 10 of E_B is live
    p, mass = _run(cut, ents, prec)
    assert np.isnan(p[200]).all()
    assert np.isfinite(np.delete(p, 200, axis=0)).all()
