"""On-device chi-square distance (Eq. 16, cqc_chi2) against the oracle's
metrics.chi2 (pinned by a hand-computed value): random distributions with
zeros, negative quasi-probabilities and cancelling pairs (a_i + b_i <= 0 is
skipped), ragged and empty sizes, every dtype pair; bitwise repeatable."""
import numpy as np
import pytest
import torch

from oracle import metrics

pytestmark = pytest.mark.gpu
cqc = pytest.importorskip("paper_2012_02333_amd")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _pair(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.exponential(1.0, n)
    b = rng.exponential(1.0, n)
    a /= a.sum()
    b /= b.sum()
    if n >= 8:
        a[rng.integers(0, n, n // 8)] = 0.0          # zeros on one side
        k = rng.integers(0, n, n // 16)
        a[k] = 0.0
        b[k] = 0.0                                   # both zero: skipped
        m = rng.integers(0, n, n // 16)
        a[m] = -rng.exponential(1e-4, len(m))        # negative quasi-probabilities
        c = rng.integers(0, n, n // 32)
        b[c] = -a[c]                                 # a + b == 0: skipped
    return a, b


@pytest.mark.parametrize("n", [0, 1, 7, 4096, 4097, 1000003, 1 << 22])
@pytest.mark.parametrize("da,db", [(torch.float64, torch.float64), (torch.float32, torch.float32),
                                   (torch.float32, torch.float64)])
def test_chi2_matches_oracle(n, da, db):
    _gpu()
    a, b = _pair(n, seed=n % 97)
    ta = torch.from_numpy(a).to(device="cuda", dtype=da)
    tb = torch.from_numpy(b).to(device="cuda", dtype=db)
    got = float(cqc.chi2(ta, tb).cpu())
    ref = metrics.chi2(ta.double().cpu().numpy(), tb.double().cpu().numpy())
    assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)) + 1e-300, (got, ref)


def test_chi2_identical_is_zero_and_repeatable():
    _gpu()
    a, b = _pair(1 << 20, seed=5)
    ta = torch.from_numpy(a).cuda()
    tb = torch.from_numpy(b).cuda()
    assert float(cqc.chi2(ta, ta).cpu()) == 0.0
    r1 = cqc.chi2(ta, tb)
    r2 = cqc.chi2(ta, tb)
    assert torch.equal(r1, r2)


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_chi2_unaligned_equals_aligned(dt):
    """Misaligned inputs take the scalar-load path with the same grouping, so
    the sum is bitwise that of an aligned copy."""
    _gpu()
    a, b = _pair(300007, seed=11)
    ta = torch.from_numpy(a).to(device="cuda", dtype=dt)
    tb = torch.from_numpy(b).to(device="cuda", dtype=dt)
    buf_a = torch.empty(len(a) + 1, dtype=dt, device="cuda")
    buf_b = torch.empty(len(b) + 1, dtype=dt, device="cuda")
    buf_a[1:].copy_(ta)
    buf_b[1:].copy_(tb)
    assert buf_a[1:].data_ptr() % 16 != 0
    assert torch.equal(cqc.chi2(buf_a[1:], buf_b[1:]), cqc.chi2(ta, tb))
    ref = metrics.chi2(ta.double().cpu().numpy(), tb.double().cpu().numpy())
    assert abs(float(cqc.chi2(buf_a[1:], tb).cpu()) - ref) <= 1e-12 * ref
