"""Fused cross-entropy gradient (cqc_xent_grad) against the oracle's
cross_entropy / cross_entropy_grad (pinned there by finite differences).

The floor test is taken on p widened to FP64 on both sides, so the zero
pattern of the gradient is exact; each live gradient is one division in the
dtype (<= 2^-24 relative in FP32, 2^-53 in FP64 against the FP64 quotient of
the same inputs); the loss adds one FP64 log per term (relative 1e-12 against
the oracle's numpy sum).  Covers values at, just above and below the floor,
zeros and negatives, ragged sizes and n = 0, unaligned buffers, bitwise
repeatability and graph replay.
"""
import numpy as np
import pytest
import torch

from oracle import adjoint

pytestmark = pytest.mark.gpu
cqc = pytest.importorskip("paper_2012_02333_amd")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _pt(n, seed, np_dt):
    rng = np.random.default_rng(seed)
    p = rng.exponential(1.0, n)
    p /= p.sum()
    t = rng.exponential(1.0, n)
    t /= t.sum()
    if n >= 16:
        k = rng.integers(0, n, n // 8)
        p[k] = 0.0
        p[rng.integers(0, n, n // 16)] = -1e-9                  # negative quasi-probabilities
        p[rng.integers(0, n, 4)] = 1e-30                         # exactly at the floor (FP64)
        p[rng.integers(0, n, 4)] = 2e-30
        p[rng.integers(0, n, 4)] = 5e-31
        t[rng.integers(0, n, n // 10)] = 0.0
    return p.astype(np_dt), t.astype(np_dt)


@pytest.mark.parametrize("n", [0, 1, 5, 4096, 4099, 1000003, 1 << 22])
@pytest.mark.parametrize("dt,np_dt,u", [(torch.float32, np.float32, 2.0 ** -24), (torch.float64, np.float64, 2.0 ** -53)])
def test_xent_grad_matches_oracle(n, dt, np_dt, u):
    _gpu()
    p, t = _pt(n, seed=n % 89 + 1, np_dt=np_dt)
    pd, td = torch.from_numpy(p).cuda(), torch.from_numpy(t).cuda()
    g, loss = cqc.xent_grad(pd, td, with_loss=True)
    p64, t64 = p.astype(np.float64), t.astype(np.float64)
    ref = adjoint.cross_entropy_grad(p64, t64)
    got = g.double().cpu().numpy()
    assert np.array_equal(got == 0, ref == 0)
    assert np.all(np.abs(got - ref) <= u * np.abs(ref))
    L = adjoint.cross_entropy(p64, t64)
    assert abs(float(loss.cpu()) - L) <= 1e-12 * max(1.0, abs(L))


def test_xent_grad_unaligned_repeatable_and_graph():
    _gpu()
    p, t = _pt(300003, seed=3, np_dt=np.float32)
    buf_p = torch.empty(len(p) + 1, dtype=torch.float32, device="cuda")
    buf_p[1:] = torch.from_numpy(p).cuda()
    td = torch.from_numpy(t).cuda()
    pd = torch.from_numpy(p).cuda()
    g1, l1 = cqc.xent_grad(pd, td, with_loss=True)
    g2, l2 = cqc.xent_grad(buf_p[1:], td, with_loss=True)        # scalar path, same grouping
    assert torch.equal(g1, g2) and torch.equal(l1, l2)
    g3, l3 = cqc.xent_grad(pd, td, with_loss=True)
    assert torch.equal(g1, g3) and torch.equal(l1, l3)
    out = torch.empty_like(pd)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        cqc.xent_grad(pd, td, grad=out)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=s):
            cqc.xent_grad(pd, td, grad=out)
    torch.cuda.synchronize()
    for _ in range(3):
        out.fill_(5.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, g1)


def test_xent_grad_arguments():
    _gpu()
    p = torch.ones(8, device="cuda")
    with pytest.raises(ValueError):
        cqc.xent_grad(p, torch.ones(8, device="cuda", dtype=torch.float64))
    with pytest.raises(ValueError):
        cqc.xent_grad(p, torch.ones(9, device="cuda"))
