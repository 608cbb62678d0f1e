"""The batched training step at its full size: 256 seeded cut instances
(n ~ U{12..24}, K ~ U{1..4}, two or three subcircuits), forward, cross-entropy
gradient against Dirichlet(1) targets and adjoint, captured in one graph and
replayed - the step the benchmark times.

Checks, on a seeded sample of instances that includes every n = 24, K = 4
instance (two and three subcircuits):
  * every graph replay reproduces the eager step bit for bit;
  * forward outputs on sampled indices against the oracle's per-output
    definition: relative L1 <= 1e-6 and every element within its rounding
    bound;
  * gradients on sampled entry elements against the oracle's element-wise
    plain-definition VJP fed the same dL/dp (the step's own, widened):
    relative L2 over each entry tensor's sample <= 1e-5.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import adjoint, metrics, native
from tests.gpu_util import oracle_inputs, elementwise_ok, U32

pytestmark = pytest.mark.gpu
cqc = pytest.importorskip("paper_2012_02333_amd")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_c5_step_graph_forward_and_gradients():
    _gpu()
    insts = W.batch_instances(256)
    print("c5: instances built", flush=True)
    cuts = [cqc.CutMap.from_workload(i.cut) for i in insts]
    e32 = [[E.astype(np.float32) for E in i.entries] for i in insts]
    ents = [[torch.from_numpy(E).cuda() for E in e] for e in e32]
    sizes = [2 ** i.n for i in insts]
    p_flat = torch.empty(sum(sizes), dtype=torch.float32, device="cuda")
    g_flat = torch.empty_like(p_flat)
    t_flat = torch.from_numpy(np.concatenate(
        [W.dirichlet_target(i.n, 1000 + k).astype(np.float32) for k, i in enumerate(insts)])).cuda()
    outs = list(torch.split(p_flat, sizes))
    gouts = list(torch.split(g_flat, sizes))
    batch = cqc.Batch(ents, cuts, precision="fp32", outs=outs)
    bwd = cqc.BatchBackward(batch, gouts)

    def body():
        batch.run()
        cqc.xent_grad(p_flat, t_flat, grad=g_flat)
        bwd.run()

    body()
    torch.cuda.synchronize()
    eager_p = p_flat.clone()
    eager_g = [[g.clone() for g in gl] for gl in bwd.grads]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        body()
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=s):
            body()
    torch.cuda.synchronize()
    for rep in range(2):
        p_flat.fill_(-1.0)
        for gl in bwd.grads:
            for g in gl:
                g.fill_(7.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(p_flat, eager_p), rep
        for k in range(len(insts)):
            for c in range(len(eager_g[k])):
                assert torch.equal(bwd.grads[k][c], eager_g[k][c]), (rep, k, c)
    print("c5: graph replays equal the eager step", flush=True)

    big = [k for k, i in enumerate(insts) if i.n == 24 and i.K == 4]
    assert {insts[k].cut.n_sub for k in big} == {2, 3}
    rng = np.random.default_rng(55)
    rest = [k for k in range(len(insts)) if k not in big]
    chosen = big + [int(k) for k in rng.choice(rest, size=4, replace=False)]
    for k in chosen:
        inst = insts[k]
        e64 = oracle_inputs(e32[k])
        xs = W.sample_outputs(inst.n, 2048, seed=5000 + k)
        got = outs[k][torch.from_numpy(xs).cuda()].double().cpu().numpy()
        ref = native.reconstruct(e64, inst.cut, xs)
        T = native.reconstruct([np.abs(E) for E in e64], inst.cut, xs)
        err = metrics.rel_l1(got, ref)
        _, macs = cqc.cost(cuts[k])
        ok, info = elementwise_ok(got, ref, T, U32, max(4, int(round(macs / 2 ** inst.n))))
        # the adjoint is judged on the dL/dp the step itself computed (FP32,
        # from the FP32 p), widened exactly; -t/p amplifies p's rounding at tiny p
        G = gouts[k].double().cpu().numpy()
        gerrs = []
        for c in range(inst.cut.n_sub):
            rows, cols = inst.cut.entry_shape(c)
            elems = [(int(rng.integers(rows)), int(rng.integers(cols))) for _ in range(12)]
            gref = adjoint.vjp_at(e64, inst.cut, G, c, elems)
            gg = bwd.grads[k][c].double().cpu().numpy()
            ggot = np.array([gg[r, y] for r, y in elems])
            gerrs.append(metrics.rel_l2(ggot, gref))
        print(f"c5 instance {k}: n={inst.n} K={inst.K} n_C={inst.cut.n_sub} fwd rel_l1={err:.2e} "
              f"grad rel_l2={max(gerrs):.2e}", flush=True)
        assert err <= 1e-6, k
        assert ok, (k, info)
        assert max(gerrs) <= 1e-5, (k, gerrs)
