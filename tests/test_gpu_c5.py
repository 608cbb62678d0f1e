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



def _c5_setup(prec):
    insts = W.batch_instances(256)
    cuts = [cqc.CutMap.from_workload(i.cut) for i in insts]
    npdt = np.float32 if prec == "fp32" else np.float64
    ent_np = [[E.astype(np.float32).astype(npdt) for E in i.entries] for i in insts]
    ents = [[torch.from_numpy(E).cuda() for E in e] for e in ent_np]
    tgts = [torch.from_numpy(W.dirichlet_target(i.n, 1000 + k).astype(np.float32).astype(npdt)).cuda()
            for k, i in enumerate(insts)]
    xb = cqc.Batch(ents, cuts, precision=prec, targets=tgts, keep_outputs=False, with_mass=False)
    bwd = cqc.BatchBackward(xb, xb.grads)
    xb.run()
    bwd.run()
    torch.cuda.synchronize()
    big = [k for k, i in enumerate(insts) if i.n == 24 and i.K == 4]
    rng = np.random.default_rng(77)
    rest = [k for k in range(len(insts)) if k not in big]
    chosen = big + [int(k) for k in rng.choice(rest, size=3, replace=False)]
    return insts, cuts, ent_np, tgts, xb, bwd, chosen, rng


def _central(call, E, r, y, h, loss):
    v0 = float(E[r, y])
    E[r, y] = v0 + h
    call.run()
    lp = loss(call.outs[0])
    E[r, y] = v0 - h
    call.run()
    lm = loss(call.outs[0])
    E[r, y] = v0
    return (lp - lm) / (2 * h)


def _central_log1p(call, E, r, y, h, t):
    """Central difference of L = -sum t log max(p, 1e-30) in E[r, y], the
    change of L summed output by output, and the largest relative change of
    an output with t > 0 over the step."""
    v0 = float(E[r, y])
    E[r, y] = v0 + h
    call.run()
    pp = torch.clamp(call.outs[0], min=1e-30).clone()
    E[r, y] = v0 - h
    call.run()
    pm = torch.clamp(call.outs[0], min=1e-30)
    E[r, y] = v0
    u = ((pp - pm).abs() / (2 * torch.minimum(pp, pm)))[t > 0].max()
    return float(-(t * torch.log1p((pp - pm) / pm)).sum()) / (2 * h), float(u)


def test_c5_fp32_gradients_match_fp64_finite_differences():
    """The configured check of the batched training step, on its FP32 form:
    the step's entry gradients (cross-entropy gradient written by the
    forward's final kernels, then the adjoint) against FP64 central finite
    differences of the linear loss L_G(E) = sum_x G_x p_x(E), G the dL/dp the
    step itself computed (widened exactly).  p is linear in each entry, so the
    central difference is exact up to FP64 rounding; the FP64 forward used for
    it is the oracle-checked one, at the FP32 entries widened exactly.  Sampled
    entry elements of every n = 24, K = 4 instance and three seeded others.

    Bar: relative L2 over each instance's sampled elements <= 1e-5 (the FP32
    adjoint's rounding, as against the oracle's VJP).  The cross-entropy
    itself is compared end to end in FP64 by the next test: against FP64 p,
    -t/p at outputs that cancel to near zero (K = 4, 256 signed terms) takes
    FP32 p's rounding relative to a tiny p, or the floor, so an FP32 step and an
    FP64 loss need not agree there."""
    _gpu()
    insts, cuts, ent_np, tgts, xb, bwd, chosen, rng = _c5_setup("fp32")
    print("c5 fd: fused FP32 step done", flush=True)
    for k in chosen:
        inst = insts[k]
        e64 = [torch.from_numpy(E.astype(np.float64)).cuda() for E in ent_np[k]]
        G = xb.grads[k].double()
        call = cqc.FDCall(e64, cuts[k], precision="fp64", with_mass=False)
        got, ref = [], []
        for c in range(inst.cut.n_sub):
            E = e64[c]
            h = float(E.abs().max())
            rows, cols = inst.cut.entry_shape(c)
            for _ in range(4):
                r, y = int(rng.integers(rows)), int(rng.integers(cols))
                ref.append(_central(call, E, r, y, h, lambda p: float((G * p).sum())))
                got.append(float(bwd.grads[k][c][r, y]))
        err = metrics.rel_l2(np.array(got), np.array(ref))
        print(f"c5 fd instance {k}: n={inst.n} K={inst.K} n_C={inst.cut.n_sub} rel_l2={err:.2e}", flush=True)
        assert err <= 1e-5, (k, err)


def test_c5_fp64_step_matches_fp64_finite_differences_of_cross_entropy():
    """The same training step in FP64 (FP64 forward writing the cross-entropy
    gradient, FP64 adjoint) against FP64 central differences of the
    cross-entropy L = -sum t log max(p, 1e-30) itself, at sampled elements of
    the same instances.  p is linear in each entry (p +- h a), so the central
    difference of L per output is (a / p)(1 + (h a / p)^2 / 3 + ...): outputs
    that cancel to near zero make that curvature term large, so the step is
    tiny (h = 1e-9 |E|max), the h^2 term is removed by Richardson extrapolation
    (4 D(h/2) - D(h)) / 3 (leaving about u^4 / 20, u = max h a / p, which the
    test measures and bounds), and each difference L(E + h) - L(E - h) is
    formed output by output as -t log1p((p+ - p-) / p-), exact for nearly
    equal p, instead of as the difference of two sums of about 17.  Bar:
    relative L2 <= 1e-6 per instance (FP64 rounding of p+ - p- is about
    1e-16 sum|terms| against 2 h dp/dE, about 1e-7 relative at this h)."""
    _gpu()
    insts, cuts, ent_np, tgts, xb, bwd, chosen, rng = _c5_setup("fp64")
    print("c5 fd: fused FP64 step done", flush=True)
    for k in chosen:
        inst = insts[k]
        e64 = [torch.from_numpy(E).cuda() for E in ent_np[k]]
        t64 = tgts[k]
        call = cqc.FDCall(e64, cuts[k], precision="fp64", with_mass=False)
        got, ref, u = [], [], 0.0
        for c in range(inst.cut.n_sub):
            E = e64[c]
            h = 1e-9 * float(E.abs().max())
            rows, cols = inst.cut.entry_shape(c)
            for _ in range(4):
                r, y = int(rng.integers(rows)), int(rng.integers(cols))
                (d1, u1), (d2, _) = (_central_log1p(call, E, r, y, s, t64) for s in (h, h / 2))
                ref.append((4 * d2 - d1) / 3)
                got.append(float(bwd.grads[k][c][r, y]))
                u = max(u, u1)
        err = metrics.rel_l2(np.array(got), np.array(ref))
        print(f"c5 fd64 instance {k}: n={inst.n} K={inst.K} n_C={inst.cut.n_sub} "
              f"max h a/p {u:.1e} rel_l2={err:.2e}", flush=True)
        # the step stays well inside every output's distance to zero
        assert u <= 0.05, (k, u)
        assert err <= 1e-6, (k, err)
