"""Throughput benchmark of the cut-circuit reconstruction hot path on one MI355X.

Default workload (the headline metric): n=24 seeded random U3+CZ circuit
(depth 8) cut by K=2 wires into two 13-qubit subcircuits; entry tensors
16 x 2^11 and 16 x 2^13 from noiseless simulation; 2^24 output probabilities.
A step is one complete library call: the term sum on matrix cores (all 16
terms are kept: with at most 16 terms a dead term only adds exact zeros, so no
row-flag pass runs), the single write of every output with per-tile FP64
partial sums, and the ordered FP64 total mass.  The FP32 form (metric) and the plain FP64 form run on the same inputs;
output buffers rotate over >= 1 GiB so the 256 MB last-level cache cannot hold
the writes.

Prints ONE JSON line.  `--config` selects another workload of the same family
(its own line, same fields):
  c3  FD fused chain, n=30, K=6, three 12-qubit subcircuits (FP32, BF16X6, BF16X3, FP64)
  c4  DD, n=40, K=8, 2^20 bins per recursion, 5 recursions (FP32, FP64 bins)
  c5  256 instances (n 12..24, K 1..4) forward + cross-entropy adjoint, one
      graph-captured step
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFS = 157.3
METRIC = "FD reconstructed probs/s n=24,K=2: MFMA-FP32 vs plain FP64 at 1e-6 rel err"

WORKLOAD = {
    "c2": "FD n=24 K=2, two 13-qubit subcircuits, E 16x2^11 and 16x2^13",
    "c3": "FD n=30 K=6, three 12-qubit subcircuits (fused chain), 4096 terms",
    "c4": "DD n=40 K=8, four 12-qubit subcircuits, 2^20 bins per recursion, 5 recursions",
    "c5": "256 FD instances n~U{12..24} K~U{1..4} 2-3 subcircuits: forward + cross-entropy adjoint",
    "entries": "entry construction from variant distributions: two 22-output-qubit subcircuits joined by 2 cuts",
    "chi2": "chi-square distance (Eq. 16) of two 2^28-outcome FP32 distributions",
    "dd35": "DD n=100 K=8, five 20-qubit subcircuits, one recursion of 2^35 FP32 bins",
}

# kernel sources whose change invalidates a committed HBM-counter record
TRAFFIC_SOURCES = {
    "c2": ["paper_2012_02333_amd/csrc/k_contract.hip", "paper_2012_02333_amd/csrc/kernels.hpp"],
    "c3": ["paper_2012_02333_amd/csrc/k_wide.hip", "paper_2012_02333_amd/csrc/kernels.hpp"],
}


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default per config)")
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--config", default="c2", choices=["c2", "c3", "c4", "c5", "entries", "chi2", "dd35"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--calibrate", action="store_true",
                    help="first run kernels of known HBM traffic (reference for the counters)")
    return ap.parse_args()


def kernel_source_hash(config):
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES.get(config, []):
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(config, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None if there is none or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{config}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_sha") != kernel_source_hash(config) or rec.get("kernel") != kernel:
        return None
    return rec.get("hbm_bytes_per_launch")


def _sync_time(fn, steps, warmup, torch):
    """Warm up, then time exactly `steps` calls of fn(i) between synchronised events."""
    for i in range(warmup):
        fn(i)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for i in range(steps):
        fn(i)
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def _traced(fn, steps, cqc, torch):
    """Per-kernel (launches, summed ms) from the start and stop events each
    launch's dispatch records (the kernels' own run times)."""
    with cqc.trace() as tr:
        for i in range(steps):
            fn(i)
        torch.cuda.synchronize()
    return tr.result


def _roof(bound, achieved, peak, unit, kernel, avg_ms, traffic):
    return {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
            "traffic": traffic, "kernel": kernel, "kernel_avg_us": avg_ms * 1e3}


def _line(cfg, metric, value, unit, steps, warmup, ms, dtype, config, roofline, higher=True, **extra):
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
           "ms_per_step": ms, "higher_is_better": higher, "scaling": "weak", "vs_baseline": None,
           "dtype": dtype, "data": "synthetic", "config": dict(workload=WORKLOAD[cfg], **config),
           "roofline": roofline}
    out.update(extra)
    return out


def _cpu_rate(run_sample, unit_count, seconds, sample0):
    """Time the oracle on growing samples until one takes >= seconds / 4, then
    repeat it to about `seconds`; returns (rate, sample size, reps, elapsed)."""
    size = sample0
    while True:
        t0 = time.perf_counter()
        run_sample(size)
        el = time.perf_counter() - t0
        if el >= seconds / 4 or size >= unit_count:
            break
        size = min(unit_count, size * max(2, int(seconds / 4 / max(el, 1e-3))))
    reps, t0 = 0, time.perf_counter()
    while True:
        run_sample(size)
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds or reps >= 100000:
            break
    return reps * size / el, size, reps, el


def _cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), for the baseline record."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


# ---------------------------------------------------------------------------
def bench_fd(args, cfg, torch, cqc, W):
    """c2 (headline) and c3: full-definition reconstruction of one instance."""
    inst = W.config_instance(cfg)
    n, K = inst.n, inst.K
    cut = cqc.CutMap.from_workload(inst.cut)
    e32_np = [E.astype(np.float32) for E in inst.entries]
    e32 = [torch.from_numpy(E).cuda() for E in e32_np]
    e64 = [torch.from_numpy(E).cuda() for E in inst.entries]
    N = 2 ** n
    steps = args.steps or (200 if cfg == "c2" else 10)
    warmup = args.warmup if args.warmup is not None else (20 if cfg == "c2" else 3)

    def measure(prec, ents, dt):
        esz = 8 if dt == torch.float64 else 4
        nbuf = max(2, min(16, (1 << 30) // (esz * N)))
        outs = [torch.empty(N, dtype=dt, device="cuda") for _ in range(nbuf)]
        call = cqc.FDCall(ents, cut, precision=prec, outs=[outs[0]])

        def step(i):
            call.set_outputs([outs[i % nbuf]])
            call.run()
        ms = _sync_time(step, steps, warmup, torch)
        kt = _traced(step, steps, cqc, torch)
        last = outs[(steps - 1) % nbuf]
        sample = None
        if n <= 26:
            sample = last.double().cpu().numpy()
        else:
            xs = W.sample_outputs(n, 1 << 14, seed=7)
            sample = (xs, last[torch.from_numpy(xs).cuda()].double().cpu().numpy())
        res = {"value": N / (ms * 1e-3), "ms_per_step": ms, "kernels_ms": kt,
               "mass": float(call.mass[0].cpu()), "output_buffers_rotated": nbuf}
        del outs, call
        torch.cuda.empty_cache()
        return res, sample

    r32, s32 = measure("fp32", e32, torch.float32)
    single = None
    if cfg == "c2":
        # the same step writing one output buffer every time (its 64 MiB can
        # stay in the Infinity Cache): labelled, never the headline value
        one = torch.empty(N, dtype=torch.float32, device="cuda")
        call1 = cqc.FDCall(e32, cut, precision="fp32", outs=[one])
        ms1 = _sync_time(lambda i: call1.run(), steps, warmup, torch)
        single = {"value": N / (ms1 * 1e-3), "ms_per_step": ms1, "output_buffers_rotated": 1}
        del one, call1
    rbf, sbf = measure("bf16x6", e32, torch.float32)
    # the two-part split (accuracy/speed study): only where steps have more
    # than 16 terms does it differ from FP32
    r3, s3 = measure("bf16x3", e32, torch.float32) if cfg != "c2" else (None, None)
    r64, s64 = measure("fp64", e64, torch.float64)

    def dominant(kt, prefix=None):
        items = [(k, v) for k, v in kt.items() if prefix is None or k.startswith(prefix)]
        name, (cnt, tot) = max(items, key=lambda kv: kv[1][1])
        return name, tot / cnt

    in_bytes = sum(E.numel() * 4 for E in e32)
    if cfg == "c2":
        name, avg = dominant(r32["kernels_ms"])
        roof = _roof("hbm", (4 * N + in_bytes) / (avg * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s", name, avg,
                     recorded_traffic(cfg, name))
        name_b, avg_b = dominant(rbf["kernels_ms"])
        roof_bf = _roof("hbm", (4 * N + in_bytes) / (avg_b * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s", name_b, avg_b, None)
    else:
        # final contraction: 2 * (live terms) * 2^n flops; output written once
        name, avg = dominant(r32["kernels_ms"], "wide_f32_final")
        _, macs = cqc.cost(cut)
        flops_final = 2.0 * 64 * N   # 4^3 shared labels of the last contraction x 2^30 outputs
        roof = _roof("mfma", flops_final / (avg * 1e-3) / 1e12, FP32_PEAK_TFS, "TFLOP/s", name, avg,
                     recorded_traffic(cfg, name))
        roof["flops_per_launch"] = flops_final
        roof["plan_flops_per_step"] = 2.0 * macs
        name_b, avg_b = dominant(rbf["kernels_ms"], "wide_bf16x6_final")
        roof_bf = _roof("hbm", (4 * N) / (avg_b * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s", name_b, avg_b, None)
        name_3, avg_3 = dominant(r3["kernels_ms"], "wide_bf16x3_final")
        roof_3 = _roof("hbm", (4 * N) / (avg_3 * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s", name_3, avg_3, None)

    metric = METRIC if cfg == "c2" else "FD reconstructed probs/s n=30,K=6 fused chain: MFMA-FP32 at 1e-6 rel err"
    out = _line(cfg, metric, r32["value"], "probs/s", steps, warmup, r32["ms_per_step"], "f32",
                {"n": n, "K": K, "precision": "fp32", "seed": W.RECIPES[cfg]["seed"],
                 "output_buffers_rotated": r32["output_buffers_rotated"]},
                roof, mass=r32["mass"], kernels_ms=r32["kernels_ms"],
                fp64_plain={k: r64[k] for k in ("value", "ms_per_step", "kernels_ms", "mass")},
                bf16x6={**{k: rbf[k] for k in ("value", "ms_per_step", "kernels_ms", "mass")}, "roofline": roof_bf})
    out["speedup_fp32_vs_fp64"] = r32["value"] / r64["value"]
    out["speedup_bf16x6_vs_fp64"] = rbf["value"] / r64["value"]
    if single is not None:
        out["fp32_single_output_buffer"] = single
    if r3 is not None:
        out["bf16x3"] = {**{k: r3[k] for k in ("value", "ms_per_step", "kernels_ms", "mass")}, "roofline": roof_3}
        out["speedup_bf16x3_vs_fp64"] = r3["value"] / r64["value"]

    if not args.no_cpu:
        from oracle import native, metrics  # CPU-baseline leg only
        e64_np = [E.astype(np.float64) for E in e32_np]
        threads = native.max_threads()
        if n <= 26:
            ref = native.reconstruct(e64_np, inst.cut)
            out["err_rel_l1_fp32"] = metrics.rel_l1(s32, ref)
            out["err_rel_l1_bf16x6"] = metrics.rel_l1(sbf, ref)
            out["fp64_plain"]["err_rel_l1"] = metrics.rel_l1(s64, native.reconstruct(inst.entries, inst.cut))
            reps, t0 = 0, time.perf_counter()
            while True:
                native.reconstruct(e64_np, inst.cut)
                reps += 1
                el = time.perf_counter() - t0
                if el >= args.cpu_seconds or reps >= 100000:
                    break
            out["kappa"] = metrics.kappa(e64_np, inst.cut, float(np.abs(ref).sum()))
            t1 = time.perf_counter()
            native.reconstruct(e64_np, inst.cut, threads=1)
            one = N / (time.perf_counter() - t1)
            out["cpu_baseline"] = {"value": reps * N / el, "unit": "probs/s", "cores": threads, "kind": "oracle",
                                   "sample": f"full 2^{n} vector x {reps} repetitions ({el:.1f} s), C/OpenMP "
                                             f"FP64 per-output definition",
                                   "one_thread_value": one, "cpu_model": _cpu_model()}
        else:
            xs, g32 = s32
            ref = native.reconstruct(e64_np, inst.cut, xs)
            out["err_rel_l1_fp32_sampled"] = metrics.rel_l1(g32, ref)
            out["err_rel_l1_bf16x6_sampled"] = metrics.rel_l1(sbf[1], ref)
            if s3 is not None:
                out["err_rel_l1_bf16x3_sampled"] = metrics.rel_l1(s3[1], ref)
            out["fp64_plain"]["err_rel_l1_sampled"] = metrics.rel_l1(
                s64[1], native.reconstruct(inst.entries, inst.cut, xs))
            rng = np.random.default_rng(11)
            rate, size, reps, el = _cpu_rate(
                lambda m: native.reconstruct(e64_np, inst.cut, np.sort(rng.integers(0, N, m))),
                N, args.cpu_seconds, 4096)
            T = native.reconstruct([np.abs(E) for E in e64_np], inst.cut, xs)
            out["kappa_sampled"] = float(T.sum() / np.abs(ref).sum())
            xs1 = np.sort(rng.integers(0, N, 4096))
            t1 = time.perf_counter()
            native.reconstruct(e64_np, inst.cut, xs1, threads=1)
            one = xs1.size / (time.perf_counter() - t1)
            out["cpu_baseline"] = {"value": rate, "unit": "probs/s", "cores": threads, "kind": "oracle",
                                   "sample": f"{size} seeded random outputs x {reps} repetitions ({el:.1f} s), "
                                             f"C/OpenMP FP64 per-output definition (4096 terms each)",
                                   "one_thread_value": one, "cpu_model": _cpu_model()}
    return out


# ---------------------------------------------------------------------------
def bench_dd(args, torch, cqc, W):
    """c4: dynamic definition, 5 recursions of 2^20 bins on an n=40 instance."""
    inst = W.config_instance("c4")
    cut = cqc.CutMap.from_workload(inst.cut)
    a, R = W.DD_C4["n_active"], W.DD_C4["n_recursions"]
    e32_np = [E.astype(np.float32) for E in inst.entries]
    e32 = [torch.from_numpy(E).cuda() for E in e32_np]
    steps = args.steps or 10
    warmup = args.warmup if args.warmup is not None else 2
    holder = {}

    # the device-resident query (every pick on the device, no host round
    # trip), captured once in a graph and replayed: the timed step
    q = cqc.DDQuery(e32, cut, a, R, precision="fp32")
    q.run()
    torch.cuda.synchronize()
    gs = torch.cuda.Stream()
    gs.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(gs):
        q.run()
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=gs):
            q.run()
    torch.cuda.synchronize()
    ms = _sync_time(lambda i: graph.replay(), steps, warmup, torch)
    kt = _traced(lambda i: q.run(), steps, cqc, torch)
    ms_eager = _sync_time(lambda i: q.run(), steps, warmup, torch)
    bins, recs = q.result()

    # the host-driven query (a read-back and host pick per recursion)
    def step(i):
        holder["r"] = cqc.reconstruct_dd(e32, cut, a, R, precision="fp32")
    ms_host = _sync_time(step, steps, warmup, torch)
    bins_h, recs_h = holder["r"]
    same_host = ([r["parent"] for r in recs_h] == [r["parent"] for r in recs] and
                 [r["mass"] for r in recs_h] == [r["mass"] for r in recs] and bool(torch.equal(bins_h, bins)))

    # the same search with four bins per host round trip: the four refinements
    # of the first recursion have no merged qubits, so they are the same four
    # picks, enqueued together behind one read-back
    def step4(i):
        holder["r4"] = cqc.reconstruct_dd(e32, cut, a, R, precision="fp32", bins_per_round=4)
    ms4 = _sync_time(step4, steps, warmup, torch)
    bins4, recs4 = holder["r4"]
    same4 = [r["parent"] for r in recs4] == [r["parent"] for r in recs] and bool(torch.equal(bins4, bins))
    nrec = len(recs)
    per_call = {k: (v[0] / steps, v[1] / steps) for k, v in kt.items()}
    name, (cnt, tot) = max(per_call.items(), key=lambda kv: kv[1][1])
    avg = tot / cnt
    # the dominant kernel's algorithmic bytes: the last contraction writes the
    # 2^a FP64 bins and reads both merged operands once
    alg = 8 * 2 ** a
    roof = _roof("hbm", alg / (avg * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s", name, avg, None)
    roof["note"] = "latency-bound: about 2 us of roofline work per recursion"
    bins_total = nrec * 2 ** a
    out = _line("c4", "DD reconstructed bins/s n=40,K=8 (2^20 bins x 5 recursions, FP32 term sum, FP64 bins)",
                bins_total / (ms * 1e-3), "bins/s", steps, warmup, ms, "f32",
                {"n": inst.n, "K": inst.K, "n_active": a, "recursions": nrec, "precision": "fp32",
                 "seed": W.RECIPES["c4"]["seed"], "query": "device-resident, graph replay"},
                roof, us_per_recursion=1e3 * ms / nrec, kernels_ms_per_call=per_call,
                device_query_eager={"ms_per_step": ms_eager},
                host_driven_query={"ms_per_step": ms_host, "same_records_and_bins": same_host},
                four_bins_per_round={"ms_per_step": ms4, "same_records": same4},
                records=[{"parent": r["parent"], "mass": r["mass"]} for r in recs])
    if not args.no_cpu:
        from oracle import dd, native  # CPU-baseline leg only
        threads = native.max_threads()
        e64_np = [E.astype(np.float64) for E in e32_np]
        role = [dd.ACTIVE if q < a else dd.MERGED for q in range(inst.n)]
        t0 = time.perf_counter()
        merged = native.dd_merge(e64_np, inst.cut, role, threads)
        t_merge = time.perf_counter() - t0
        g = bins[0].cpu().numpy()
        rng = np.random.default_rng(12)
        probe = np.sort(rng.choice(2 ** a, 256, replace=False))
        ref = native.dd_bins(merged, inst.cut, role, probe, threads)
        out["err_rel_l1_recursion1_sampled"] = float(np.abs(g[probe] - ref).sum() / np.abs(ref).sum())
        rate, size, reps, el = _cpu_rate(
            lambda m: native.dd_bins(merged, inst.cut, role, np.sort(rng.choice(2 ** a, m, replace=False)), threads),
            2 ** a, args.cpu_seconds, 1024)
        full = 2 ** a / (t_merge + 2 ** a / rate)
        out["cpu_baseline"] = {"value": full, "unit": "bins/s", "cores": threads, "kind": "oracle",
                               "cpu_model": _cpu_model(),
                               "sample": f"recursion 1 by the C/OpenMP twin: merge ({t_merge:.3f} s) plus {size} "
                                         f"seeded bins x {reps} repetitions ({el:.1f} s) of the per-bin FP64 "
                                         f"definition over 4^8 terms, scaled to 2^{a} bins; "
                                         f"rate = 2^{a} / (merge + scaled bin time)"}
    return out


# ---------------------------------------------------------------------------
def bench_entries(args, torch, cqc, W):
    """entries: on-device entry construction (Eq. 3 attribution and the
    initialisation combination) for the upstream and downstream subcircuits of
    a two-cut pair, 2^22 output columns each, FP32 variants and entries."""
    f = 22
    gen = torch.Generator(device="cuda")
    gen.manual_seed(6)

    def variants_of(k_in, k_out):
        V = torch.empty((4 ** k_in, 3 ** k_out, 2 ** f, 2 ** k_out), dtype=torch.float32, device="cuda")
        V.exponential_(generator=gen)
        V /= V.sum(dim=(2, 3), keepdim=True)
        return V
    jobs = [(variants_of(0, 2), [1, 1]), (variants_of(2, 0), [0, 0])]
    outs = cqc.build_entries(jobs)
    steps = args.steps or 20
    warmup = args.warmup if args.warmup is not None else 3

    def step(i):
        cqc.build_entries(jobs, outs=outs)
    ms = _sync_time(step, steps, warmup, torch)
    kt = _traced(step, steps, cqc, torch)
    cnt, tot = kt["build_entries"]
    in_bytes = sum(V.numel() * 4 for V, _ in jobs)
    out_elems = sum(E.numel() for E in outs)
    # algorithmic bytes of a step: every variant value read once, every entry written once
    roof = _roof("hbm", (in_bytes + 4 * out_elems) / (tot / steps * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s",
                 "build_entries", tot / cnt, None)
    roof["bytes_per_step"] = in_bytes + 4 * out_elems
    roof["launches_per_step"] = cnt / steps
    out = _line("entries", "entry-tensor elements built per second from variant distributions (FP32)",
                out_elems / (ms * 1e-3), "entries/s", steps, warmup, ms, "f32",
                {"f": f, "cuts": 2, "variants_bytes": in_bytes}, roof, kernels_ms=kt)
    if not args.no_cpu:
        from oracle import variants  # CPU-baseline leg only
        xs = np.sort(np.random.default_rng(9).choice(2 ** f, 4096, replace=False))
        samples = [(V[:, :, torch.from_numpy(xs).cuda(), :].double().cpu().numpy(), k) for V, k in jobs]
        for (Vs, k), E in zip(samples, outs):
            ref = variants.entries_from_variants(Vs, k)
            got = E[:, torch.from_numpy(xs).cuda()].double().cpu().numpy()
            out.setdefault("err_max_abs_sampled", 0.0)
            out["err_max_abs_sampled"] = max(out["err_max_abs_sampled"], float(np.max(np.abs(got - ref))))
        per = sum(4 ** len(k) * len(xs) for _, k in samples)
        t0, reps = time.perf_counter(), 0
        while time.perf_counter() - t0 < args.cpu_seconds:
            for Vs, k in samples:
                variants.entries_from_variants(Vs, k)
            reps += 1
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": per * reps / el, "unit": "entries/s", "cores": 1, "kind": "oracle",
                               "sample": f"4096 seeded output columns of both jobs x {reps} repetitions "
                                         f"({el:.1f} s), numpy FP64 per-label definition"}
    return out


# ---------------------------------------------------------------------------
def bench_dd_scale(args, torch, cqc, W):
    """dd35: one DD recursion of 2^35 FP32 bins (128 GiB) on a 100-qubit cut."""
    wcut, ents = W.dd_scale_instance()
    a = W.DD_SCALE["n_active"]
    cut = cqc.CutMap.from_workload(wcut)
    dev = [torch.from_numpy(E).cuda() for E in ents]
    steps = args.steps or 5
    warmup = args.warmup if args.warmup is not None else 1
    holder = {}

    def step(i):
        holder.pop("r", None)          # one 128 GiB bins buffer at a time
        holder["r"] = cqc.reconstruct_dd(dev, cut, a, 1, precision="fp32", bins_dtype=torch.float32)
    ms = _sync_time(step, steps, warmup, torch)
    kt = _traced(step, steps, cqc, torch)
    bins, recs = holder["r"]
    per_call = {k: (v[0] / steps, v[1] / steps) for k, v in kt.items()}
    name, (cnt, tot) = max(per_call.items(), key=lambda kv: kv[1][1])
    avg = tot / cnt
    # the final contraction writes the 2^35 FP32 bins once and reads its two
    # operands (16 x 2^20 and 16 x 2^15 FP32)
    alg = 4 * 2 ** a + 4 * 16 * (2 ** 20 + 2 ** 15)
    roof = _roof("hbm", alg / (avg * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s", name, avg, None)
    out = _line("dd35", "DD reconstructed bins/s, n=100 K=8, one recursion of 2^35 bins (FP32 term sum and bins)",
                2 ** a / (ms * 1e-3), "bins/s", steps, warmup, ms, "f32",
                {"n": wcut.n, "K": wcut.n_cuts, "n_active": a, "recursions": 1, "precision": "fp32",
                 "bins": "fp32", "seed": W.DD_SCALE["seed"]},
                roof, kernels_ms_per_call=per_call, mass=recs[0]["mass"])
    if not args.no_cpu:
        from oracle import native  # CPU-baseline leg only
        threads = native.max_threads()
        role = recs[0]["role"]
        rng = np.random.default_rng(13)
        probe = np.sort(rng.choice(2 ** a, 64, replace=False))
        got = bins[0, torch.from_numpy(probe).cuda()].double().cpu().numpy()
        del holder["r"], bins
        torch.cuda.empty_cache()
        e64_np = [E.astype(np.float64) for E in ents]
        t0 = time.perf_counter()
        merged = native.dd_merge(e64_np, wcut, role, threads)
        t_merge = time.perf_counter() - t0
        del e64_np
        ref = native.dd_bins(merged, wcut, role, probe, threads)
        out["err_rel_l1_sampled"] = float(np.abs(got - ref).sum() / np.abs(ref).sum())
        rate, size, reps, el = _cpu_rate(
            lambda m: native.dd_bins(merged, wcut, role, np.sort(rng.choice(2 ** a, m, replace=False)), threads),
            2 ** a, args.cpu_seconds, 1024)
        full = 2 ** a / (t_merge + 2 ** a / rate)
        out["cpu_baseline"] = {"value": full, "unit": "bins/s", "cores": threads, "kind": "oracle",
                               "cpu_model": _cpu_model(),
                               "sample": f"the C/OpenMP twin: merge ({t_merge:.1f} s) plus {size} seeded bins x "
                                         f"{reps} repetitions ({el:.1f} s) of the per-bin FP64 definition over "
                                         f"4^8 terms, scaled to 2^{a} bins; rate = 2^{a} / (merge + scaled bin time)"}
    return out


# ---------------------------------------------------------------------------
def bench_chi2(args, torch, cqc, W):
    """chi2: Eq. 16 over two 2^28-outcome FP32 distributions (2 GiB read)."""
    n = 1 << 28
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    a = torch.empty(n, dtype=torch.float32, device="cuda").exponential_(generator=gen)
    b = torch.empty(n, dtype=torch.float32, device="cuda").exponential_(generator=gen)
    a /= a.sum()
    b /= b.sum()
    steps = args.steps or 20
    warmup = args.warmup if args.warmup is not None else 3
    ms = _sync_time(lambda i: cqc.chi2(a, b), steps, warmup, torch)
    kt = _traced(lambda i: cqc.chi2(a, b), steps, cqc, torch)
    cnt, tot = kt["chi2_part"]
    roof = _roof("hbm", 8.0 * n / (tot / cnt * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s", "chi2_part", tot / cnt, None)
    out = _line("chi2", "chi-square distance outcomes/s (Eq. 16, FP32 inputs, FP64 terms)", n / (ms * 1e-3),
                "outcomes/s", steps, warmup, ms, "f32", {"n": n}, roof, kernels_ms=kt)
    if not args.no_cpu:
        from oracle import native  # CPU-baseline leg only
        threads = native.max_threads()
        m = 1 << 26
        an, bn = a[:m].double().cpu().numpy(), b[:m].double().cpu().numpy()
        t0, reps = time.perf_counter(), 0
        while time.perf_counter() - t0 < args.cpu_seconds / 2:
            native.chi2(an, bn, threads)
            reps += 1
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": m * reps / el, "unit": "outcomes/s", "cores": threads, "kind": "oracle",
                               "cpu_model": _cpu_model(),
                               "sample": f"first 2^26 outcomes x {reps} repetitions ({el:.1f} s), "
                                         f"C/OpenMP FP64 twin of Eq. 16"}
    return out


# ---------------------------------------------------------------------------
def bench_batch(args, torch, cqc, W):
    """c5: 256 instances, forward + cross-entropy gradient + adjoint, one graph."""
    insts = W.batch_instances(256)
    cuts = [cqc.CutMap.from_workload(i.cut) for i in insts]
    e32_np = [[E.astype(np.float32) for E in i.entries] for i in insts]
    ents = [[torch.from_numpy(E).cuda() for E in e] for e in e32_np]
    # every instance's p, target and dL/dp are slices of one flat buffer, so
    # the cross-entropy gradient (dL/dp = -t/p where p > 1e-30, else 0) of all
    # instances is one fused library pass
    sizes = [2 ** i.n for i in insts]
    total = sum(sizes)
    p_flat = torch.empty(total, dtype=torch.float32, device="cuda")
    g_flat = torch.empty(total, dtype=torch.float32, device="cuda")
    t_flat = torch.from_numpy(np.concatenate(
        [W.dirichlet_target(i.n, 1000 + k).astype(np.float32) for k, i in enumerate(insts)])).cuda()
    outs = list(torch.split(p_flat, sizes))
    grads_out = list(torch.split(g_flat, sizes))
    batch = cqc.Batch(ents, cuts, precision="fp32", outs=outs)
    bwd = cqc.BatchBackward(batch, grads_out)

    def body():
        batch.run()
        cqc.xent_grad(p_flat, t_flat, grad=g_flat)
        bwd.run()
    steps = args.steps or 20
    warmup = args.warmup if args.warmup is not None else 3

    def graphed(fn):
        fn()
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            fn()
            torch.cuda.synchronize()
            with torch.cuda.graph(graph, stream=s):
                fn()
        torch.cuda.synchronize()
        return graph

    graph2 = graphed(body)
    ms2 = _sync_time(lambda i: graph2.replay(), steps, warmup, torch)
    kt2 = _traced(lambda i: body(), 3, cqc, torch)
    del graph2
    # the same step with the cross-entropy gradient computed inside the
    # kernels that produce p (cqc_batch_create_xent): p itself is not kept
    t_split = list(torch.split(t_flat, sizes))
    xb = cqc.Batch(ents, cuts, precision="fp32", targets=t_split, grads=grads_out, keep_outputs=False,
                   with_mass=False)
    xbwd = cqc.BatchBackward(xb, grads_out)

    def fused():
        xb.run()
        xbwd.run()
    graph = graphed(fused)
    ms = _sync_time(lambda i: graph.replay(), steps, warmup, torch)
    kt = _traced(lambda i: fused(), 3, cqc, torch)
    # identical gradients to the two-pass step
    body()
    torch.cuda.synchronize()
    g_two = [[g.clone() for g in gl] for gl in bwd.grads]
    graph.replay()
    torch.cuda.synchronize()
    same = all(torch.equal(a, b) for ga, gb in zip(g_two, xbwd.grads) for a, b in zip(ga, gb))
    del graph
    xl = cqc.Batch(ents, cuts, precision="fp32", targets=t_split, grads=grads_out, keep_outputs=False,
                   with_loss=True)
    xlb = cqc.BatchBackward(xl, grads_out)

    def fused_loss():
        xl.run()
        xlb.run()
    graph_l = graphed(fused_loss)
    ms_l = _sync_time(lambda i: graph_l.replay(), steps, warmup, torch)
    del graph_l
    outputs = sum(2 ** i.n for i in insts)
    # roofline of the step: per instance the larger of its HBM time (read t,
    # write G, read G in the adjoint: 12 bytes per output, p never leaving the
    # chip) and its FP32 matrix-core time (forward and both adjoint sides)
    roof_s = 0.0
    for c, i in zip(cuts, insts):
        _, macs = cqc.cost(c)
        byts = 4.0 * 2 ** i.n * 3
        roof_s += max(byts / (HBM_PEAK_GBS * 1e9), 3 * 2 * macs / (FP32_PEAK_TFS * 1e12))
    name, (cnt, tot) = max(kt.items(), key=lambda kv: kv[1][1])
    roof = {"bound": "mixed", "achieved": roof_s * 1e3, "peak": ms, "unit": "ms per step (roofline vs measured)",
            "frac": roof_s * 1e3 / ms, "traffic": None, "dominant_kernel": name,
            "dominant_kernel_ms_per_step": tot / 3,
            "note": "per instance max(12 bytes per output / 8 TB/s, 3 x forward flops / 157.3 TF)"}
    out = _line("c5", "batched FD forward + adjoint outputs/s (256 instances, n 12..24, K 1..4, graph replay)",
                outputs / (ms * 1e-3), "probs/s", steps, warmup, ms, "f32",
                {"instances": len(insts), "sum_2^n": outputs, "precision": "fp32", "seed": 5,
                 "step": "forward with the cross-entropy gradient in its final kernels, then the adjoint"},
                roof, kernels_ms_per_step={k: v[1] / 3 for k, v in kt.items()})
    out["two_pass"] = {"ms_per_step": ms2, "value": outputs / (ms2 * 1e-3),
                       "step": "forward writing p, one cross-entropy gradient pass, adjoint",
                       "kernels_ms_per_step": {k: v[1] / 3 for k, v in kt2.items()},
                       "same_entry_gradients_as_fused": same}
    out["fused_with_loss"] = {"ms_per_step": ms_l, "value": outputs / (ms_l * 1e-3)}
    if not args.no_cpu:
        from oracle import native, metrics  # CPU-baseline leg only
        threads = native.max_threads()
        order = sorted(range(len(insts)), key=lambda k: insts[k].n)
        small = [k for k in order if insts[k].n <= 18][:64]
        errs = []
        for k in small[:8]:
            ref = native.reconstruct([E.astype(np.float64) for E in e32_np[k]], insts[k].cut)
            errs.append(metrics.rel_l1(batch.outs[k].double().cpu().numpy(), ref))
        out["err_rel_l1_fp32_max_of_8"] = max(errs)
        tot_out, reps, t0 = 0, 0, time.perf_counter()
        while True:
            for k in small:
                native.reconstruct([E.astype(np.float64) for E in e32_np[k]], insts[k].cut)
                tot_out += 2 ** insts[k].n
            reps += 1
            el = time.perf_counter() - t0
            if el >= args.cpu_seconds or reps >= 100000:
                break
        out["cpu_baseline"] = {"value": tot_out / el, "unit": "probs/s", "cores": threads, "kind": "oracle",
                               "sample": f"forward only: {len(small)} instances with n <= 18 x {reps} repetitions "
                                         f"({el:.1f} s), C/OpenMP FP64 per-output definition"}
    return out


def main():
    args = _args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the FD output space shards across GPUs with no "
              "exchange, so N>1 is not measured by this build", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2012_02333_amd as cqc
    import workloads as W

    if not torch.cuda.is_available():
        print("no GPU", file=sys.stderr)
        sys.exit(1)
    if args.calibrate:
        # reference kernels of known traffic for the HBM counters: a 256 MiB
        # fill (writes 256 MiB) and a 256 MiB elementwise add (reads 256 MiB,
        # writes 256 MiB), each on buffers not touched just before
        a = torch.empty(1 << 26, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        c = torch.empty_like(a)
        a.fill_(1.0)
        c.fill_(0.0)
        torch.cuda.synchronize()
        for _ in range(3):
            torch.add(a, 1.0, out=b)
            torch.add(c, 1.0, out=a)
            torch.add(b, 1.0, out=c)
        torch.cuda.synchronize()
        del a, b, c
    if args.config in ("c2", "c3"):
        out = bench_fd(args, args.config, torch, cqc, W)
    elif args.config == "c4":
        out = bench_dd(args, torch, cqc, W)
    elif args.config == "entries":
        out = bench_entries(args, torch, cqc, W)
    elif args.config == "chi2":
        out = bench_chi2(args, torch, cqc, W)
    elif args.config == "dd35":
        out = bench_dd_scale(args, torch, cqc, W)
    else:
        out = bench_batch(args, torch, cqc, W)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
