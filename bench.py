"""Throughput benchmark of the FD reconstruction hot path on one MI355X.

Default workload: n=24 seeded random U3+CZ circuit (depth 8) cut by K=2 wires
into two 13-qubit subcircuits; entry tensors 16 x 2^11 and 16 x 2^13 from
noiseless simulation; 2^24 output probabilities.  A step is one complete
library call: entry row flags (early termination), the term sum on matrix
cores, the single write of every output and the FP64 total mass.  The FP32
form (metric) and the plain FP64 form run on the same inputs; output buffers
rotate over >= 1 GiB so the 256 MB last-level cache cannot hold the writes.

Prints ONE JSON line.  `--config c3|c4|c5` measures the other workloads
(extra lines, not the headline).
"""
from __future__ import annotations

import argparse
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


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="c2", choices=["c2", "c3"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--calibrate", action="store_true",
                    help="first run a plain 256 MiB device copy 10 times (reference for HBM counters)")
    return ap.parse_args()


TRAFFIC_KERNEL_SOURCES = ["paper_2012_02333_amd/csrc/k_contract.hip", "paper_2012_02333_amd/csrc/kernels.hpp"]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_KERNEL_SOURCES:
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
    if rec.get("source_sha") != kernel_source_hash() or rec.get("kernel") != kernel:
        return None
    return rec.get("hbm_bytes_per_launch")


def _time_steps(call, outs, steps, warmup, torch):
    """Warm up, then time exactly `steps` calls, rotating output buffers."""
    nb = len(outs)
    for i in range(warmup):
        call.set_outputs([outs[i % nb]])
        call.run()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for i in range(steps):
        call.set_outputs([outs[i % nb]])
        call.run()
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def _kernel_time(call, outs, steps, cqc, torch):
    """Per-kernel average duration from HIP events bracketing every launch."""
    nb = len(outs)
    with cqc.trace() as tr:
        for i in range(steps):
            call.set_outputs([outs[i % nb]])
            call.run()
        torch.cuda.synchronize()
    return tr.result


def _cpu_baseline(inst, e64, seconds):
    """The oracle's C twin (plain per-output FP64 definition) on the host cores."""
    from oracle import native, metrics  # noqa: F401  (CPU-baseline leg only)
    n = inst.n
    threads = native.max_threads()
    p = native.reconstruct(e64, inst.cut)          # full vector once (also the parity reference)
    reps, t0 = 0, time.perf_counter()
    while True:
        native.reconstruct(e64, inst.cut)
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds or reps >= 50:
            break
    rate = reps * (2 ** n) / el
    return p, {"value": rate, "unit": "probs/s", "cores": threads, "kind": "oracle",
               "sample": f"full 2^{n} vector x {reps} repetitions ({el:.1f} s), C/OpenMP FP64 "
                         f"per-output definition"}


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
    inst = W.config_instance(args.config)
    n, K = inst.n, inst.K
    cut = cqc.CutMap.from_workload(inst.cut)
    e32_np = [E.astype(np.float32) for E in inst.entries]
    e32 = [torch.from_numpy(E).cuda() for E in e32_np]
    e64 = [torch.from_numpy(E).cuda() for E in inst.entries]
    N = 2 ** n

    nbuf32 = max(2, min(16, (1 << 30) // (4 * N)))
    outs32 = [torch.empty(N, dtype=torch.float32, device="cuda") for _ in range(nbuf32)]
    call32 = cqc.FDCall(e32, cut, precision="fp32", outs=[outs32[0]])
    ms32 = _time_steps(call32, outs32, args.steps, args.warmup, torch)
    kt32 = _kernel_time(call32, outs32, args.steps, cqc, torch)
    p32 = outs32[(args.steps - 1) % nbuf32].double().cpu().numpy() if n <= 26 else None
    mass32 = float(call32.mass[0].cpu())
    del outs32, call32
    torch.cuda.empty_cache()

    fp64 = None
    if args.config == "c2":
        nbuf64 = max(2, min(16, (1 << 30) // (8 * N)))
        outs64 = [torch.empty(N, dtype=torch.float64, device="cuda") for _ in range(nbuf64)]
        call64 = cqc.FDCall(e64, cut, precision="fp64", outs=[outs64[0]])
        ms64 = _time_steps(call64, outs64, args.steps, args.warmup, torch)
        kt64 = _kernel_time(call64, outs64, args.steps, cqc, torch)
        p64 = outs64[(args.steps - 1) % nbuf64].cpu().numpy()
        fp64 = {"value": N / (ms64 * 1e-3), "ms_per_step": ms64, "kernels_ms": kt64}
        del outs64, call64

    # dominant kernel: the last contraction (writes every output once)
    name, (cnt, tot) = max(kt32.items(), key=lambda kv: kv[1][1])
    avg_ms = tot / cnt
    in_bytes = sum(E.numel() * 4 for E in e32)
    if args.config == "c2":
        alg_bytes = 4 * N + in_bytes
        roof = {"bound": "hbm", "achieved": alg_bytes / (avg_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s"}
    else:
        _, macs = cqc.cost(cut)
        roof = {"bound": "mfma", "achieved": 2 * macs / (avg_ms * 1e-3) / 1e12, "peak": FP32_PEAK_TFS,
                "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    tr = recorded_traffic(args.config, name)
    roof["traffic"] = tr
    roof["kernel"] = name
    roof["kernel_avg_us"] = avg_ms * 1e3

    out = {
        "metric": METRIC if args.config == "c2" else f"FD reconstructed probs/s ({args.config})",
        "value": N / (ms32 * 1e-3),
        "unit": "probs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": {"c2": "FD n=24 K=2, two 13-qubit subcircuits, E 16x2^11 and 16x2^13",
                                "c3": "FD n=30 K=6, three 12-qubit subcircuits, 4096 terms"}[args.config],
                   "n": n, "K": K, "precision": "fp32", "seed": W.RECIPES[args.config]["seed"],
                   "output_buffers_rotated": nbuf32},
        "roofline": roof,
        "mass": mass32,
        "kernels_ms": kt32,
    }
    if fp64:
        out["fp64_plain"] = fp64
        out["speedup_fp32_vs_fp64"] = out["value"] / fp64["value"]
    if not args.no_cpu and n <= 26:
        ref, cpu = _cpu_baseline(inst, [E.astype(np.float64) for E in e32_np], args.cpu_seconds)
        from oracle import metrics
        out["cpu_baseline"] = cpu
        out["err_rel_l1_fp32"] = metrics.rel_l1(p32, ref)
        if fp64:
            from oracle import native
            ref64 = native.reconstruct(inst.entries, inst.cut)
            out["fp64_plain"]["err_rel_l1"] = metrics.rel_l1(p64, ref64)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
