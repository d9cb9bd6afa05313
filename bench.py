#!/usr/bin/env python3
"""Benchmark of the batched trust-region Newton solve on one MI355X.

Default workload: 65,536 branch subproblems of the component ADMM (BR6, n = 6, FP64,
warm-started at their nominal operating point), solved to an absolute projected-gradient
tolerance of 1e-6 in one launch. A step is one full solve of the batch (every instance from
its x0 with the cold radius rule), with inputs resident in HBM.

Prints one JSON line: solves/s, per-launch p50/p99 latency, the roofline of the solve
kernel (algorithmic FP64 flops from the oracle's counters / measured kernel time, against
the 78.6 TFLOP/s FP64 vector peak) and the CPU oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_VECTOR = 78.6e12   # MI355X FP64 vector, FLOP/s
PEAK_HBM = 8.0e12            # MI355X HBM3E, B/s
BR6_BYTES = 36 * 8 + 3 * 6 * 8 + 6 * 8 + 8 + 4 + 4   # params, lo/hi/x0 in; x, f, status, iters out


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(kernel):
    """HBM bytes per launch from the committed counter summary (profiles/traffic.json), or
    None when the kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(kernel)
    if not rec:
        return None
    h = hashlib.sha256()
    for src in rec["kernel_sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return rec["hbm_bytes_per_launch"] if h.hexdigest() == rec["source_sha256"] else None


def cpu_baseline(bt, budget_s):
    """The oracle (as it stands) on all host cores over the same batch, repeated until about
    `budget_s` seconds of CPU work; also returns its algorithmic flop count per instance."""
    import oracle
    oracle.lib()
    t0 = time.perf_counter()
    r = oracle.solve(bt, nthreads=0)
    t1 = time.perf_counter()
    threads = int(r["threads"])
    flops = r["stats"][:, 0].astype(np.float64)
    reps, wall = 1, t1 - t0
    while wall * threads < budget_s and reps < 200:
        t0 = time.perf_counter()
        oracle.solve(bt, nthreads=0, with_stats=False)
        wall += time.perf_counter() - t0
        reps += 1
    return dict(value=bt.batch * reps / wall, threads=threads, reps=reps, wall=wall,
                flops_per_instance=float(flops.mean()), status=r["status"])


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="CPU work budget of the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", default="br6", choices=["br6", "copy"],
                    help="copy: a plain device-to-device copy of known size, used to scale the "
                         "FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the instances are independent; see the sharding notes in DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2106_14995_amd import tron
    from paper_2106_14995_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.mode == "copy":
        nbytes = 256 << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_read_per_copy": nbytes,
                          "bytes_written_per_copy": nbytes, "copies": args.steps}), flush=True)
        return
    log(f"generating {args.batch} BR6 instances")
    bt = W.br6_batch(args.batch, config_id=1)
    params, lo, hi, x0 = tron.to_device(bt)
    h = tron.Batch(W.BR6, 6, batch=args.batch)
    B = args.batch
    x = torch.empty(6 * B, dtype=torch.float64, device="cuda")
    f = torch.empty(B, dtype=torch.float64, device="cuda")
    st = torch.empty(B, dtype=torch.int32, device="cuda")
    it = torch.empty(B, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    log("warmup")
    for _ in range(args.warmup):
        h.solve(params, lo, hi, x0, x, f, st, it, stream=stream)
    torch.cuda.synchronize()
    n_conv = int((st == 0).sum().item())
    log(f"converged {n_conv}/{B}; iters p50 {int(it.median().item())} max {int(it.max().item())}")

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        h.solve(params, lo, hi, x0, x, f, st, it, stream=stream)
        ends[k].record(stream)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    lat = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])  # ms per launch
    log(f"timed {args.steps} steps in {total:.3f} s; launch ms p50 {np.median(lat):.4f}")

    result = {
        "metric": "TRON subproblem solves/sec at 1e-6 proj-grad tol; p50/p99 solve latency",
        "value": B * args.steps / total,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "BR6 branch-subproblem batch (ADMM), 65,536 x n=6, warm start, gtol 1e-6",
                   "batch": B, "n": 6, "family": "br6", "converged": n_conv},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cb = cpu_baseline(bt, args.cpu_seconds)
        kern_s = float(lat.mean()) * 1e-3
        flops = cb["flops_per_instance"] * B
        bytes_ = BR6_BYTES * B
        t_flop, t_byte = flops / PEAK_FP64_VECTOR, bytes_ / PEAK_HBM
        if t_flop >= t_byte:
            roof = {"bound": "alu", "achieved": flops / kern_s / 1e12, "peak": PEAK_FP64_VECTOR / 1e12,
                    "unit": "TFLOP/s"}
        else:
            roof = {"bound": "hbm", "achieved": bytes_ / kern_s / 1e9, "peak": PEAK_HBM / 1e9,
                    "unit": "GB/s"}
        roof["frac"] = roof["achieved"] / roof["peak"]
        traffic = measured_traffic("lane_kernel<mt::BR6, 6>")
        roof["traffic"] = traffic
        if traffic is not None:
            roof["traffic_unit"] = "bytes per launch (FETCH_SIZE x2.000 + WRITE_SIZE x1.000)"
            roof["traffic_over_algorithmic"] = traffic / bytes_
        roof["flops_per_instance"] = cb["flops_per_instance"]
        roof["bytes_per_instance"] = BR6_BYTES
        roof["hbm_gbs_algorithmic"] = bytes_ / kern_s / 1e9
        result["roofline"] = roof
        result["cpu_baseline"] = {
            "value": cb["value"], "unit": "solves/s", "cores": cb["threads"], "kind": "oracle",
            "sample": f"the same {B}-instance batch, {cb['reps']} passes, {cb['wall']:.2f} s wall",
        }
    print(json.dumps(result), flush=True)
    h.close()


if __name__ == "__main__":
    main()
