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


def measured_peaks(stream):
    """Achievable rates on this device, the measured references beside the published peaks:
    FP64 from the library's FMA-chain kernel (8 waves per SIMD, 8 independent chains per lane),
    HBM from a 512 MiB device-to-device copy (bytes read plus bytes written). Each is the best
    of five timed launches after one warm-up."""
    import torch
    from paper_2106_14995_amd import tron
    blocks, iters = 256 * 8, 20000
    sink = torch.empty(blocks * 256, dtype=torch.float64, device="cuda")
    flops = blocks * 256 * 8 * iters * 2.0
    src = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    nbytes = 2.0 * src.numel() * 8

    def best(fn, work):
        fn()
        torch.cuda.synchronize()
        rates = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            rates.append(work / (e0.elapsed_time(e1) * 1e-3))
        return max(rates)

    fp64 = best(lambda: tron.design_fma_peak(blocks, iters, sink, stream=stream), flops)
    hbm = best(lambda: dst.copy_(src), nbytes)
    return {"fp64_tflops": fp64 / 1e12, "hbm_gbs": hbm / 1e9,
            "fp64_kernel": f"FMA chains, {blocks} x 256 lanes x 8 chains x {iters}",
            "hbm_kernel": "device-to-device copy of 512 MiB"}


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


def time_solves(solve, steps, warmup, stream):
    """Run `solve()` warmup times, then `steps` times back to back for the wall time (s), then
    `steps` more times, each between its own pair of HIP events, for per-step latencies (ms);
    the event packets add a few microseconds between steps, so they stay out of the wall time."""
    import torch
    for _ in range(warmup):
        solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        solve()
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    for k in range(steps):
        starts[k].record(stream)
        solve()
        ends[k].record(stream)
    torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) for a, b in zip(starts, ends)]), total


def bench_qp4(args):
    """256 quartic problems, n = 8: the oracle's CPU seconds (1 thread and all threads) and the
    GPU's time for the same batch."""
    import torch
    import oracle
    from paper_2106_14995_amd import tron
    from paper_2106_14995_amd import workloads as W
    bt = W.qp4_batch(256, 8, config_id=0)
    cpu = {}
    for nt in (1, 0):
        best = None
        for _ in range(5):
            t0 = time.perf_counter()
            r = oracle.solve(bt, nthreads=nt, with_stats=False)
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        cpu["threads_%d" % (r["threads"])] = best
    h = tron.Batch(W.QP4, 8, batch=256)
    dev = tron.to_device(bt)
    stream = torch.cuda.current_stream()
    lat, total = time_solves(lambda: h.solve(*dev, stream=stream), args.steps, args.warmup, stream)
    print(json.dumps({"config": "qp4 256 x n=8 (quartic, strictly convex), gtol 1e-6",
                      "oracle_cpu_seconds": cpu, "gpu_ms_per_batch_p50": float(np.median(lat)),
                      "gpu_ms_per_batch_p99": float(np.percentile(lat, 99)),
                      "gpu_solves_per_s": 256 * args.steps / total}), flush=True)
    h.close()


def bench_uneven(args):
    """50,000 quartic problems with n log-uniform in [4,64]: the persistent size-bucketed
    launch (one launch for every wavefront instance, one for the lane packs) and the bucketed
    plan (a kernel per size bucket, buckets concurrent on four streams), each captured once
    in a graph and replayed, the autotuned plan, and one launch per distinct n on one stream
    (the same kernels, each sized exactly for its n). The roofline line prices the fastest
    plan's batch time against the oracle's algorithmic flop count for the batch (FP64 vector
    peak); the oracle on the host cores is timed over the same batch."""
    import torch
    import oracle
    from paper_2106_14995_amd import tron
    from paper_2106_14995_amd import workloads as W
    B = args.batch if args.batch != 65536 else 50000
    log(f"generating {B} uneven QP4 instances")
    sizes = W.loguniform_sizes(B, 4, 64, config_id=3)
    bt = W.qp4_batch(B, sizes, config_id=3)
    stream = torch.cuda.current_stream()
    dev = tron.to_device(bt)
    out = dict(x=torch.empty(bt.n.astype(np.int64).sum(), dtype=torch.float64, device="cuda"),
               f=torch.empty(B, dtype=torch.float64, device="cuda"),
               status=torch.empty(B, dtype=torch.int32, device="cuda"),
               iters=torch.empty(B, dtype=torch.int32, device="cuda"))
    res = {"config": f"qp4 uneven, {B} instances, n log-uniform in [4,64], gtol 1e-6"}
    plans = [("bucketed_streams", tron.plan_spec(pool_waves=0), False),
             ("bucketed_graph", tron.plan_spec(pool_waves=0), True),
             ("persistent_8_graph", tron.plan_spec(pool_waves=8), True),
             ("persistent_12_graph", tron.plan_spec(pool_waves=12), True)]
    if args.plan:
        plans = [p for p in plans if p[0] == args.plan]
        if not plans:
            raise SystemExit(f"unknown plan {args.plan}")
    for key, spec, graph in plans:
        h = tron.Batch(W.QP4, sizes, opts=tron.options(graph=graph), spec=spec)
        lat, total = time_solves(lambda: h.solve(*dev, **out, stream=stream), args.steps, args.warmup, stream)
        res[key] = {"solves_per_s": B * args.steps / total, "ms_per_batch": 1e3 * total / args.steps,
                    "p50_ms": float(np.median(lat)), "p99_ms": float(np.percentile(lat, 99)),
                    "launches": len(h.plan()) if spec is None else 1 + int(any(p["lanes"] == 1 for p in h.plan()))}
        res[key]["converged"] = int((out["status"] == 0).sum().item())
        log(f"{key}: {res[key]['ms_per_batch']:.3f} ms per batch")
        h.close()
    if args.plan:  # one plan only (for profiling)
        print(json.dumps(res), flush=True)
        return
    # autotuned plan (the C autotuner times candidate edge sets / streams / lane split / the
    # persistent form on this batch), then the same graph-captured timing with the chosen plan
    spec, tune_ms = tron.autotune(W.QP4, sizes, *dev, out["x"], out["f"], out["status"], out["iters"],
                                  reps=2, stream=stream)
    h = tron.Batch(W.QP4, sizes, opts=tron.options(graph=True), spec=spec)
    lat, total = time_solves(lambda: h.solve(*dev, **out, stream=stream), args.steps, args.warmup, stream)
    res["autotuned_graph"] = {"solves_per_s": B * args.steps / total, "ms_per_batch": 1e3 * total / args.steps,
                              "p50_ms": float(np.median(lat)), "p99_ms": float(np.percentile(lat, 99)),
                              "plan": spec.describe(), "tuner_best_ms": tune_ms}
    h.close()
    # one launch per distinct n, serial on one stream
    per = []
    for k in np.unique(sizes):
        idx = np.nonzero(sizes == k)[0]
        sub = bt.subset(idx)
        hk = tron.Batch(W.QP4, int(k), batch=len(idx))
        dk = tron.to_device(sub)
        per.append((hk, dk))
    lat, total = time_solves(lambda: [hk.solve(*dk, stream=stream) for hk, dk in per],
                             args.steps, args.warmup, stream)
    res["one_launch_per_size"] = {"solves_per_s": B * args.steps / total, "ms_per_batch": 1e3 * total / args.steps,
                                  "p50_ms": float(np.median(lat)), "p99_ms": float(np.percentile(lat, 99)),
                                  "launches": len(per)}
    for hk, _ in per:
        hk.close()
    if not args.no_cpu_baseline:
        log("oracle over the same batch (flop count and CPU baseline)")
        cb = cpu_baseline(bt, args.cpu_seconds)
        flops = cb["flops_per_instance"] * B
        best_key = min((k for k in res if isinstance(res[k], dict) and "ms_per_batch" in res[k]),
                       key=lambda k: res[k]["ms_per_batch"])
        t = res[best_key]["ms_per_batch"] * 1e-3
        res["roofline"] = {"bound": "alu", "achieved": flops / t / 1e12, "peak": PEAK_FP64_VECTOR / 1e12,
                           "unit": "TFLOP/s", "frac": flops / t / PEAK_FP64_VECTOR, "traffic": None,
                           "plan": best_key, "flops_per_batch": flops,
                           "note": "wave instances with n > 16 use FP64 matrix-core products in their "
                                   "factorisation; the peak is the FP64 vector one"}
        # HBM bytes of the persistent launch's wavefront kernel, from its committed counters
        # (that plan, or an autotuned plan that chose the same launch)
        tuned_pool12 = best_key == "autotuned_graph" and res[best_key].get("plan", {}).get("pool_waves") == 12
        if best_key == "persistent_12_graph" or tuned_pool12:
            kname = "pool_kernel<mt::WaveFamQP4<1>, mt::WaveFamQP4<1>, 12>"
            tr = measured_traffic(kname)
            if tr is not None:
                rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))[kname]
                res["roofline"].update({"traffic": tr, "traffic_kernel": kname,
                                        "traffic_unit": "bytes per launch (FETCH_SIZE x2.000 + WRITE_SIZE x1.000)",
                                        "traffic_over_algorithmic": tr / rec["algorithmic_bytes_per_launch"]})
        res["cpu_baseline"] = {"value": cb["value"], "unit": "solves/s", "cores": cb["threads"], "kind": "oracle",
                               "sample": f"the same {B}-instance batch, {cb['reps']} passes, {cb['wall']:.2f} s wall"}
    print(json.dumps(res), flush=True)


def bench_admm(args):
    """Component ADMM on the synthetic 2,000-bus network: time per iteration (all kernels,
    including the 3,000 branch solves) and the residuals after the run."""
    import torch
    from paper_2106_14995_amd import tron
    from paper_2106_14995_amd import workloads as W
    net = W.network()
    a = tron.Admm(net)
    iters = 1000 if args.steps == 100 else args.steps
    stream = torch.cuda.current_stream()
    resid = torch.empty(2 * iters, dtype=torch.float64, device="cuda")
    a.step(5)
    torch.cuda.synchronize()
    a.close()
    a = tron.Admm(net)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a.step(iters, resid=resid, stream=stream)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    r = resid.view(iters, 2).cpu().numpy()
    print(json.dumps({"config": "component ADMM, 2,000 buses, 3,000 branches, 500 generators, rho 400",
                      "iterations": iters, "ms_per_iteration": 1e3 * total / iters,
                      "branch_solves_per_s": net.nbranch * iters / total,
                      "primal_residual_first_last": [float(r[0, 0]), float(r[-1, 0])],
                      "dual_residual_first_last": [float(r[0, 1]), float(r[-1, 1])]}), flush=True)
    a.close()


def bench_hs45m(args):
    """The paper's kernel-design workload: 10,000 identical modified-hs45 problems
    (f = 120 - prod x_i, 0 <= x_i <= i, x0_i = i/2), one batch per step, n = 1..32. The paper's
    Table 3 reports 9.536 ms per batch on one V100 with shared memory, n unstated (context)."""
    import torch
    from paper_2106_14995_amd import tron
    from paper_2106_14995_amd import workloads as W
    stream = torch.cuda.current_stream()
    rows = []
    for n in range(1, 33):
        bt = W.hs45m_batch(10000, n)
        h = tron.Batch(W.HS45M, n, batch=10000)
        dev = tron.to_device(bt)
        lat, total = time_solves(lambda: h.solve(*dev, stream=stream), args.steps, args.warmup, stream)
        _, f, st, it = h.solve(*dev, stream=stream)
        torch.cuda.synchronize()
        rows.append({"n": n, "ms_per_batch_p50": float(np.median(lat)), "solves_per_s": 10000 * args.steps / total,
                     "converged": int((st == 0).sum().item()), "iters_max": int(it.max().item())})
        h.close()
    print(json.dumps({"config": "10,000 identical modified-hs45 problems per batch", "rows": rows,
                      "paper_context": "9.536 ms per batch, one V100, shared memory, n unstated (Table 3)"}),
          flush=True)


def bench_large(args):
    """QP4 beyond the LDS limit (n > 128): one wavefront per instance with the Hessian and its
    factor in the handle's global-memory workspace, 512 instances per size. Each batch takes
    tens to hundreds of milliseconds, so at most 3 timed steps per size."""
    import torch
    from paper_2106_14995_amd import tron
    from paper_2106_14995_amd import workloads as W
    stream = torch.cuda.current_stream()
    B = 512
    steps, warmup = min(args.steps, 3), min(args.warmup, 1)
    rows = []
    for n in (136, 200, 256, 300, 512):
        log(f"generating {B} QP4 instances, n = {n}")
        bt = W.qp4_batch(B, n, config_id=3)
        h = tron.Batch(W.QP4, n, batch=B)
        dev = tron.to_device(bt)
        lat, total = time_solves(lambda: h.solve(*dev, stream=stream), steps, warmup, stream)
        _, f, st, it = h.solve(*dev, stream=stream)
        torch.cuda.synchronize()
        rows.append({"n": n, "ms_per_batch_p50": float(np.median(lat)), "solves_per_s": B * steps / total,
                     "converged": int((st == 0).sum().item()), "iters_mean": float(it.double().mean().item())})
        log(f"n={n}: {rows[-1]['ms_per_batch_p50']:.1f} ms per batch")
        h.close()
        del dev
    print(json.dumps({"config": f"QP4, {B} instances per size, n > 128 (global-memory workspace), gtol 1e-6",
                      "rows": rows}), flush=True)


def bench_al(args):
    """Augmented-Lagrangian loop on branch subproblems with line limits (BR8L, n = 8): every
    instance runs its own multiplier loop on the device (ctol 1e-6, gtol 1e-6). Each step
    restores the initial multipliers and penalties, so every step does the same work."""
    import torch
    from paper_2106_14995_amd import tron
    from paper_2106_14995_amd import workloads as W
    B = args.batch
    log(f"generating {B} BR8L instances")
    bt = W.br8l_batch(B)
    stream = torch.cuda.current_stream()
    params0, lo, hi, x0 = tron.to_device(bt)
    params = params0.clone()
    x = torch.empty(8 * B, dtype=torch.float64, device="cuda")
    h = tron.Batch(W.BR8L, 8, batch=B)

    def step():
        params.copy_(params0)
        return h.al_solve(params, lo, hi, x0, x=x, stream=stream)

    lat, total = time_solves(step, args.steps, args.warmup, stream)
    _, f, st, it, outer, viol = step()
    torch.cuda.synchronize()
    st, outer, it = st.cpu().numpy(), outer.cpu().numpy(), it.cpu().numpy()
    print(json.dumps({"config": f"{B} BR8L branch subproblems with line limits, multiplier loop on the device",
                      "al_solves_per_s": B * args.steps / total, "p50_ms": float(np.median(lat)),
                      "p99_ms": float(np.percentile(lat, 99)), "converged": int((st == 0).sum()),
                      "status_counts": np.bincount(st, minlength=6).tolist(),
                      "outer_mean": float(outer.mean()), "outer_max": int(outer.max()),
                      "tron_iters_mean": float(it.mean()), "binding_limits": int(((x.view(B, 8)[:, 6:] <= 0.0).any(1)).sum().item())}),
          flush=True)
    h.close()


def bench_design(args):
    """The kernel-design comparisons of section 4 on gfx950: 10,000 SPD blocks per size,
    n = 1..32 as in the paper (plus 48 and 64): left- against right-looking Cholesky in LDS and
    left-looking in global memory (Tables 1 and 3), and the forward + backward substitution
    pair with L^T read in place (row stride n, or odd stride n|1), with an explicit L^T copy,
    and from global memory (Table 2). Each figure is the mean HIP-event time of one batched
    launch; the solves run `reps` = 8 times inside the kernel and are reported per pair."""
    import torch
    from paper_2106_14995_amd import tron
    from paper_2106_14995_amd import workloads as W
    count, reps = 10000, 8
    stream = torch.cuda.current_stream()
    chol_names = {tron.CHOL_LEFT_LDS: "left_lds", tron.CHOL_RIGHT_LDS: "right_lds",
                  tron.CHOL_LEFT_GLOBAL: "left_global", tron.CHOL_BLOCKED_MFMA: "blocked_mfma"}
    trsv_names = {tron.TRSV_IMPLICIT: "implicit_stride_n", tron.TRSV_PADDED: "implicit_stride_odd",
                  tron.TRSV_EXPLICIT: "explicit_lt", tron.TRSV_GLOBAL: "global"}
    rows = []
    for n in list(range(1, 33)) + [48, 64]:
        A, B = W.spd_blocks(count, n)
        Ad = torch.from_numpy(A).cuda()
        Bd = torch.from_numpy(B).cuda()
        Ld, info = tron.design_chol(tron.CHOL_LEFT_LDS, Ad)
        Lout = torch.empty_like(Ad)
        x = torch.empty_like(Bd)
        row = {"n": n}
        for v, nm in chol_names.items():
            lat, _ = time_solves(lambda: tron.design_chol(v, Ad, l=Lout, info=info, stream=stream),
                                 args.steps, args.warmup, stream)
            row["chol_" + nm + "_ms"] = float(np.mean(lat))
        for v, nm in trsv_names.items():
            lat, _ = time_solves(lambda: tron.design_trsv(v, Ld, Bd, x=x, reps=reps, stream=stream),
                                 args.steps, args.warmup, stream)
            row["trsv_" + nm + "_ms"] = float(np.mean(lat)) / reps
        rows.append(row)
        log(f"n={n}: " + ", ".join(f"{k} {v:.4f}" for k, v in row.items() if k != "n"))
    paper_range = [r for r in rows if r["n"] <= 32]
    mean = {k: float(np.mean([r[k] for r in paper_range])) for k in rows[0] if k != "n"}
    print(json.dumps({"config": f"{count} SPD blocks per size (A = M'M + nI), one wavefront per block",
                      "mean_over_n_1_to_32_ms": mean, "rows": rows,
                      "paper_context": "V100, 10,000 matrices, 1 <= n <= 32: Cholesky left 0.362 ms, right 0.437 ms "
                                       "(Table 1); backward substitution explicit 0.875 ms, implicit 1.408 ms "
                                       "(Table 2)"}), flush=True)


def bench_groups(args):
    """The group-width sweep (section 4.2's thread configuration): one instance per G lanes,
    G = 1 (the lane kernel), 2, 4, 8, 16, or the whole 64-lane wavefront (the wave kernel),
    on uniform batches of 16,384 instances of the quartic family and of the hs45 variant
    (random starts) for every n = 1..32, with every width that has a build at that n (1, 2, 4,
    8 and 64 lanes up to n = 8; 8, 16 and 64 up to 16; the wavefront above), and on the
    65,536-instance branch batch. Each figure is the time of one solve of the batch (mean of
    the timed steps); the summary names the fastest width per family and n."""
    import torch
    from paper_2106_14995_amd import tron
    from paper_2106_14995_amd import workloads as W
    stream = torch.cuda.current_stream()
    rows = []

    def run(label, fam, bt, n, spec, dev):
        h = tron.Batch(fam, n, batch=bt.batch, spec=spec)
        lat, total = time_solves(lambda: h.solve(*dev, stream=stream), args.steps, args.warmup, stream)
        _, _, st, it = h.solve(*dev, stream=stream)
        torch.cuda.synchronize()
        row = {"case": label, "n": n, "batch": bt.batch, "lanes_per_instance": h.plan()[0]["lanes"],
               "ms_per_batch": 1e3 * total / args.steps, "converged": int((st == 0).sum().item()),
               "iters_max": int(it.max().item())}
        h.close()
        rows.append(row)
        log(f"{label} n={n} G={row['lanes_per_instance']}: {row['ms_per_batch']:.4f} ms")

    br = W.br6_batch(65536, config_id=1)
    dev = tron.to_device(br)
    for g in (1, 2, 4, 8):
        run("br6", W.BR6, br, 6, tron.plan_spec(lane_group=g), dev)
    for label, fam in (("qp4", W.QP4), ("hs45m_random_start", W.HS45M)):
        for n in range(1, 33):
            bt = W.qp4_batch(16384, n, config_id=120 + n) if fam == W.QP4 else \
                W.hs45m_random_start(16384, n, config_id=130 + n)
            dev = tron.to_device(bt)
            if n <= 8:
                specs = [tron.plan_spec(lane_group=g) for g in (1, 2, 4, 8)] + [tron.plan_spec(lane_max_n=0)]
            elif n <= 16:
                specs = [tron.plan_spec(group16=g) for g in (8, 16)] + [tron.plan_spec()]
            else:
                specs = [tron.plan_spec()]
            for sp in specs:
                run(label, fam, bt, n, sp, dev)
            del dev
    best = {}
    for r in rows:
        k = (r["case"], r["n"])
        if k not in best or r["ms_per_batch"] < best[k]["ms_per_batch"]:
            best[k] = r
    summary = [{"case": c, "n": n, "best_lanes_per_instance": r["lanes_per_instance"],
                "ms_per_batch": r["ms_per_batch"]} for (c, n), r in sorted(best.items())]
    print(json.dumps({"config": "group-width sweep: uniform batches, one solve per step, gtol 1e-6",
                      "rows": rows, "best": summary}), flush=True)


def bench_workspace(args):
    """Where the solver keeps its matrices (section 4.5, Table 3, for the whole solve rather
    than one factorisation): registers (the lane kernel, n <= 8, and the group kernel of 16
    lanes, n <= 16), LDS (the wavefront kernel) and a global-memory workspace read through L2
    (the wavefront kernel's form beyond n = 128, forced below it), on 10,000 quartic problems
    per size."""
    import torch
    from paper_2106_14995_amd import tron
    from paper_2106_14995_amd import workloads as W
    stream = torch.cuda.current_stream()
    B = 10000
    rows = []
    for n in (8, 16, 32, 64, 128):
        bt = W.qp4_batch(B, n, config_id=140 + n)
        dev = tron.to_device(bt)
        forms = [("lds", tron.plan_spec(lane_max_n=0)), ("global", tron.plan_spec(lane_max_n=0, wave_global=1))]
        if n <= 8:
            forms.insert(0, ("registers_lane", tron.plan_spec()))
        if n <= 16:
            forms.insert(0, ("registers_group16", tron.plan_spec(lane_max_n=0, group16=16)))
        row = {"n": n}
        for name, spec in forms:
            h = tron.Batch(W.QP4, n, batch=B, spec=spec)
            lat, total = time_solves(lambda: h.solve(*dev, stream=stream), args.steps, args.warmup, stream)
            _, _, st, _ = h.solve(*dev, stream=stream)
            torch.cuda.synchronize()
            row[name + "_ms"] = 1e3 * total / args.steps
            row[name + "_converged"] = int((st == 0).sum().item())
            h.close()
        rows.append(row)
        log(f"n={n}: " + ", ".join(f"{k} {v:.3f}" for k, v in row.items() if k.endswith("_ms")))
    print(json.dumps({"config": f"whole-solve workspace comparison, {B} quartic problems per size, gtol 1e-6",
                      "rows": rows, "paper_context": "Table 3 (V100): shared memory 9.536 ms, global "
                      "memory slower, for its hs45 batch"}), flush=True)


def bench_serve(args):
    """Serving: requests of B = round(exp(U[0, ln 4096])) quartic problems with n log-uniform
    in [4,128], drawn as slices of a seeded pool. The saturated instance rate is measured with
    every request submitted at once; then Poisson arrivals at 0.25/0.5/0.75/0.9 of that rate
    (in requests/s = rate / E[B]) give per-request latency (submission to completion) and
    throughput, for the continuous-batching server and for the naive FIFO configuration (one
    request on the device at a time, one stream, no coalescing: a launch per size bucket per
    request)."""
    import math
    import threading
    from paper_2106_14995_amd import tron
    from paper_2106_14995_amd import workloads as W
    P = 12000
    log(f"generating a pool of {P} instances, n log-uniform in [4,128]")
    sizes = W.loguniform_sizes(P, 4, 128, config_id=4)
    pool = W.qp4_batch(P, sizes, config_id=4)
    vo, po = pool.voff(), pool.poff()
    rng = np.random.default_rng(4)
    R = args.requests

    def make_requests(seed):
        r = np.random.default_rng(seed)
        out = []
        for _ in range(R):
            b = int(round(math.exp(r.uniform(0.0, math.log(4096)))))
            b = max(1, min(b, 4096))
            s0 = int(r.integers(0, P - b + 1))
            out.append((pool.n[s0:s0 + b], pool.params[po[s0]:po[s0 + b]], pool.lo[vo[s0]:vo[s0 + b]],
                        pool.hi[vo[s0]:vo[s0 + b]], pool.x0[vo[s0]:vo[s0 + b]]))
        return out

    reqs = make_requests(44)
    mean_b = float(np.mean([len(q[0]) for q in reqs]))

    def run(srv_kw, qps):
        srv = tron.Server(W.QP4, **srv_kw)
        t_arr = np.cumsum(rng.exponential(1.0 / qps, R)) if qps else np.zeros(R)
        tickets = [None] * R
        t0 = time.perf_counter()

        def feeder():
            for i, q in enumerate(reqs):
                d = t0 + t_arr[i] - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                tickets[i] = srv.submit(*q)

        th = threading.Thread(target=feeder)
        th.start()
        th.join()
        lat = np.empty(R)
        for i, t in enumerate(tickets):
            srv.wait(t)
            lat[i] = srv.result(t)["latency"]
        wall = time.perf_counter() - t0
        inst = srv.stats()["instances"]
        srv.close()
        return dict(solves_per_s=inst / wall, p50_ms=1e3 * float(np.percentile(lat, 50)),
                    p99_ms=1e3 * float(np.percentile(lat, 99)), wall_s=wall)

    served = dict(hbm_budget=4 << 30, max_inflight=8, streams=4, coalesce=True)
    naive = dict(hbm_budget=4 << 30, max_inflight=1, streams=1, coalesce=False)
    log("saturation (all requests at once)")
    sat = run(served, 0.0)
    sat_naive = run(naive, 0.0)
    res = {"config": f"serving: {R} requests per level, B log-uniform in [1,4096] (mean {mean_b:.0f}), "
                     "n log-uniform in [4,128], quartic problems, gtol 1e-6",
           "saturated": {"served": sat, "naive": sat_naive}, "levels": []}
    for frac in (0.25, 0.5, 0.75, 0.9):
        qps = frac * sat["solves_per_s"] / mean_b
        log(f"load {frac}: {qps:.0f} requests/s")
        res["levels"].append({"load": frac, "qps": qps, "served": run(served, qps), "naive": run(naive, qps)})
    print(json.dumps(res), flush=True)


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
    ap.add_argument("--config", default="br6", choices=["br6", "qp4", "uneven", "admm", "serve", "hs45m", "al", "design", "large", "groups", "workspace"],
                    help="br6: the headline batch (default); qp4: 256 x n=8 quartic problems "
                         "(oracle CPU seconds and GPU time); uneven: 50,000 quartic problems with "
                         "n log-uniform in [4,64], bucketed graph vs one launch per size; admm: "
                         "the component ADMM on the 2,000-bus synthetic network; serve: Poisson "
                         "stream of requests of 1-4,096 quartic problems, n log-uniform in [4,128]; "
                         "hs45m: the paper's hs45 variant, 10,000 instances, n = 1..32; al: the "
                         "multiplier loop on branch subproblems with line limits; design: the "
                         "Cholesky / triangular-solve / workspace variants of section 4; groups: "
                         "the group-width sweep (lanes per instance); workspace: registers vs "
                         "LDS vs global memory for the whole solve")
    ap.add_argument("--requests", type=int, default=2000, help="serve: requests per load level")
    ap.add_argument("--plan", default="", help="uneven: time only this plan (bucketed_streams, "
                    "bucketed_graph, persistent_8_graph, persistent_12_graph), e.g. for profiling")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path here (the instances "
              "are independent, so a multi-GPU run would split the batch by instance)",
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
    if args.config != "br6":
        {"qp4": bench_qp4, "uneven": bench_uneven, "admm": bench_admm, "serve": bench_serve,
         "hs45m": bench_hs45m, "al": bench_al, "design": bench_design, "large": bench_large,
         "groups": bench_groups, "workspace": bench_workspace}[args.config](args)
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

    # throughput: K back-to-back solves between two device synchronisations; one pair of
    # events on the launch stream around them gives the kernel's mean launch duration
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        h.solve(params, lo, hi, x0, x, f, st, it, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    launch_ms = ev0.elapsed_time(ev1) / args.steps

    # latency: K more solves, each between its own pair of events (the event packets add a
    # few microseconds between launches, so this pass is kept out of the throughput)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    for k in range(args.steps):
        starts[k].record(stream)
        h.solve(params, lo, hi, x0, x, f, st, it, stream=stream)
        ends[k].record(stream)
    torch.cuda.synchronize()
    lat = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])  # ms per launch
    log(f"timed {args.steps} steps in {total:.3f} s; launch ms mean {launch_ms:.4f}, "
        f"bracketed one by one p50 {np.median(lat):.4f}")

    # per-instance solve latency from device timestamps (one more solve, outside the timing)
    ts = torch.zeros(2 * B, dtype=torch.int64, device="cuda")
    tron.lib().tron_batch_set_timestamps(h._h, tron.C.c_void_p(ts.data_ptr()))
    h.solve(params, lo, hi, x0, x, f, st, it, stream=stream)
    torch.cuda.synchronize()
    tron.lib().tron_batch_set_timestamps(h._h, None)
    rate = float(tron.lib().tron_clock_rate_hz())
    tsn = ts.cpu().numpy().reshape(B, 2).astype(np.float64)
    inst_us = (tsn[:, 1] - tsn[:, 0]) / rate * 1e6 if rate > 0 else np.zeros(B)

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
        "instance_latency_us": {"p50": float(np.percentile(inst_us, 50)),
                                "p99": float(np.percentile(inst_us, 99)),
                                "max": float(inst_us.max())},
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
        kern_s = launch_ms * 1e-3
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
        # both bounds, since the branch batch sits at the ridge (~9.7 flop/B against 9.8)
        roof["frac_fp64"] = flops / kern_s / PEAK_FP64_VECTOR
        roof["frac_hbm"] = bytes_ / kern_s / PEAK_HBM
        traffic = measured_traffic("lane_kernel<mt::BR6, 6>")
        roof["traffic"] = traffic
        if traffic is not None:
            roof["traffic_unit"] = "bytes per launch (FETCH_SIZE x2.000 + WRITE_SIZE x1.000)"
            roof["traffic_over_algorithmic"] = traffic / bytes_
        roof["flops_per_instance"] = cb["flops_per_instance"]
        roof["bytes_per_instance"] = BR6_BYTES
        roof["hbm_gbs_algorithmic"] = bytes_ / kern_s / 1e9
        log("measured peaks (FMA chains, copy)")
        mp = measured_peaks(stream)
        roof["measured_peaks"] = mp
        roof["frac_of_measured"] = {"fp64": flops / kern_s / (mp["fp64_tflops"] * 1e12),
                                    "hbm": bytes_ / kern_s / (mp["hbm_gbs"] * 1e9)}
        result["roofline"] = roof
        result["cpu_baseline"] = {
            "value": cb["value"], "unit": "solves/s", "cores": cb["threads"], "kind": "oracle",
            "sample": f"the same {B}-instance batch, {cb['reps']} passes, {cb['wall']:.2f} s wall",
        }
    print(json.dumps(result), flush=True)
    h.close()


if __name__ == "__main__":
    main()
