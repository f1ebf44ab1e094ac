"""Throughput of the exact K-S change-point scan on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]

One step = one ks_scan_batch call over the whole batch (eq. 2 reduction,
K-S at every candidate, choice, significance and p-value for every series),
with the samples already resident in HBM. Prints ONE JSON line.

Workloads (seeded synthetic sweeps, see paper_2511_05958_amd.synth):
  c1  1 series, K=64, N=256            (launch-latency bound, not an HBM number)
  c2  4096 series, K=256, N=1024        (default; 4 GiB of samples)
  c3  16384 uneven series, K~logU[32,512], N~logU[64,4096]
  c5  8192 series, K=1024, N=2048       (64 GiB of samples)
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published

WORKLOADS = {
    "c1": (1, None, "plain exact scan, 1 series x K=64 x N=256 (one 120->320 cycle change)"),
    "c2": (2, None, "plain exact scan, 4096 series x K=256 x N=1024 (1-4 planted levels)"),
    "c3": (3, None, "plain exact scan, 16384 uneven series, K~logU[32,512], N~logU[64,4096], ramps"),
    "c5": (5, None, "plain exact scan, 8192 series x K=1024 x N=2048 (hard regime)"),
}


def cpu_baseline(batch, sample_series: int, threads: int) -> dict:
    """The CPU oracle, as it stands, on a bounded sample of the same workload."""
    import numpy as np

    import oracle as O
    from paper_2511_05958_amd import synth as S

    sub = batch.subset(np.arange(min(sample_series, batch.num_series)))
    x = S.fill_host(sub, threads=threads)
    t0 = time.perf_counter()
    O.scan_batch(x, sub.specs["offset"], sub.specs["K"], sub.specs["N"], threads=threads)
    dt = time.perf_counter() - t0
    return {
        "value": sub.num_series / dt,
        "unit": "series/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"first {sub.num_series} series of the same batch, {threads} threads, {dt:.2f} s",
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=0, help="series in the CPU sample (0 = auto)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        return 2

    import numpy as np
    import torch

    import paper_2511_05958_amd as P
    from paper_2511_05958_amd import synth as S

    recipe, count, label = WORKLOADS[args.workload]
    batch = S.make_batch(recipe, num_series=count)
    n = batch.num_series
    dev = torch.device("cuda:0")
    samples = torch.empty(batch.total_elems, dtype=torch.int32, device=dev)
    S.fill_device(batch, samples.data_ptr(), batch.total_elems)
    desc = P.to_device(P.make_desc(batch.specs["offset"], batch.specs["K"], batch.specs["N"]), dev)
    out = P.empty_results(n, dev)
    prm = P.ks_params_init(0.05)
    prm.max_K = int(batch.specs["K"].max())
    ctx = P.Context(0)
    stream = torch.cuda.current_stream(dev)

    def step():
        P.ks_scan_batch(ctx.handle, samples, desc, n, prm, out, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev0[k].record(stream)
        step()
        ev1[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in zip(ev0, ev1)]
    avg_kern_s = sum(kern_ms) / len(kern_ms) / 1e3
    ms_per_step = wall / args.steps * 1e3

    res = P.results_to_numpy(out)
    bad = int(np.count_nonzero(res["flags"] & (P.KS_BAD_SHAPE | P.KS_OUT_OF_RANGE)))
    bytes_per_launch = batch.sample_bytes + 48 * n
    achieved = bytes_per_launch / avg_kern_s / 1e9
    line = {
        "metric": "KS change-point series/s at 1 GPU (plain exact scan), % HBM roofline",
        "value": n / (ms_per_step / 1e3),
        "unit": "series/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": label,
            "series": n,
            "sample_bytes": batch.sample_bytes,
            "max_K": prm.max_K,
            "alpha": prm.alpha,
            "significant": int(np.count_nonzero(res["flags"] & P.KS_SIGNIFICANT)),
            "flagged_bad": bad,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "kernel": "ks::scan_kernel",
            "kernel_ms": avg_kern_s * 1e3,
        },
    }
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        sample = args.cpu_sample or {1: 1, 2: 512, 3: 512, 5: 48}[recipe]
        line["cpu_baseline"] = cpu_baseline(batch, sample, threads)
    ctx.close()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
