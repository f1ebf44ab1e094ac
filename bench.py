"""Throughput of the exact K-S change-point scan on one MI355X: plain scan and CNN proposal.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c5] [--extra c2,c3]

One step = one ks_scan_batch call over the whole batch (eq. 2 reduction,
K-S at every candidate, choice, significance and p-value for every series),
with the samples already resident in HBM. Prints ONE JSON line for the
headline workload (default c5, the largest configuration: 8192 series x K=1024
x N=2048, 64 GiB of samples). Besides the plain scan it carries:
  learned     propose + exact refine with the trained network (and the same
              refine around the proposal of the method without the network)
  segment     every level boundary by binary segmentation
  row_stats   per-row mean, std, min, p50, p95, max
  check       workflow step 3's outlier check and widening, and the L2 segment
              alignment, on the same detections
  line_size   the cache-line-size scoring on its own synthetic experiments
  workloads   the plain scan and the learned leg on the --extra workloads
  cpu_baseline  the CPU oracle on a bounded sample of the headline workload,
              on every core of this process's CPU share and on one core

Workloads (seeded synthetic sweeps, see paper_2511_05958_amd.synth):
  c1  1 series, K=64, N=256            (launch-latency bound, not an HBM number)
  c2  4096 series, K=256, N=1024        (4 GiB of samples)
  c3  16384 uneven series, K~logU[32,512], N~logU[64,4096]
  c5  8192 series, K=1024, N=2048       (default; 64 GiB of samples)
  copy  a plain device-to-device copy of 1 GiB (the reference kernel that
        calibrates the FETCH_SIZE / WRITE_SIZE counters; prints bytes moved)
  ceiling  the achievable HBM read bandwidth: ks_probe_read over 4 GiB, best
        of a sweep of grid sizes and unroll depths (prints GB/s per point)
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
MODEL_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2511_05958_amd", "models")

# proposal networks trained on each workload's shapes (recipe 4 = recipe 2 under its own seed;
# recipes 3 and 5 from series ids 2^20 on, disjoint from the benchmark batches)
MODELS = {"c1": "proposal_r4.ckpt", "c2": "proposal_r4.ckpt", "c3": "proposal_r3.ckpt", "c5": "proposal_r5.ckpt"}

WORKLOADS = {
    "c1": (1, None, "1 series x K=64 x N=256 (one 120->320 cycle change)"),
    "c2": (2, None, "4096 series x K=256 x N=1024 (1-4 planted levels)"),
    "c3": (3, None, "16384 uneven series, K~logU[32,512], N~logU[64,4096], 0-4 changes with ramps"),
    "c5": (5, None, "8192 series x K=1024 x N=2048, hard regime (adjacent level ratios 1.05-1.2, Pareto tails, "
                    "5% outliers)"),
}
METRIC = "KS change-point series/s at 1 GPU (plain vs CNN-proposal), % HBM roofline"
# scan-kernel variants of ks_launch.variant (include/ks.h): workgroup threads, radix bits, walk slots (0: share)
SCAN_VARIANTS = [(256, 4, 0), (128, 4, 0), (512, 4, 0), (256, 8, 0), (256, 4, 1), (256, 4, 2)]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(batch, samples_dev, sample_series: int = 512, target_s: float = 8.0) -> dict:
    """The CPU oracle, as it stands, on a bounded sample of the headline workload: the
    first `sample_series` series of the batch, copied from HBM (the generator is keyed by
    series id and bit-identical on host and device, so these are exactly the series the
    host generator would regenerate). Timed on every core of this process's CPU share
    (os.sched_getaffinity, capped at OMP_NUM_THREADS when that is set) and on one core;
    one core takes as many of those series as fit in about target_s seconds. Rates are
    series/s, so they scale to the whole batch directly (batch seconds = series / rate)."""
    import numpy as np

    import oracle as O

    sp = batch.specs
    count = max(1, min(sample_series, batch.num_series))
    ends = sp["offset"].astype(np.int64) + sp["K"].astype(np.int64) * sp["N"].astype(np.int64)
    x = samples_dev[: int(ends[count - 1])].cpu().numpy().view(np.uint32)
    affinity = len(os.sched_getaffinity(0))
    share = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    cores = min(affinity, share) if share > 0 else affinity

    def timed_run(n, threads):
        t0 = time.perf_counter()
        O.scan_batch(x, sp["offset"][:n], sp["K"][:n], sp["N"][:n], threads=threads)
        return time.perf_counter() - t0

    dt_all = timed_run(count, cores)
    probe = min(count, 8)
    rate1 = probe / timed_run(probe, 1)
    n1 = int(min(count, max(probe, rate1 * target_s)))
    dt1 = timed_run(n1, 1)
    gib = 4 * int(ends[count - 1]) / 2**30
    full_s = batch.num_series / (count / dt_all)
    return {
        "value": count / dt_all,
        "unit": "series/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"series 0..{count - 1} of the {batch.num_series}-series batch ({gib:.2f} GiB, copied from HBM; "
                  f"bit-identical to regenerating them from their Philox streams), {cores} threads, {dt_all:.2f} s; "
                  f"scaled to the whole batch: {full_s:.1f} s",
        "one_core": {"value": n1 / dt1, "unit": "series/s", "cores": 1, "series": n1, "seconds": dt1,
                     "batch_seconds_scaled": batch.num_series / (n1 / dt1)},
        "nproc": os.cpu_count(),
        "affinity_cores": affinity,
        "cpu_model": cpu_model(),
    }


def learned_leg(args, ctx, batch, samples, desc, prm, stream, res_plain, plain_value, model_path) -> dict:
    """Propose + exact refine on the same batch, timed like the plain step; agreement with the
    plain scan and fallback rate at the model's calibrated tau. Beside it, the same refine around
    the proposal of the method without the network (ks_propose with no model: the largest jump
    of the per-row median, always refined), its agreement and series/s."""
    import numpy as np
    import torch

    import paper_2511_05958_amd as P

    rep_path = os.path.splitext(model_path)[0] + ".json"
    with open(rep_path) as f:
        rep = json.load(f)
    n = batch.num_series
    lp = P.ks_params_init(prm.alpha)
    lp.max_K = prm.max_K
    lp.w = 8
    lp.tau = float(rep["tau"])
    model = P.Model(ctx, seed=0)
    P.ks_model_load(model.handle, model_path)
    prop = torch.empty(n, dtype=torch.int32, device="cuda")
    conf = torch.empty(n, dtype=torch.float32, device="cuda")
    out = P.empty_results(n)

    def run(handle):
        def step():
            P.ks_propose(ctx.handle, handle, samples, desc, n, lp, prop, conf, stream=stream)
            P.ks_refine(ctx.handle, desc, n, batch.total_elems, prop, conf, lp, out, stream=stream)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(args.steps):
            step()
        e1.record(stream)
        torch.cuda.synchronize()
        wall_ms = (time.perf_counter() - t0) / args.steps * 1e3
        r = P.results_to_numpy(out)
        agree = (r["cp"] == res_plain["cp"]) & (r["U"] == res_plain["U"])
        return wall_ms, e0.elapsed_time(e1) / args.steps, r, agree

    wall_ms, ev_ms, r, agree = run(model.handle)
    t_ms, _, _, t_agree = run(None)
    model.close()
    value = n / (wall_ms / 1e3)
    cal = rep.get("calibration", {})
    return {
        "value": value,
        "unit": "series/s",
        "ms_per_step": wall_ms,
        "step_ms_events": ev_ms,
        "vs_plain": value / plain_value,
        "agreement": float(agree.mean()),
        "fallback_rate": float(np.mean((r["flags"] & P.KS_FALLBACK) != 0)),
        "w": lp.w,
        "tau": lp.tau,
        "tau_calibration": {"series": cal.get("series", rep.get("val_series")),
                            "target": cal.get("target", rep.get("target")),
                            "held_out_agreement": cal.get("agreement_at_tau", rep.get("val_agreement_at_tau"))},
        "hbm_GBps_whole_step": (batch.sample_bytes + 48 * n) / (ev_ms / 1e3) / 1e9,
        "model": os.path.basename(model_path),
        "without_network": {"value": n / (t_ms / 1e3), "unit": "series/s", "ms_per_step": t_ms,
                            "agreement": float(t_agree.mean()), "fallback_rate": 0.0,
                            "proposal": "largest jump of the per-row median, always refined"},
    }


def segment_leg(args, ctx, batch, samples, desc, prm, stream) -> dict:
    """Every level boundary of each series (binary segmentation), timed per whole batch.
    HBM bytes are counted exactly from the output: the samples once (depth 0), the 24-byte
    row moments written at depth 0, and read again for every row of a later window (both
    sides, of >= 2 rows, of every boundary's window)."""
    import numpy as np
    import torch

    import paper_2511_05958_amd as P

    n = batch.num_series
    max_cp = 64
    cps = torch.empty(n * max_cp * 48, dtype=torch.uint8, device="cuda")
    counts = torch.empty(n, dtype=torch.int32, device="cuda")

    def step():
        P.ks_segment_batch(ctx.handle, samples, desc, n, prm, 0, max_cp, cps, counts, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) / args.steps * 1e3
    c = counts.cpu().numpy().view(np.uint32)
    v = cps.cpu().numpy().view(P.RESULT_DTYPE).reshape(n, max_cp)
    Ns = batch.specs["N"].astype(np.int64)
    rows = batch.specs["K"].astype(np.int64).copy()
    depth = 0
    for t in range(n):
        k = min(int(c[t]), max_cp) if c[t] != P.KS_SEGMENT_BAD else 0
        w = v[t][:k]
        rows[t] += int(np.sum(np.where(w["n"] >= 2, w["n"], 0)) + np.sum(np.where(w["m"] >= 2, w["m"], 0)))
        depth = max(depth, int(w["pad"].max()) + 1 if k else 0)
    K0 = batch.specs["K"].astype(np.int64)
    hbm = int(np.sum(4 * K0 * Ns) + 24 * np.sum(K0) + 24 * np.sum(rows - K0))
    return {
        "value": n / (wall_ms / 1e3),
        "unit": "series/s",
        "ms_per_step": wall_ms,
        "boundaries_per_series": float(np.mean(np.where(c == P.KS_SEGMENT_BAD, 0, c))),
        "truncated_series": int(np.count_nonzero((c != P.KS_SEGMENT_BAD) & (c > max_cp))),
        "depths": depth + 1,
        "window_rows": int(np.sum(rows)),
        "hbm_bytes": hbm,
        "hbm_GBps": hbm / (wall_ms / 1e3) / 1e9,
    }


def stats_leg(args, batch, samples, desc, prm, ctx, stream, out=None) -> dict:
    """Per-row latency statistics (ks_stats_batch) of the whole batch: one read of the samples.
    `out` is an output buffer of at least 32 bytes per row allocated beforehand, or None."""
    import numpy as np
    import torch

    import paper_2511_05958_amd as P

    rows = int(batch.specs["K"].astype(np.int64).sum())
    if out is None or out.numel() < rows * 32:
        out = torch.empty(rows * 32, dtype=torch.uint8, device="cuda")

    def step():
        P.ks_stats_batch(ctx.handle, samples, desc, batch.num_series, prm.max_K, out, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(args.steps):
        step()
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / args.steps
    return {"value": rows / (ms / 1e3), "unit": "rows/s", "ms_per_step": ms,
            "series_per_s": batch.num_series / (ms / 1e3),
            "hbm_GBps": (batch.sample_bytes + 32 * rows) / (ms / 1e3) / 1e9}, out


def timed(args, stream, fn) -> float:
    """Average ms of fn over args.steps calls after args.warmup, HIP events on `stream`."""
    import torch

    for _ in range(args.warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(args.steps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / args.steps


def check_leg(args, ctx, batch, desc, prm, out_plain, stats, stats_ms, stream) -> dict:
    """Workflow step 3 on every sweep (ks_check_batch: outlier check and widening from the
    detection and the per-step p50), and the L2 segment alignment (ks_align_batch) of each
    significant sweep's boundary size against a 32 MiB reported L2 (8 XCDs x 4 MiB). The
    chain after the scan is ks_stats_batch (timed in row_stats) + ks_check_batch."""
    import numpy as np
    import torch

    import paper_2511_05958_amd as P

    n = batch.num_series
    out = torch.empty(n * 32, dtype=torch.uint8, device="cuda")
    ms = timed(args, stream, lambda: P.ks_check_batch(ctx.handle, desc, n, prm.max_K, out_plain, stats, out,
                                                       stream=stream))
    chk = out.cpu().numpy().view(P.CHECK_DTYPE)
    fl = chk["flags"]
    res = P.results_to_numpy(out_plain)
    sig = np.nonzero(res["flags"] & P.KS_SIGNIFICANT)[0]
    # boundary size of a significant sweep: footprint 1 KiB * 2^(16 cp / (K - 1)) (the sweep's rows)
    K = batch.specs["K"][sig].astype(np.float64)
    S_ = np.rint(1024.0 * np.exp2(16.0 * res["cp"][sig] / (K - 1))).astype(np.int64)
    m = len(sig)
    Sd = torch.tensor(S_, device="cuda")
    Td = torch.full((m,), 32 << 20, dtype=torch.int64, device="cuda")
    seg = torch.empty(m, dtype=torch.int32, device="cuda")
    al = torch.empty(m, dtype=torch.float64, device="cuda")
    di = torch.empty(m, dtype=torch.float64, device="cuda")
    ams = timed(args, stream, lambda: P.ks_align_batch(Sd, Td, m, seg, al, di, stream=stream)) if m else 0.0
    return {"value": n / ((stats_ms + ms) / 1e3), "unit": "sweeps/s", "ms_per_step": stats_ms + ms,
            "check_kernel_ms": ms, "per_step_stats_ms": stats_ms,
            "edge_low": int(np.count_nonzero(fl & P.KS_CHECK_EDGE_LOW)),
            "edge_high": int(np.count_nonzero(fl & P.KS_CHECK_EDGE_HIGH)),
            "no_change": int(np.count_nonzero(fl & P.KS_CHECK_NO_CHANGE)),
            "disturbed": int(np.count_nonzero(fl & P.KS_CHECK_DISTURBED)),
            "invalid": int(np.count_nonzero(fl & P.KS_CHECK_INVALID)),
            "align": {"items": m, "ms": ams}}


def line_leg(args, ctx, stream, num_exp: int = 1024, J: int = 16, A: int = 32, N: int = 256) -> dict:
    """Cache-line-size scoring: num_exp synthetic experiments (J strides x A array sizes x N
    latencies, synth.line_experiments) through ks_stats_batch (p50 per stride and size) and
    ks_line_batch, timed as one step; accuracy = share of experiments whose line size is
    the planted one."""
    import numpy as np
    import torch

    import paper_2511_05958_amd as P
    from paper_2511_05958_amd import synth as S

    x, strides, planted = S.line_experiments(num_exp, J, A, N)
    K = J * A
    d = P.make_desc(np.arange(num_exp, dtype=np.int64) * K * N, [K] * num_exp, [N] * num_exp)
    xd, dd = P.to_device(x), P.to_device(d)
    st = torch.tensor(strides.view(np.int32), device="cuda")
    stats = torch.empty(num_exp * K * 32, dtype=torch.uint8, device="cuda")
    out = torch.empty(num_exp * 24, dtype=torch.uint8, device="cuda")

    def step():
        P.ks_stats_batch(ctx.handle, xd, dd, num_exp, K, stats, stream=stream)
        P.ks_line_batch(ctx.handle, dd, num_exp, stats, J, st, out, stream=stream)

    ms = timed(args, stream, step)
    lms = timed(args, stream, lambda: P.ks_line_batch(ctx.handle, dd, num_exp, stats, J, st, out, stream=stream))
    r = out.cpu().numpy().view(P.LINE_DTYPE)
    return {"value": num_exp / (ms / 1e3), "unit": "experiments/s", "ms_per_step": ms, "line_kernel_ms": lms,
            "experiments": num_exp, "strides": J, "sizes": A, "samples": N, "sample_bytes": int(x.nbytes),
            "hbm_GBps": x.nbytes / (ms / 1e3) / 1e9,
            "planted_found": float(np.mean(r["line"] == planted)),
            "inconclusive": int(np.count_nonzero(r["flags"] & (P.KS_LINE_INCONCLUSIVE | P.KS_LINE_INVALID)))}


# Sources of the scan kernels (plain path); their hash ties a recorded HBM
# traffic figure to the code it was measured on.
# (The ABI structs of include/ks.h are pinned separately: static_asserts on their sizes and the
# ctypes layouts' itemsize checks.)
SCAN_SOURCES = ["paper_2511_05958_amd/csrc/ks_wave.hpp", "paper_2511_05958_amd/csrc/ks_scan.hpp",
                "paper_2511_05958_amd/csrc/ks_persist.hpp", "paper_2511_05958_amd/csrc/ks_ctx.hpp",
                "paper_2511_05958_amd/csrc/ks_api.hip", "paper_2511_05958_amd/csrc/ks_scan_variants.hip"]
TRAFFIC_FILE = os.path.join("profiles", "hbm_traffic.txt")


def scan_sources_sha() -> str:
    import hashlib

    root = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for f in SCAN_SOURCES:
        h.update(f.encode())
        h.update(b"\0")
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(kernel: str, workload: str):
    """HBM bytes per launch measured by rocprofv3 for this kernel configuration
    (<kernel>:v<variant>:<split bytes>) and workload on the current sources, or
    None (no record, or the kernel changed since)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    sha = scan_sources_sha()
    with open(path) as fh:
        for line in fh:
            f = line.split()
            if len(f) == 5 and not line.startswith("#") and f[0] == kernel and f[1] == workload and f[2] == sha:
                return int(f[3]) + int(f[4])
    return None


def copy_calibration(args) -> int:
    import torch

    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(args.warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(args.steps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / args.steps
    print(json.dumps({"workload": "copy", "read_bytes": nbytes, "write_bytes": nbytes, "ms": ms,
                      "GBps_read_plus_write": 2 * nbytes / ms / 1e6}), flush=True)
    return 0


def ceiling_points(grids_unrolls, steps: int, warmup: int) -> list[dict]:
    """ks_probe_read over 4 GiB: GB/s per (grid, unroll)."""
    import torch

    import paper_2511_05958_amd as P

    nbytes = 4 << 30
    buf = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    points = []
    for grid, unroll in grids_unrolls:
        for _ in range(max(1, warmup)):
            P.ks_probe_read(buf, grid, unroll, sink)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            P.ks_probe_read(buf, grid, unroll, sink)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        points.append({"grid": grid, "unroll": unroll, "ms": ms, "GBps": nbytes / ms / 1e6})
    del buf
    torch.cuda.empty_cache()
    return points


def read_ceiling(args) -> int:
    nbytes = 4 << 30
    points = ceiling_points([(g, u) for g in (1024, 2048, 4096, 8192, 16384, 65536) for u in (1, 8)], args.steps,
                            args.warmup)
    best = max(points, key=lambda q: q["GBps"])
    print(json.dumps({"workload": "ceiling", "bytes": nbytes, "best_GBps": best["GBps"],
                      "best_frac_of_peak": best["GBps"] / HBM_PEAK_GBS, "best": best, "points": points}), flush=True)
    return 0


def row_length_sweep(args) -> int:
    """Feature pass (ks_features) and statistics pass (ks_stats_batch) against row length: 4 GiB of
    samples per length, 256 rows per series, values uniform on [200, 500) (every decile inside the
    1024-bin window, as in latency rows). Shows the fixed per-row cost of the row pass."""
    import numpy as np
    import torch

    import paper_2511_05958_amd as P

    ctx = P.Context(0)
    st = torch.cuda.current_stream()
    points = []
    K = 256
    for N in (64, 128, 256, 512, 1024, 2048):
        n = (4 << 30) // (K * N * 4)
        total = n * K * N
        gen = torch.Generator(device="cuda")
        gen.manual_seed(1000 + N)
        x = torch.randint(0, 300, (total,), device="cuda", dtype=torch.int32, generator=gen) + 200
        d = P.make_desc(np.arange(n, dtype=np.uint64) * (K * N), np.full(n, K, np.uint32), np.full(n, N, np.uint32))
        dd = P.to_device(d)
        rows = n * K
        P.ks_learn_reserve(ctx.handle, n, K)
        out = torch.empty(rows * 32, dtype=torch.uint8, device="cuda")
        pt = {"N": N, "series": n, "rows": rows, "bytes": total * 4}
        for name, fn in (("features", lambda: P.ks_features(ctx.handle, x, dd, n, K, None, stream=st)),
                         ("stats", lambda: P.ks_stats_batch(ctx.handle, x, dd, n, K, out, stream=st))):
            ms = timed(args, st, fn)
            pt[name] = {"ms": ms, "ns_per_row": ms * 1e6 / rows, "TBps": total * 4 / ms / 1e9}
        points.append(pt)
        print(json.dumps(pt), flush=True)
        del x, out, dd
        torch.cuda.empty_cache()
    ctx.close()
    print(json.dumps({"workload": "rowlen", "points": points}), flush=True)
    return 0


def reserve_outputs(args, ctx, keys):
    """Allocate the per-row buffers of the learned and statistics legs before any sample batch, as an
    application sizes its workspaces before loading data: the learned-path workspace for every workload
    in `keys` whose learned leg runs, and the statistics output of the first one (None if skipped)."""
    import numpy as np
    import torch

    import paper_2511_05958_amd as P
    from paper_2511_05958_amd import synth as S

    stats_out = None
    for i, key in enumerate(keys):
        recipe, count, _ = WORKLOADS[key]
        spec = S.make_batch(recipe, num_series=count).specs
        if spec["N"].max() > P.KS_FEATURE_MAX_N:
            continue
        mp = args.model if (i == 0 and args.model) else os.path.join(MODEL_DIR, MODELS.get(key, "proposal_r4.ckpt"))
        if not args.no_learned and os.path.exists(mp):
            P.ks_learn_reserve(ctx.handle, len(spec), int(spec["K"].max()))
        if i == 0 and not args.no_stats:
            stats_out = torch.empty(int(spec["K"].astype(np.int64).sum()) * 32, dtype=torch.uint8, device="cuda")
    return stats_out


def plain_scan(args, ctx, key, stream, launch="autotune"):
    """Generate workload `key` in HBM and time the plain exact scan on it: (record, state)."""
    import numpy as np
    import torch

    import paper_2511_05958_amd as P
    from paper_2511_05958_amd import synth as S

    recipe, count, label = WORKLOADS[key]
    batch = S.make_batch(recipe, num_series=count)
    n = batch.num_series
    samples = torch.empty(batch.total_elems, dtype=torch.int32, device="cuda")
    S.fill_device(batch, samples.data_ptr(), batch.total_elems)
    desc = P.to_device(P.make_desc(batch.specs["offset"], batch.specs["K"], batch.specs["N"]))
    out = P.empty_results(n)
    prm = P.ks_params_init(0.05)
    prm.max_K = int(batch.specs["K"].max())
    tune_ms = None
    if launch == "autotune":
        t0 = time.perf_counter()
        P.ks_autotune(ctx.handle, samples, desc, n, prm, out, stream=stream)
        tune_ms = (time.perf_counter() - t0) * 1e3
    elif launch != "default":
        cfg = {"grid": (P.KS_LAUNCH_GRID, args.chunk, 0), "ordered": (P.KS_LAUNCH_ORDERED, args.chunk, 1),
               "persistent": (P.KS_LAUNCH_PERSISTENT, args.chunk, 1),
               "persistent-direct": (P.KS_LAUNCH_PERSISTENT, args.chunk, 0)}[launch]
        P.ks_launch_set(ctx.handle, prm.max_K, n, *cfg, variant=args.variant)
    c = P.ks_launch_get(ctx.handle, prm.max_K, n)
    nt, rb, gm = SCAN_VARIANTS[c.variant]
    chosen = {"mode": ["grid", "persistent", "ordered"][c.mode], "chunk_bytes": c.chunk_bytes, "graph": c.graph,
              "variant": c.variant, "workgroup_threads": nt, "radix_bits": rb,
              "walk_slots_per_wave": gm or "share", "autotune_ms": tune_ms}

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
    bytes_per_launch = batch.sample_bytes + 48 * n
    kernel_name = "ks::scan_persistent" if c.mode == P.KS_LAUNCH_PERSISTENT else "ks::scan_kernel"
    achieved = bytes_per_launch / avg_kern_s / 1e9
    rec = {
        "value": n / (ms_per_step / 1e3),
        "unit": "series/s",
        "ms_per_step": ms_per_step,
        "config": {
            "workload": label,
            "series": n,
            "sample_bytes": batch.sample_bytes,
            "max_K": prm.max_K,
            "alpha": prm.alpha,
            "launch": chosen,
            "significant": int(np.count_nonzero(res["flags"] & P.KS_SIGNIFICANT)),
            "flagged_bad": int(np.count_nonzero(res["flags"] & (P.KS_BAD_SHAPE | P.KS_OUT_OF_RANGE))),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": recorded_traffic(f"{kernel_name}:v{c.variant}:{c.chunk_bytes if c.mode == P.KS_LAUNCH_PERSISTENT else 0}",
                                        key),
            "kernel": kernel_name,
            "kernel_ms": avg_kern_s * 1e3,
        },
    }
    return rec, (batch, samples, desc, out, prm, res)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c5", choices=sorted(WORKLOADS) + ["copy", "ceiling", "rowlen"])
    ap.add_argument("--extra", default="c2,c3",
                    help="comma-separated workloads whose plain scan, learned leg and statistics leg are added "
                         "under 'workloads' ('' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--launch", default="autotune",
                    choices=["autotune", "default", "grid", "ordered", "persistent", "persistent-direct"],
                    help="launch plan: autotune (time the candidates first, untimed), the library default, "
                         "one workgroup per series, largest-first ordered grid, persistent queue (hipGraph), "
                         "persistent queue with direct launches")
    ap.add_argument("--chunk", type=int, default=1 << 20, help="split size of the persistent plan (bytes)")
    ap.add_argument("--variant", type=int, default=0, help="scan-kernel variant with a fixed --launch plan")
    ap.add_argument("--model", default=None,
                    help="trained proposal network for the headline workload; its .json report holds tau (the "
                         "learned leg is skipped if absent). Default: the network trained on the workload's own "
                         "shapes (series ids disjoint from the benchmark batch)")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-segment", action="store_true", help="skip the binary-segmentation leg")
    ap.add_argument("--no-ceiling", action="store_true", help="skip the measured read-ceiling probe")
    ap.add_argument("--no-stats", action="store_true", help="skip the per-row statistics leg")
    ap.add_argument("--no-check", action="store_true",
                    help="skip the workflow-check legs (outlier check, L2 alignment, cache-line size)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU only (one GPU's share of a batch sharded by "
                                   "series); --gpus must be 1", "n_gpus": args.gpus}))
        return 2

    import torch

    import paper_2511_05958_amd as P

    if args.workload == "copy":
        return copy_calibration(args)
    if args.workload == "ceiling":
        return read_ceiling(args)
    if args.workload == "rowlen":
        return row_length_sweep(args)
    extras = [w for w in args.extra.split(",") if w and w != args.workload]
    for w in extras:
        if w not in WORKLOADS:
            raise SystemExit(f"unknown workload {w}")
    model_path = args.model or os.path.join(MODEL_DIR, MODELS.get(args.workload, "proposal_r4.ckpt"))
    ctx = P.Context(0)
    stream = torch.cuda.current_stream()
    stats_buf = reserve_outputs(args, ctx, [args.workload] + extras)
    rec, (batch, samples, desc, out, prm, res) = plain_scan(args, ctx, args.workload, stream, args.launch)
    n = batch.num_series
    line = {
        "metric": METRIC,
        "value": rec["value"],
        "unit": "series/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rec["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": rec["config"],
        "roofline": rec["roofline"],
    }
    achieved = rec["roofline"]["achieved"]
    if not args.no_ceiling:
        # the read bandwidth a plain 16-byte-load kernel reaches on this device (best of three
        # launch shapes of ks_probe_read; the full sweep is --workload ceiling)
        pts = ceiling_points([(2048, 1), (16384, 8), (65536, 8)], 5, 1)
        ceil_gbps = max(q["GBps"] for q in pts)
        line["roofline"]["measured_read_ceiling_GBps"] = ceil_gbps
        line["roofline"]["frac_of_measured_ceiling"] = achieved / ceil_gbps
    if not args.no_learned and os.path.exists(model_path) and batch.specs["N"].max() <= P.KS_FEATURE_MAX_N:
        line["learned"] = learned_leg(args, ctx, batch, samples, desc, prm, stream, res, rec["value"], model_path)
    if not args.no_segment:
        line["segment"] = segment_leg(args, ctx, batch, samples, desc, prm, stream)
    if not args.no_stats and batch.specs["N"].max() <= P.KS_FEATURE_MAX_N:
        line["row_stats"], stats_out = stats_leg(args, batch, samples, desc, prm, ctx, stream, stats_buf)
        if not args.no_check:
            line["check"] = check_leg(args, ctx, batch, desc, prm, out, stats_out, line["row_stats"]["ms_per_step"],
                                      stream)
        del stats_out
    stats_buf = None
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(batch, samples)
    del samples, desc, out
    torch.cuda.empty_cache()
    if not args.no_check:
        line["line_size"] = line_leg(args, ctx, stream)
    if extras:
        line["workloads"] = {}
    for w in extras:
        r, (b, s_, d_, o_, p_, res_) = plain_scan(args, ctx, w, stream, args.launch)
        mp = os.path.join(MODEL_DIR, MODELS.get(w, "proposal_r4.ckpt"))
        if not args.no_learned and os.path.exists(mp) and b.specs["N"].max() <= P.KS_FEATURE_MAX_N:
            r["learned"] = learned_leg(args, ctx, b, s_, d_, p_, stream, res_, r["value"], mp)
        if not args.no_stats and b.specs["N"].max() <= P.KS_FEATURE_MAX_N:
            r["row_stats"], so_ = stats_leg(args, b, s_, d_, p_, ctx, stream)
            del so_
        line["workloads"][w] = r
        del s_, d_, o_
        torch.cuda.empty_cache()
    ctx.close()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
