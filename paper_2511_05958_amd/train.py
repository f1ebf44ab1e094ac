"""Training and evaluation of the proposal network, on the GPU with the library's kernels.

    python -m paper_2511_05958_amd.train --series 200000 --epochs 10 --out model.ckpt
    python -m paper_2511_05958_amd.train --recipe 5 --first-series 1048576 --series 40000 \
        --val 4000 --chunk 1024 --out proposal_r5.ckpt
    python -m paper_2511_05958_amd.train --calibrate --model proposal_r4.ckpt --recipe 4 \
        --first-series 2097152 --series 40000 --target 0.9975

Data: seeded synthetic sweeps of a training recipe, generated on the device in
chunks (only the per-row features stay resident). Recipe 4 is the shape of
recipe 2 under its own seed. For the hard regime (recipe 5) the training
series are recipe 5 series with ids from --first-series on, disjoint from the
benchmark batch's ids 0..8191 (the generator is keyed by series id). Labels: the
exact scan (ks_scan_batch): the change point of every significant series, -1
(skipped by the loss) otherwise. Inputs: ks_features. Steps: ks_train_step
(softmax cross-entropy, Adam). The last `val` series are held out; on them the
confidence threshold tau is calibrated as the smallest value at which the
refined choice agrees with the full scan on at least `target` of the series.

Agreement of a series = the refined result has the same change point and the
same D numerator as the full exact scan.
"""

from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import _binding as P
from . import synth as S


def _labels_from(res) -> np.ndarray:
    sig = (res["flags"] & P.KS_SIGNIFICANT) != 0
    return np.where(sig, res["cp"].astype(np.int32), -1).astype(np.int32)


def generate(ctx, recipe: int, num_series: int, first_series: int = 0, chunk: int = 2048,
             alpha: float = 0.05, seed: int | None = None):
    """Device features [rows*9] (float32), host desc (aux_offset = feature row), labels, full-scan results."""
    import torch

    feats, descs, labels, results = [], [], [], []
    row0 = 0
    prm = P.ks_params_init(alpha)
    for c0 in range(0, num_series, chunk):
        n = min(chunk, num_series - c0)
        b = S.make_batch(recipe, num_series=n, first_series=first_series + c0, seed=seed)
        buf = torch.empty(b.total_elems, dtype=torch.int32, device="cuda")
        S.fill_device(b, buf.data_ptr(), b.total_elems)
        d = P.make_desc(b.specs["offset"], b.specs["K"], b.specs["N"])
        prm.max_K = int(d["K"].max())
        d_dev = P.to_device(d)
        out = P.empty_results(n)
        P.ks_scan_batch(ctx, buf, d_dev, n, prm, out)
        rows = int(d["K"].astype(np.int64).sum())
        f = torch.empty(rows * 9, dtype=torch.float32, device="cuda")
        P.ks_features(ctx, buf, d_dev, n, prm.max_K, f)
        res = P.results_to_numpy(out)
        feats.append(f)
        dd = d.copy()
        dd["aux_offset"] += row0
        descs.append(dd)
        labels.append(_labels_from(res))
        results.append(res)
        row0 += rows
        del buf
    torch.cuda.synchronize()
    return torch.cat(feats), np.concatenate(descs), np.concatenate(labels), np.concatenate(results)


def train(ctx, model, feats, desc, labels, epochs: int, batch: int, lr: float, seed: int = 0,
          log=print) -> list[float]:
    import torch

    rng = np.random.default_rng(seed)
    idx = np.nonzero(labels >= 1)[0]
    max_K = int(desc["K"].max())
    losses = []
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    for ep in range(epochs):
        perm = rng.permutation(idx)
        t0 = time.perf_counter()
        acc = []
        for b0 in range(0, len(perm) - batch + 1, batch):
            sel = np.sort(perm[b0:b0 + batch])
            d_dev = P.to_device(desc[sel])
            lab = torch.from_numpy(labels[sel]).to("cuda")
            P.ks_train_step(ctx, model, feats, d_dev, lab, len(sel), max_K, lr, loss)
            acc.append(loss.clone())
        torch.cuda.synchronize()
        ep_loss = float(torch.cat(acc).mean()) if acc else float("nan")
        losses.append(ep_loss)
        log(f"epoch {ep}: loss {ep_loss:.4f} ({len(acc)} steps, {time.perf_counter() - t0:.1f} s)")
    return losses


def trivial_proposal(feats_host: np.ndarray, desc: np.ndarray) -> np.ndarray:
    """Baseline without the network: the row after the largest jump of the per-row median (decile 5),
    on the host (ks_propose with no model computes the same on the device)."""
    out = np.zeros(len(desc), np.int32)
    for s, dd in enumerate(desc):
        a, K = int(dd["aux_offset"]), int(dd["K"])
        med = feats_host[a:a + K, 4].astype(np.float64)
        out[s] = 1 + int(np.argmax(np.abs(np.diff(med))))
    return out


def evaluate(ctx, model, recipe: int, num_series: int, first_series: int, w: int = 8, chunk: int = 2048,
             seed: int | None = None) -> dict:
    """Per series: agreement of the tau = 0 refine (learned and trivial proposals) with the full scan,
    and the learned confidence."""
    import torch

    prm = P.ks_params_init(0.05)
    prm.w = w
    agree, agree_triv, conf_all = [], [], []
    for c0 in range(0, num_series, chunk):
        n = min(chunk, num_series - c0)
        b = S.make_batch(recipe, num_series=n, first_series=first_series + c0, seed=seed)
        buf = torch.empty(b.total_elems, dtype=torch.int32, device="cuda")
        S.fill_device(b, buf.data_ptr(), b.total_elems)
        d = P.make_desc(b.specs["offset"], b.specs["K"], b.specs["N"])
        prm.max_K = int(d["K"].max())
        d_dev = P.to_device(d)
        full = P.empty_results(n)
        P.ks_scan_batch(ctx, buf, d_dev, n, prm, full)
        rows = int(d["K"].astype(np.int64).sum())
        f = torch.empty(rows * 9, dtype=torch.float32, device="cuda")
        prop = torch.empty(n, dtype=torch.int32, device="cuda")
        conf = torch.empty(n, dtype=torch.float32, device="cuda")
        P.ks_propose(ctx, model, buf, d_dev, n, prm, prop, conf, f)
        ref = P.empty_results(n)
        prm.tau = 0.0
        P.ks_refine(ctx, d_dev, n, b.total_elems, prop, conf, prm, ref)
        # the method without the network (ks_propose with no model), refined the same way
        tp = torch.empty(n, dtype=torch.int32, device="cuda")
        tc = torch.empty(n, dtype=torch.float32, device="cuda")
        P.ks_propose(ctx, None, buf, d_dev, n, prm, tp, tc)
        ref_t = P.empty_results(n)
        P.ks_refine(ctx, d_dev, n, b.total_elems, tp, tc, prm, ref_t)
        g, r, rt = P.results_to_numpy(full), P.results_to_numpy(ref), P.results_to_numpy(ref_t)
        agree.append((g["cp"] == r["cp"]) & (g["U"] == r["U"]))
        agree_triv.append((g["cp"] == rt["cp"]) & (g["U"] == rt["U"]))
        conf_all.append(conf.cpu().numpy())
        del buf
    return {"agree": np.concatenate(agree), "agree_trivial": np.concatenate(agree_triv),
            "confidence": np.concatenate(conf_all)}


def calibrate_tau(agree: np.ndarray, conf: np.ndarray, target: float = 0.995) -> tuple[float, float, float]:
    """Smallest tau (among the observed confidences, plus 0) whose agreement (series with
    confidence < tau fall back and agree) reaches target: (tau, agreement, fallback rate)."""
    n = len(agree)
    order = np.argsort(conf)
    c = conf[order]
    a = agree[order]
    # tau = c[k]: series 0..k-1 fall back
    bad_from = np.cumsum(~a[::-1])[::-1]  # disagreements among series k..n-1
    for k in range(n + 1):
        if 0 < k < n and c[k] == c[k - 1]:
            continue  # tau = c[k] would not make the tied series at k-1 fall back
        bad = bad_from[k] if k < n else 0
        if 1.0 - bad / n >= target:
            tau = float(c[k]) if k < n else float(np.nextafter(np.float32(c[-1]), np.float32(2.0)))
            # ties: every series with confidence < tau falls back
            fb = float(np.mean(conf < tau))
            agr = 1.0 - float(np.sum(~agree & (conf >= tau))) / n
            return tau, agr, fb
    return 1.0, 1.0, 1.0


def recalibrate(args) -> int:
    """Calibrate tau of a trained model again, on held-out series of its recipe
    (ids from --first-series on, disjoint from its training and validation
    series and from the benchmark batches), at --target; the model's report gets
    the new tau and a "calibration" record."""
    import os

    ctx = P.Context(0)
    model = P.Model(ctx, seed=0)
    P.ks_model_load(model.handle, args.model)
    t0 = time.perf_counter()
    ev = evaluate(ctx.handle, model.handle, args.recipe, args.series, args.first_series, chunk=args.chunk)
    tau, agr, fb = calibrate_tau(ev["agree"], ev["confidence"], args.target)
    rep_path = os.path.splitext(args.model)[0] + ".json"
    with open(rep_path) as f:
        rep = json.load(f)
    rep_path = args.report or rep_path  # where the updated report goes
    rep["tau"] = tau
    rep["calibration"] = {"recipe": args.recipe, "first_series": args.first_series, "series": args.series,
                          "target": args.target, "agreement_at_tau": agr, "fallback_at_tau": fb,
                          "agreement_no_fallback": float(ev["agree"].mean()),
                          "agreement_trivial_no_fallback": float(ev["agree_trivial"].mean()),
                          "seconds": time.perf_counter() - t0,
                          "command": "python -m paper_2511_05958_amd.train --calibrate " + " ".join(
                              f"--{k.replace('_', '-')} {v}" for k, v in
                              [("model", os.path.basename(args.model)), ("recipe", args.recipe),
                               ("first_series", args.first_series), ("series", args.series),
                               ("target", args.target), ("chunk", args.chunk)])}
    with open(rep_path, "w") as f:
        json.dump(rep, f, indent=1)
    print(json.dumps(rep["calibration"] | {"tau": tau}), flush=True)
    model.close()
    ctx.close()
    return 0


def main() -> int:
    import torch

    ap = argparse.ArgumentParser()
    ap.add_argument("--series", type=int, default=200_000)
    ap.add_argument("--val", type=int, default=10_000)
    ap.add_argument("--epochs", type=int, default=10)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--target", type=float, default=0.995)
    ap.add_argument("--out", default="proposal.ckpt")
    ap.add_argument("--report", default=None)
    ap.add_argument("--recipe", type=int, default=4, help="training recipe (4: recipe-2 shapes, own seed; 5: hard regime)")
    ap.add_argument("--first-series", type=int, default=0, help="first series id of the training data")
    ap.add_argument("--chunk", type=int, default=2048, help="series generated per device chunk")
    ap.add_argument("--calibrate", action="store_true",
                    help="only calibrate tau of --model on --series held-out series from --first-series on")
    ap.add_argument("--model", default=None, help="trained model (with --calibrate)")
    args = ap.parse_args()
    if args.calibrate:
        return recalibrate(args)
    ctx = P.Context(0)
    model = P.Model(ctx, seed=args.seed)
    t0 = time.perf_counter()
    ntrain = args.series - args.val
    feats, desc, labels, _ = generate(ctx.handle, args.recipe, ntrain, args.first_series, chunk=args.chunk)
    print(f"generated {ntrain} training series ({int((labels >= 1).sum())} significant) in "
          f"{time.perf_counter() - t0:.1f} s", flush=True)
    t1 = time.perf_counter()
    losses = train(ctx.handle, model.handle, feats, desc, labels, args.epochs, args.batch, args.lr, args.seed,
                   log=lambda m: print(m, flush=True))
    train_s = time.perf_counter() - t1
    del feats
    torch.cuda.empty_cache()
    ev = evaluate(ctx.handle, model.handle, args.recipe, args.val, args.first_series + ntrain, chunk=args.chunk)
    tau, agr, fb = calibrate_tau(ev["agree"], ev["confidence"], args.target)
    P.ks_model_save(model.handle, args.out)
    rep = {"recipe": args.recipe, "first_series": args.first_series, "train_series": ntrain, "val_series": args.val,
           "epochs": args.epochs, "batch": args.batch,
           "lr": args.lr, "losses": losses, "train_seconds": train_s,
           "val_agreement_no_fallback": float(ev["agree"].mean()),
           "val_agreement_trivial_no_fallback": float(ev["agree_trivial"].mean()),
           "tau": tau, "val_agreement_at_tau": agr, "val_fallback_at_tau": fb, "target": args.target}
    print(json.dumps(rep), flush=True)
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)
    model.close()
    ctx.close()
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
