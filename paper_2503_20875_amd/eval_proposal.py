"""Evaluate a trained period-window proposal against the plain periodic
search on held-out curves of the learned-proposal workload.

The first half of the curves (calibration, run at K = 64 windows without a
fallback) fixes two operating points that keep `target` of the plain
detections above SNR 7: the smallest number of windows K whose top-K holds
them, and the smallest restricted-SNR threshold of the full-fold fallback at
K = 64.  The second half (test) runs K = 64 alone, the calibrated K, and
K = 64 with the calibrated fallback, and reports recall (over all plain
detections and over those of injected planets) and the device-time speedup
over the full periodic search, fallback runs included.

    python -m paper_2503_20875_amd.eval_proposal --weights weights/proposal.npz --n 1000 --out eval.json
"""

from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np


def log(msg: str) -> None:
    print(f"[eval] {msg}", flush=True)


def summary(r: dict) -> dict:
    keys = ("top_k", "fallback_snr", "n_detections", "n_recalled", "recall", "n_true_detections", "recall_true",
            "plain_ms_per_curve", "learned_ms_per_curve", "speedup", "periods_folded_fraction", "fallback_fraction")
    return {k: r[k] for k in keys}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    here = os.path.dirname(os.path.abspath(__file__))
    ap.add_argument("--weights", default=os.path.join(here, "weights", "proposal.npz"),
                    help="weights file, or a comma-separated list evaluated on the same curves")
    ap.add_argument("--n", type=int, default=1000, help="held-out curves (half calibration, half test)")
    ap.add_argument("--target", type=float, default=0.99)
    ap.add_argument("--seed", type=int, default=20250410)
    ap.add_argument("--out", default="")
    ap.add_argument("--quick", action="store_true",
                    help="rank recall only: one K = 64 run per half, no operating-point runs")
    ap.add_argument("--store-calibration", action="store_true",
                    help="write the calibration half's operating points into the (single) weights file")
    ap.add_argument("--rows", action="store_true",
                    help="also write every detection of the test half (rank, periods, SNR, truth)")
    a = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        print("eval_proposal: no GPU", file=sys.stderr)
        return 2
    from .learned import evaluate, fallback_threshold, k_for_recall, load_weights
    from .train_proposal import curve_source, make_pipeline
    paths = [w for w in a.weights.split(",") if w]
    nets = [load_weights(w) for w in paths]
    workload = nets[0][1].get("workload", "learned")
    pipe = make_pipeline(workload=workload)
    n_cal = a.n // 2
    draw_cal, draw_test = curve_source(workload, a.seed), curve_source(workload, a.seed + 1)
    cal_curves = [draw_cal() for _ in range(n_cal)]
    test_curves = [draw_test() for _ in range(a.n - n_cal)]
    results = {}
    plain_cal = plain_test = None  # the full searches run once, for the first network
    for path, (net, meta) in zip(paths, nets):
        log(f"network {path}")
        cal = evaluate(pipe, net, cal_curves, log=log, plain=plain_cal)
        plain_cal = cal["plain"]
        k_target = k_for_recall(cal["ranks"], a.target, pipe.windows.n)
        tau = fallback_threshold(cal["rows"], a.target)
        log(f"calibration: {cal['n_detections']} detections, recall at K=64 {cal['recall']:.3f}; "
            f"K for target {k_target}, fallback threshold {tau:.3f}")
        out = {"calibration": {"k64": summary(cal), "k_for_target": k_target,
                               "fallback_snr_for_target": tau if np.isfinite(tau) else None,
                               "rank_recall": {K: float(np.mean(np.asarray(cal["ranks"]) < K))
                                               for K in (16, 32, 64, 96, 128, 192, 256, 384)}},
               "trained_on": {k: meta.get(k) for k in ("n_train", "epochs", "batch", "lr", "seed")}}
        test_k64 = evaluate(pipe, net, test_curves, top_k=64, log=log, plain=plain_test)
        plain_test = test_k64["plain"]
        out["test_k64"] = summary(test_k64)
        out["test_rank_recall"] = {K: float(np.mean(np.asarray(test_k64["ranks"]) < K))
                                   for K in (16, 32, 64, 96, 128, 192, 256, 384)}
        if a.rows:
            out["test_detections"] = [{k: r[k] for k in ("curve", "rank", "plain_period", "plain_snr",
                                                         "true_detection", "injected")}
                                      for r in test_k64["rows"] if r["detected"]]
        if a.quick:
            results[os.path.basename(path)] = out
            continue
        out["test_k_target"] = summary(evaluate(pipe, net, test_curves, top_k=k_target, log=log, plain=plain_test))
        out["test_k96"] = summary(evaluate(pipe, net, test_curves, top_k=96, log=log, plain=plain_test))
        out["test_fallback"] = summary(evaluate(pipe, net, test_curves, top_k=64,
                                                fallback_snr=tau if np.isfinite(tau) else None, log=log,
                                                plain=plain_test))
        results[os.path.basename(path)] = out
        if a.store_calibration:
            from .learned import store_calibration
            store_calibration(path, k_target, tau if np.isfinite(tau) else None,
                              f"eval_proposal --n {a.n} --seed {a.seed}: calibration half of {n_cal} curves, "
                              f"{cal['n_detections']} plain detections above SNR 7, target {a.target}")
    out = {"n_curves": a.n, "seed": a.seed, "workload": workload, "target_recall": a.target, "networks": results}
    text = json.dumps(out)
    print(text, flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
