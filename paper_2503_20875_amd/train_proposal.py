"""Train the period-window proposal network on method-generated data.

Synthetic light curves of the learned-proposal workload (80 000 points at
2-min cadence, half with one injected planet) go through the library's own
linear search on the GPU; the downsampled single-event statistics are the
inputs and the windows within 2% of the injected period (and of its half
and double, the aliases a fold can prefer) are the labels.  Training runs the library's
forward, backward and Adam kernels.  The weights are written as a NumPy
archive together with the settings they were trained with.

    python -m paper_2503_20875_amd.train_proposal --n-train 4000 --epochs 20 --out weights.npz
"""

from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def log(msg: str) -> None:
    print(f"[train] {msg}", flush=True)


# Duration rows the network reads on the long-baseline grid (16 of its 30).
LONG_FEATURE_ROWS = (0, 2, 4, 6, 8, 10, 12, 14, 15, 17, 19, 21, 23, 25, 27, 29)


def make_pipeline(cfg=None, workload: str = "learned"):
    """Search pipeline of the learned-proposal workload (80 000 points at
    120 s, periods 1-100 d) or of the long-baseline workload (2.5 M points
    at 25 s, periods 1-400 d, 16 of its 30 durations as network input)."""
    from synthlc import transit
    from synthlc import workloads as W
    from .learned import LearnedConfig, Pipeline
    if workload == "long":
        sh = W.long_baseline_shape()
        return Pipeline(0.0, sh["span"], sh["cadence"], sh["durations"], sh["periods"], transit.dense_template(),
                        cfg or LearnedConfig(p_lo=1.0, p_hi=400.0, feature_rows=LONG_FEATURE_ROWS))
    durations, periods = W.learned_grid()
    cad = 120.0 / 86400.0
    return Pipeline(0.0, (W.LEARNED_N_POINTS - 1) * cad, cad, durations, periods, transit.dense_template(),
                    cfg or LearnedConfig())


def curve_source(workload: str, seed: int, device_gen: bool = True):
    """A callable returning one (t, f, sigma, injections) curve per call:
    generated on the device (LongCurves, LearnedCurves), or for the learned
    workload with device_gen=False on the host (learned_curve)."""
    from synthlc import workloads as W
    if workload == "long":
        return W.LongCurves(seed).draw
    if device_gen:
        return W.LearnedCurves(seed).draw
    rng = np.random.default_rng(seed)
    return lambda: W.learned_curve(rng)


LABEL_BAND = 0.02  # relative half-width of the labelled period band


def labels_for(pipe, injections) -> np.ndarray:
    """Multi-hot window labels: every window overlapping [P (1 - band),
    P (1 + band)] for the injected period P, its half and its double (the
    aliases a fold may prefer).  The band covers the period scatter of
    planets with only a few transits in the span."""
    y = np.zeros(pipe.windows.n, dtype=np.float32)
    for inj in injections:
        for mult in (1.0, 0.5, 2.0):
            P = inj.period * mult
            lo = np.searchsorted(pipe.windows.edges, P * (1 - LABEL_BAND), side="right") - 1
            hi = np.searchsorted(pipe.windows.edges, P * (1 + LABEL_BAND), side="right") - 1
            lo, hi = max(lo, 0), min(hi, pipe.windows.n - 1)
            if lo <= hi:
                y[lo:hi + 1] = 1.0
    return y


def build_dataset(pipe, n: int, seed: int, workload: str = "learned", plain_labels: bool = False,
                  snr_min: float = 7.0, signed: bool = False):
    """Device features [n][n_bins][16] (bf16) and labels [n][W], plus the
    injections of every curve.  With plain_labels the full periodic search
    also runs on every curve and its best period's window is marked when its
    SNR reaches snr_min, whether or not a planet caused it: the network then
    learns where the full search will report its detection, noise peaks at
    the threshold included."""
    import torch
    from .proposal import C_IN
    draw = curve_source(workload, seed)
    x = torch.empty((n, pipe.cfg.n_bins, C_IN), dtype=torch.bfloat16, device="cuda")
    y = np.zeros((n, pipe.windows.n), dtype=np.float32)
    injs = []
    t0 = time.time()
    for i in range(n):
        t, f, s, inj = draw()
        fold = pipe.linear(torch.as_tensor(t, device="cuda"), torch.as_tensor(f, device="cuda"),
                           torch.as_tensor(s, device="cuda"))
        pipe.features(fold, out=x[i], signed=signed)
        y[i] = labels_for(pipe, inj)
        if plain_labels:
            rec = pipe.plain(fold)
            if rec["k"] >= 0 and rec["snr"] >= snr_min:
                w = pipe.window_of(rec["period"])
                if w >= 0:
                    y[i, w] = 1.0
        injs.append(inj)
        if (i + 1) % 500 == 0:
            log(f"features {i + 1}/{n} ({time.time() - t0:.1f} s)")
    torch.cuda.synchronize()
    return x, torch.as_tensor(y, device="cuda"), injs


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n-train", type=int, default=4000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--pos-weight", type=float, default=32.0)
    ap.add_argument("--seed", type=int, default=20250401)
    ap.add_argument("--n-trial", type=int, default=4)
    ap.add_argument("--workload", default="learned", choices=["learned", "long"])
    ap.add_argument("--plain-labels", action="store_true",
                    help="also label each curve's full-search best window when its SNR is at least 7")
    ap.add_argument("--signed-input", action="store_true",
                    help="network input: the binned signed single-event SNR instead of its absolute value")
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)

    import torch
    if not torch.cuda.is_available():
        print("train_proposal: no GPU", file=sys.stderr)
        return 2
    from .learned import save_weights, train
    from .proposal import ProposalNet
    pipe = make_pipeline(workload=a.workload)
    log(f"grid I={pipe.grid.n_t0} J={pipe.grid.n_dur} K={pipe.K} windows={pipe.windows.n} "
        f"bin {pipe.windows.bin_days:.5f} d")
    x, y, _ = build_dataset(pipe, a.n_train, a.seed, a.workload, plain_labels=a.plain_labels,
                            signed=a.signed_input)
    log(f"labelled windows per curve {float(y.sum()) / a.n_train:.3f}")
    net = ProposalNet(n_event=pipe.cfg.n_event, hidden=pipe.cfg.hidden, seed=a.seed, n_trial=a.n_trial)
    net.signed_input = bool(a.signed_input)
    losses = train(net, x, y, pipe.windows, a.epochs, a.batch, a.lr, a.pos_weight, seed=a.seed, log=log)
    meta = dict(n_event=net.E, hidden=net.H, pool="fold", n_trial=net.S, workload=a.workload,
                plain_labels=bool(a.plain_labels), input="signed" if a.signed_input else "abs",
                feature_rows=list(pipe.cfg.feature_rows), n_train=a.n_train, epochs=a.epochs,
                batch=a.batch, lr=a.lr,
                pos_weight=a.pos_weight, seed=a.seed, losses=losses, n_bins=pipe.cfg.n_bins,
                n_windows=pipe.cfg.n_windows, p_lo=pipe.cfg.p_lo, p_hi=pipe.cfg.p_hi)
    save_weights(net, a.out, meta)
    log(f"wrote {a.out}: {json.dumps({k: v for k, v in meta.items() if k != 'losses'})}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
