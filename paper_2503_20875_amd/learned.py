"""Learned proposal around the plain search: features, training, proposal.

The single-event statistics of the linear search (Sec. 2.2) are turned into
network inputs on the device (cetra_net_downsample: per duration, the
maximum single-event SNR in each of n_bins time bins), the proposal network
scores log-spaced period windows, and the periodic search (Sec. 2.3) runs
on the periods of the top-K windows only.  The plain search over every
period stays available and is what the proposal's recall is measured
against.
"""

from __future__ import annotations

import io
import json
import time
from dataclasses import dataclass

import numpy as np

from . import best, best_record, grid_plan, linear_search, periodic_search, periodic_workspace, resample, \
    template_resample
from .proposal import C_IN, ProposalNet, Windows, downsample, topk_windows, windows_to_periods


@dataclass
class LearnedConfig:
    n_bins: int = 8192
    n_windows: int = 512
    top_k: int = 64
    p_lo: float = 1.0
    p_hi: float = 100.0
    n_event: int = 8
    hidden: int = 64
    feature_rows: tuple = ()  # duration rows read by the network (all when empty)


class Pipeline:
    """Search of light curves that share one time grid (same cadence and
    span), the same durations and the same period grid."""

    def __init__(self, t_first: float, t_last: float, cadence: float, durations, periods, dense,
                 cfg: LearnedConfig = LearnedConfig(), n_model: int = 1024):
        import torch
        rows = cfg.feature_rows or tuple(range(len(durations)))
        if len(rows) != C_IN or max(rows) >= len(durations) or min(rows) < 0:
            raise ValueError(f"the proposal network reads {C_IN} of the durations")
        self.cfg = cfg
        self.grid = grid_plan(t_first, t_last, cadence, durations, 0.0, n_model)
        self.model = template_resample(torch.as_tensor(np.asarray(dense, np.float64), device="cuda"), n_model)
        self.periods_host = np.ascontiguousarray(periods, dtype=np.float64)
        if np.any(np.diff(self.periods_host) <= 0):
            raise ValueError("periods must be ascending")
        self.periods = torch.as_tensor(self.periods_host, device="cuda")
        self.K = int(self.periods.numel())
        bin_days = self.grid.n_t0 * self.grid.t0_step / cfg.n_bins
        self.windows = Windows.log_spaced(cfg.n_windows, cfg.p_lo, cfg.p_hi, bin_days)
        self.work = torch.empty(max(periodic_workspace(self.grid, self.K), 1), dtype=torch.uint8, device="cuda")
        self.per = None
        self.last_scores = None
        self.rows = None if not cfg.feature_rows else torch.as_tensor(list(cfg.feature_rows), device="cuda")

    # ------------------------------------------------------------ features
    def linear(self, t, f, sigma):
        """Resample + linear search: fold-ready [J][I][2] (device).  The
        times must be finite and ascending: this path skips resample's order
        check (status=False) so that it stays free of host synchronisation;
        resample(status=True) or the batched search report unsorted input."""
        flux, ivar, _ = resample(self.grid, t, f, sigma, status=False)
        return linear_search(self.grid, flux, ivar, self.model)

    def features(self, fold, out=None, signed: bool = False):
        """bf16 [n_bins][16] network input from a fold-ready array (its
        feature rows only, when the grid has more durations): the binned
        |SNR|, or the signed SNR for a network trained on it."""
        if self.rows is not None:
            fold = fold.index_select(0, self.rows)
        return downsample(fold, self.cfg.n_bins, out=out, signed=signed)

    # -------------------------------------------------------------- search
    def plain(self, fold):
        """Periodic search over every period; host best record."""
        self.per = periodic_search(self.grid, fold, self.periods, work=self.work, out=self.per)
        return best_record(best(self.grid, self.periods, self.per))

    def propose(self, net: ProposalNet, x):
        """Top-K window indices [B][K] (device) for inputs x [B][n_bins][J]."""
        z = net.forward(x, self.windows)
        return topk_windows(z, self.cfg.top_k)

    def restricted(self, fold, sel):
        """Periodic search over the periods of the selected windows only
        (one curve); host best record and the number of periods folded."""
        subset, n = windows_to_periods(self.periods, self.windows, sel)
        n_sub = int(n.item())
        if n_sub == 0:
            return None, 0
        self.per = periodic_search(self.grid, fold, self.periods, subset=subset[:n_sub], work=self.work,
                                   out=self.per)
        return best_record(best(self.grid, self.periods, self.per)), n_sub

    def search(self, net: ProposalNet, fold, top_k: int = 0, fallback_snr=None):
        """Proposal + restricted search of one curve, with the full-fold
        fallback: when the restricted best is missing or its SNR is below
        `fallback_snr`, the plain search over every period runs and its
        result is returned instead.  Returns (host best record, restricted
        SNR (-inf when nothing was folded), fell back, periods folded).  The
        window scores [1][W] stay in `last_scores`."""
        x = self.features(fold, signed=net.signed_input)
        z = net.forward(x.unsqueeze(0), self.windows)
        self.last_scores = z
        sel = topk_windows(z, int(top_k or self.cfg.top_k))
        rec, n_sub = self.restricted(fold, sel[0])
        snr_r = float(rec["snr"]) if rec is not None and rec["k"] >= 0 else float("-inf")
        if fallback_snr is not None and snr_r < fallback_snr:
            return self.plain(fold), snr_r, True, n_sub + self.K
        return rec, snr_r, False, n_sub

    def search_batch(self, net: ProposalNet, folds, top_k: int = 0):
        """The learned search over a batch of curves: features of every curve,
        one network forward over the batch, the top-K windows per curve, then
        the restricted periodic searches back to back.  `folds` are the
        curves' fold-ready arrays (this pipeline's grid).  Returns per curve
        (host best record or None, periods folded)."""
        import torch
        from .proposal import C_IN
        x = torch.empty((len(folds), self.cfg.n_bins, C_IN), dtype=torch.bfloat16, device="cuda")
        for b, fold in enumerate(folds):
            self.features(fold, out=x[b], signed=net.signed_input)
        z = net.forward(x, self.windows)
        self.last_scores = z
        sel = topk_windows(z, int(top_k or self.cfg.top_k))
        return [self.restricted(fold, sel[b]) for b, fold in enumerate(folds)]

    def window_of(self, period: float) -> int:
        w = int(np.searchsorted(self.windows.edges, period, side="right") - 1)
        return w if 0 <= w < self.windows.n else -1


# ------------------------------------------------------------------ training
def train(net: ProposalNet, x, y, windows: Windows, epochs: int, batch: int = 32, lr: float = 1e-3,
          pos_weight: float = 32.0, seed: int = 0, log=None):
    """Adam on (x [N][n_bins][J] bf16, y [N][W] FP32) device tensors, in
    shuffled mini-batches; returns the per-epoch mean losses."""
    import torch
    N = int(x.shape[0])
    g = torch.Generator(device="cpu").manual_seed(seed)
    losses = []
    for ep in range(epochs):
        perm = torch.randperm(N, generator=g).to(x.device)
        tot, nb, t0 = torch.zeros((), device=x.device), 0, time.time()
        for s in range(0, N - batch + 1, batch):
            idx = perm[s:s + batch]
            net.forward(x.index_select(0, idx), windows)
            tot += net.backward(y.index_select(0, idx), pos_weight=pos_weight)[0]
            net.adam(lr=lr)
            nb += 1
        losses.append(float(tot.item()) / max(nb, 1))
        if log:
            log(f"epoch {ep} loss {losses[-1]:.5f} ({time.time() - t0:.1f} s)")
    return losses


def save_weights(net: ProposalNet, path: str, meta: dict) -> None:
    """Parameters (FP32) and metadata in a NumPy archive (no pickled objects)."""
    arrays = {name: net.view(name).cpu().numpy() for name in net.offsets}
    arrays["__meta__"] = np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8)
    with open(path, "wb") as fh:
        np.savez(fh, **arrays)


def store_calibration(path: str, k: int, fallback_snr, note: str) -> None:
    """Record calibrated operating points in a weights archive's metadata:
    the K whose top-K windows held the target share of a calibration set's
    plain detections, and the full-fold fallback threshold at K = 64."""
    with np.load(path, allow_pickle=False) as z:
        arrays = {name: z[name] for name in z.files if name != "__meta__"}
        meta = json.loads(bytes(z["__meta__"]).decode())
    meta.update(calibrated_k=int(k), calibrated_fallback_snr=None if fallback_snr is None else float(fallback_snr),
                calibration=note)
    arrays["__meta__"] = np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8)
    with open(path, "wb") as fh:
        np.savez(fh, **arrays)


def load_weights(path: str) -> tuple:
    with np.load(path, allow_pickle=False) as z:
        meta = json.loads(bytes(z["__meta__"]).decode())
        if meta.get("pool", "fold") != "fold":
            raise ValueError(f"{path}: weights of an unsupported pooling ({meta.get('pool')})")
        net = ProposalNet(n_event=meta["n_event"], hidden=meta["hidden"], n_trial=meta.get("n_trial", 4))
        net.signed_input = meta.get("input", "abs") == "signed"
        import torch
        for name in net.offsets:
            net.view(name).copy_(torch.as_tensor(z[name]))
        net.pack()
    return net, meta


# ---------------------------------------------------------------- evaluation
def evaluate(pipe: Pipeline, net: ProposalNet, curves, snr_min: float = 7.0, top_k: int = 0, fallback_snr=None,
             log=None, plain=None) -> dict:
    """Plain search versus proposal + restricted search on each curve
    (t, f, sigma, injections).  A plain detection is a best period with
    SNR > snr_min; it is recalled when the learned search (restricted search
    over the top_k windows, default the pipeline's, with the full-fold
    fallback below `fallback_snr` when given) returns the same best period.
    Also returned: for every detection, the rank of its window among the
    network's scores (0 = best; ties to the smaller window), so recall at any
    K is the fraction of ranks below K, and per curve the restricted best
    SNR, from which a fallback threshold can be chosen.  Times are device
    times per curve (events on the current stream): the plain periodic search
    + best, and downsample + network + top-K + subset + restricted search +
    best (+ the fallback's full search when it runs).  `plain`, the "plain"
    list of an earlier evaluation of the same curves, reuses its full-search
    records and times."""
    import torch
    top_k = int(top_k or pipe.cfg.top_k)
    n_det = n_hit = n_true = n_true_hit = n_fb = 0
    t_plain = t_learned = 0.0
    n_folded = 0
    rows, ranks, plain_out = [], [], []
    for ci, (t, f, s, injs) in enumerate(curves):
        fold = pipe.linear(torch.as_tensor(t, device="cuda"), torch.as_tensor(f, device="cuda"),
                           torch.as_tensor(s, device="cuda"))
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        if plain is None:
            e[0].record()
            bp = pipe.plain(fold)
            e[1].record()
        e[2].record()
        bl, snr_r, fell_back, n_sub = pipe.search(net, fold, top_k, fallback_snr)
        e[3].record()
        torch.cuda.synchronize()
        z = pipe.last_scores
        if plain is None:
            ms_plain = e[0].elapsed_time(e[1])
        else:
            bp, ms_plain = plain[ci]
        plain_out.append((bp, ms_plain))
        t_plain += ms_plain
        t_learned += e[2].elapsed_time(e[3])
        n_folded += n_sub
        n_fb += fell_back
        det = bool(bp["k"] >= 0 and bp["snr"] > snr_min)
        hit = bool(det and bl is not None and bl["k"] == bp["k"])
        # the paper's recovery criterion: within 1% of P, P/2 or 2P
        true = bool(det and any(abs(bp["period"] / (i.period * m) - 1.0) < 0.01
                                for i in injs for m in (1.0, 0.5, 2.0)))
        n_true += true
        n_true_hit += true and hit
        rank = -1
        if det:
            zs = z[0].float().cpu().numpy()
            w = pipe.window_of(float(bp["period"]))
            rank = int(np.count_nonzero(zs > zs[w]) + np.count_nonzero(zs[:w] == zs[w])) if w >= 0 else pipe.windows.n
            ranks.append(rank)
        n_det += det
        n_hit += hit
        rows.append(dict(curve=ci, plain_k=int(bp["k"]), plain_period=float(bp["period"]), plain_snr=float(bp["snr"]),
                         learned_k=-1 if bl is None else int(bl["k"]), restricted_snr=snr_r, fell_back=fell_back,
                         detected=det, recalled=hit, rank=rank, true_detection=true,
                         injected=[float(i.period) for i in injs]))
        if log and (ci + 1) % 16 == 0:
            log(f"eval {ci + 1}/{len(curves)}: detections {n_det}, recalled {n_hit}")
    n = max(len(curves), 1)
    return dict(n_curves=len(curves), top_k=top_k, fallback_snr=fallback_snr, n_detections=n_det, n_recalled=n_hit,
                recall=(n_hit / n_det) if n_det else None, n_true_detections=n_true,
                recall_true=(n_true_hit / n_true) if n_true else None, plain_ms_per_curve=t_plain / n,
                learned_ms_per_curve=t_learned / n, speedup=(t_plain / t_learned) if t_learned > 0 else None,
                fallback_fraction=n_fb / n, periods_folded_fraction=n_folded / (n * pipe.K), ranks=ranks, rows=rows,
                plain=plain_out)


def fallback_threshold(rows, target: float) -> float:
    """Smallest restricted-SNR threshold for the full-fold fallback at which
    at least `target` of the plain detections in `rows` (evaluated without a
    fallback) are recalled: a missed detection is rescued when its curve's
    restricted best SNR is below the threshold.  -inf when the proposal alone
    already reaches the target."""
    det = [r for r in rows if r["detected"]]
    if not det:
        return float("-inf")
    allowed = int(np.floor((1.0 - target) * len(det) + 1e-9))
    miss = sorted((r["restricted_snr"] for r in det if not r["recalled"]), reverse=True)
    if len(miss) <= allowed:
        return float("-inf")
    # rescue every miss except the `allowed` ones with the highest restricted SNR
    return float(np.nextafter(miss[allowed], np.inf))


def k_for_recall(ranks, target: float, n_windows: int) -> int:
    """Smallest K whose top-K windows hold at least `target` of the
    detections' windows (n_windows if none does)."""
    if not ranks:
        return 1
    r = np.sort(np.asarray(ranks))
    need = int(np.ceil(target * len(r)))
    return int(min(n_windows, r[need - 1] + 1))
