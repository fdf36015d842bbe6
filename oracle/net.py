"""FP64 oracle of the period-window proposal network -- TEST INFRASTRUCTURE ONLY.

The proposal network is not part of the paper; it ranks period windows from
the linear search's single-event statistics so that the periodic search
(Sec. 2.3) folds only the best-ranked windows.  This module is the plain
numpy definition (forward and hand-derived backward, FP64) the GPU kernels
are checked against; its gradients are pinned by central finite differences
in the tests.

Architecture (B examples, C_in input channels = durations, L bins):
  x [B, C_in, L]                        downsampled single-event features
  h_l = relu(conv1d(h_{l-1}, W_l) + b_l), l = 1..5, kernel 9, zero padding 4,
        64 channels                      (trunk)
  e = P h_5 + p                          linear 1x1 projection to E channels
  per window w, trial period T (bins) and phase phi:
        F = sum_k e_c[phi + round(k T)] / sqrt(#k)      fold pooling, the
        nearest-epoch rule of the periodic search at bin resolution
        g[w, c] = F at the window's best (trial, phase), chosen on F in
        FP32 (the kernel's precision; see score32)
  f[w] = [g[w, :], q_w]                  q_w = window position in [0, 1]
  z[w] = v . relu(U f[w] + u) + v0       shared head -> one logit per window
  loss = mean_{b,w} pos_w(y) * bce(z, y),  pos weight for the positives
"""

from __future__ import annotations

import numpy as np

K_CONV = 9
PAD = 4


def init_params(c_in: int = 16, width: int = 64, n_layers: int = 5, n_event: int = 8, hidden: int = 64,
                seed: int = 0) -> dict:
    """He-style initialisation (FP64)."""
    rng = np.random.default_rng(seed)
    p = {}
    ch = c_in
    for l in range(n_layers):
        fan_in = ch * K_CONV
        p[f"W{l}"] = rng.normal(0, np.sqrt(2.0 / fan_in), (width, ch, K_CONV))
        p[f"b{l}"] = np.zeros(width)
        ch = width
    p["P"] = rng.normal(0, np.sqrt(2.0 / width), (n_event, width))
    p["p"] = np.full(n_event, 0.01)
    n_feat = n_event + 1
    p["U"] = rng.normal(0, np.sqrt(2.0 / n_feat), (hidden, n_feat))
    p["u"] = np.zeros(hidden)
    p["v"] = rng.normal(0, np.sqrt(1.0 / hidden), hidden)
    p["v0"] = np.array([-2.0])
    return p


def n_params(p: dict) -> int:
    return int(sum(np.asarray(v).size for v in p.values()))


def conv1d(x, W, b):
    """'Same' 1-D convolution (cross-correlation) with zero padding 4."""
    B, C, L = x.shape
    O = W.shape[0]
    xp = np.zeros((B, C, L + 2 * PAD))
    xp[:, :, PAD:PAD + L] = x
    y = np.zeros((B, O, L))
    for k in range(K_CONV):
        y += np.einsum("oc,bcl->bol", W[:, :, k], xp[:, :, k:k + L])
    return y + b[None, :, None]


def conv1d_backward(x, W, gy):
    """Gradients of conv1d with respect to x, W, b given dL/dy."""
    B, C, L = x.shape
    xp = np.zeros((B, C, L + 2 * PAD))
    xp[:, :, PAD:PAD + L] = x
    gW = np.zeros_like(W)
    gxp = np.zeros_like(xp)
    for k in range(K_CONV):
        gW[:, :, k] = np.einsum("bol,bcl->oc", gy, xp[:, :, k:k + L])
        gxp[:, :, k:k + L] += np.einsum("oc,bol->bcl", W[:, :, k], gy)
    return gxp[:, :, PAD:PAD + L], gW, gy.sum(axis=(0, 2))


def fold_trials(edges, n_trial: int, bin_days: float):
    """Trial periods (in bins) of every window: n_trial log-spaced points at
    the centres of n_trial equal log-steps of [edges[w], edges[w+1])."""
    edges = np.asarray(edges, dtype=np.float64)
    frac = (np.arange(n_trial) + 0.5) / n_trial
    return edges[:-1, None] * (edges[1:, None] / edges[:-1, None]) ** frac[None, :] / bin_days


def fold_step(T: float) -> int:
    """32.32 fixed-point step of a trial period of T bins (round half up)."""
    return int(np.floor(4294967296.0 * float(T) + 0.5))


def score32(s, n):
    """The FP32 score on which fold pooling decides a window's winner:
    fl32(fl32(s) * fl32(1 / sqrt(n))), the reciprocal square root rounded
    once from FP64 (numpy's float32 arithmetic is IEEE, correctly rounded)."""
    r = np.float32(1.0 / np.sqrt(np.float64(n)))
    return np.asarray(s, dtype=np.float64).astype(np.float32) * r


def fold_pool(e, trials, runner_up: bool = False):
    """Coarse fold of each event series at every trial period.  For trial T
    (bins) with fixed-point step R, phase phi in [0, min(L, ceil(R/2^32)))
    sums e over the transit positions phi + ((k R + 2^31) >> 32), k = 0, 1,
    ..., inside the series; the score is that sum over sqrt(number of
    terms).  Per window: the (trial, phase) of the maximum score (ties: the
    first trial, then the smallest phase), the decision taken on the FP32
    score of score32 (the kernel's precision); the feature is that winner's
    score in FP64.  Returns g [B][W][E] and the winning (trial, phase)
    [B][W][E][2]; with runner_up, also the best FP64 score of any other
    (trial, phase) [B][W][E] (to check that a test's maxima are
    unambiguous)."""
    B, E, L = e.shape
    W, S = trials.shape
    g = np.zeros((B, W, E))
    second = np.full((B, W, E), -np.inf)
    arg = np.zeros((B, W, E, 2), dtype=np.int64)
    for w in range(W):
        best = np.full((B, E), -np.inf)
        best32 = np.full((B, E), -np.inf, dtype=np.float32)
        sec = np.full((B, E), -np.inf)
        for s_ in range(S):
            if not (1.0 <= trials[w, s_] < 1e9):
                continue  # a trial shorter than one bin is skipped
            R = fold_step(trials[w, s_])
            n_ph = min(L, -(-R // 4294967296))
            o = []
            k = 0
            while True:
                ok = (k * R + 2147483648) >> 32
                if ok >= L:
                    break
                o.append(ok)
                k += 1
            o = np.array(o, dtype=np.int64)
            for ph in range(n_ph):
                pos = ph + o
                pos = pos[pos < L]
                tot = e[:, :, pos].sum(axis=2)
                sc = tot / np.sqrt(len(pos))
                sc32 = score32(tot, len(pos))
                better = sc32 > best32
                sec = np.where(better, best, np.maximum(sec, sc))
                best = np.where(better, sc, best)
                best32 = np.where(better, sc32, best32)
                arg[:, w, :, 0] = np.where(better, s_, arg[:, w, :, 0])
                arg[:, w, :, 1] = np.where(better, ph, arg[:, w, :, 1])
        g[:, w, :] = np.where(np.isfinite(best), best, 0.0)
        second[:, w, :] = sec
        arg[:, w, :, 0] = np.where(np.isfinite(best), arg[:, w, :, 0], -1)
    return (g, arg, second) if runner_up else (g, arg)


def fold_pool_backward(gg, arg, trials, L):
    """Gradient of the window maxima w.r.t. e: each window's winning phase
    passes gg / sqrt(n) to every one of its transit positions."""
    B, W, E = gg.shape
    ge = np.zeros((B, E, L))
    for b in range(B):
        for w in range(W):
            for c in range(E):
                s_, ph = arg[b, w, c]
                if s_ < 0:
                    continue
                R = fold_step(trials[w, s_])
                pos = []
                k = 0
                while True:
                    x = ph + ((k * R + 2147483648) >> 32)
                    if x >= L:
                        break
                    pos.append(x)
                    k += 1
                ge[b, c, pos] += gg[b, w, c] / np.sqrt(len(pos))
    return ge


def windows_for(n_windows: int, p_lo: float, p_hi: float):
    """Edges of n_windows log-spaced period windows over [p_lo, p_hi] days
    (window w covers [edges[w], edges[w+1])) and each window's position q in
    [0, 1]."""
    edges = p_lo * (p_hi / p_lo) ** (np.arange(n_windows + 1) / n_windows)
    q = (np.arange(n_windows) + 0.5) / n_windows
    return q, edges


def downsample(fold, n_bins: int):
    """Network input from the linear search's fold-ready pairs (reading N1).

    fold: [J, I, 2] (S_fm, S_mm) per duration and reference time.  For
    duration j and bin b, which covers the reference times
    [floor(b I / L), floor((b + 1) I / L)), the feature is the largest
    single-event SNR over the bin, |S_fm| / sqrt(S_mm) = |depth| / sqrt(var)
    (Sec. 2.2; a null element, S_mm = 0, counts as 0), clipped at 30 and
    divided by 8.  Returns [L, J] (bin-major, the network's layout), FP64.
    """
    fold = np.asarray(fold, dtype=np.float64)
    J, I = fold.shape[0], fold.shape[1]
    out = np.zeros((n_bins, J))
    for b in range(n_bins):
        i0, i1 = b * I // n_bins, (b + 1) * I // n_bins
        a = fold[:, i0:i1, 0]
        s = fold[:, i0:i1, 1]
        snr = np.zeros_like(a)
        ok = s > 0
        snr[ok] = np.abs(a[ok]) / np.sqrt(s[ok])
        if i1 > i0:
            out[b] = snr.max(axis=1)
    return np.minimum(out, 30.0) / 8.0


def downsample_signed(fold, n_bins: int):
    """The signed form of the network input: per duration and bin, the
    largest S_fm / sqrt(S_mm) over the bin (the single-event depth over its
    error, keeping the sign, so that a dimming is positive), clipped to
    [-30, 30] and divided by 8; a bin whose elements are all null gives 0.
    Same bins and layout as downsample; FP64."""
    fold = np.asarray(fold, dtype=np.float64)
    J, I = fold.shape[0], fold.shape[1]
    out = np.zeros((n_bins, J))
    for b in range(n_bins):
        i0, i1 = b * I // n_bins, (b + 1) * I // n_bins
        for j in range(J):
            a = fold[j, i0:i1, 0]
            s = fold[j, i0:i1, 1]
            ok = s > 0
            if np.any(ok):
                out[b, j] = np.max(a[ok] / np.sqrt(s[ok]))
    return np.clip(out, -30.0, 30.0) / 8.0


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    a = (a + 0x7FFF + ((a >> 16) & 1)) & 0xFFFF0000
    return a.astype(np.uint32).view(np.float32).astype(np.float64)


def _q(x, on):
    return bf16(x) if on else x


def forward(p: dict, x, win_q, trials, n_layers: int = 5, keep: bool = False, bf16_trunk: bool = False):
    """trials: [W][S] trial periods in bins.  bf16_trunk: round the
    convolution inputs, weights and outputs to bfloat16 (the storage
    precision of the device trunk); the arithmetic stays FP64."""
    trials = np.asarray(trials, dtype=np.float64)
    h = [_q(x, bf16_trunk)]
    for l in range(n_layers):
        y = np.maximum(conv1d(h[-1], _q(p[f"W{l}"], bf16_trunk), p[f"b{l}"]), 0.0)
        h.append(_q(y, bf16_trunk))
    e = np.einsum("ec,bcl->bel", p["P"], h[-1]) + p["p"][None, :, None]
    g, arg = fold_pool(e, trials)
    B, W = g.shape[:2]
    f = np.concatenate([g, np.broadcast_to(np.asarray(win_q)[None, :, None], (B, W, 1))], axis=2)
    pre_r = np.einsum("hf,bwf->bwh", p["U"], f) + p["u"]
    r = np.maximum(pre_r, 0.0)
    z = np.einsum("h,bwh->bw", p["v"], r) + p["v0"][0]
    if not keep:
        return z
    return z, dict(h=h, e=e, arg=arg, f=f, pre_r=pre_r, r=r, bf16_trunk=bf16_trunk, trials=trials)


def bce_loss(z, y, pos_weight: float = 1.0):
    """Mean over (b, w) of the weighted binary cross-entropy with logits."""
    w = np.where(y > 0.5, pos_weight, 1.0)
    l = np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z)))
    loss = np.sum(w * l) / z.size
    gz = w * (1.0 / (1.0 + np.exp(-z)) - y) / z.size
    return loss, gz


def backward(p: dict, cache: dict, gz, n_layers: int = 5) -> dict:
    g = {}
    r, pre_r, f = cache["r"], cache["pre_r"], cache["f"]
    g["v0"] = np.array([gz.sum()])
    g["v"] = np.einsum("bw,bwh->h", gz, r)
    gr = gz[:, :, None] * p["v"][None, None, :]
    gpre_r = gr * (pre_r > 0)
    g["U"] = np.einsum("bwh,bwf->hf", gpre_r, f)
    g["u"] = gpre_r.sum(axis=(0, 1))
    gf = np.einsum("bwh,hf->bwf", gpre_r, p["U"])
    E = p["P"].shape[0]
    L = cache["e"].shape[2]
    ge = fold_pool_backward(gf[:, :, :E], cache["arg"], cache["trials"], L)
    return _trunk_backward(p, g, cache["h"], ge, cache, n_layers)


def _trunk_backward(p, g, h, gpre_e, cache, n_layers):
    g["P"] = np.einsum("bel,bcl->ec", gpre_e, h[-1])
    g["p"] = gpre_e.sum(axis=(0, 2))
    gh = np.einsum("ec,bel->bcl", p["P"], gpre_e)
    rq = cache.get("bf16_trunk", False)
    for l in reversed(range(n_layers)):
        gh = _q(gh * (h[l + 1] > 0), rq)
        cache[f"G{l}"] = gh  # masked gradient entering layer l's convolution
        gx, g[f"W{l}"], g[f"b{l}"] = conv1d_backward(h[l], _q(p[f"W{l}"], rq), gh)
        gh = gx
    g["x"] = gh
    return g
