"""FP64 oracle of the period-window proposal network -- TEST INFRASTRUCTURE ONLY.

The proposal network is not part of the paper; it ranks period windows from
the linear search's single-event likelihood ratios so that the periodic
search (Sec. 2.3) folds only the best-ranked windows.  This module is the
plain numpy definition (forward and hand-derived backward, FP64) the GPU
kernels are checked against; its gradients are pinned by central finite
differences in the tests.

Architecture (B examples, C_in input channels = durations, L bins):
  x [B, C_in, L]                        downsampled single-event features
  h_l = relu(conv1d(h_{l-1}, W_l) + b_l), l = 1..5, kernel 9, zero padding 4,
        64 channels                      (trunk)
  e = relu(P h_5 + p)                    1x1 projection to E event channels
  a_c(tau) = (1/L) sum_t e_c[t] e_c[t + tau]   lag correlation, tau >= 1
  n_c(tau) = (a_c(tau) - mean_tau a_c) / sqrt(var_tau a_c + EPS)
                                         standardised over the computed lags
  per window w (lag range [lo_w, hi_w]):
        g[w, c] = max_tau n_c(tau)   (ties: smallest tau)
        m[w, c] = mean_tau n_c(tau)
  f[w] = [g[w, :], m[w, :], q_w]         q_w = window position in [0, 1]
  z[w] = v . relu(U f[w] + u) + v0       shared head -> one logit per window
  loss = mean_{b,w} pos_w(y) * bce(z, y),  pos weight for the single positive
"""

from __future__ import annotations

import numpy as np

K_CONV = 9
PAD = 4
EPS = 1e-12  # variance floor of the lag standardisation


def init_params(c_in: int = 16, width: int = 64, n_layers: int = 5, n_event: int = 8, hidden: int = 64,
                seed: int = 0, fold: bool = False) -> dict:
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
    n_feat = n_event + 1 if fold else 2 * n_event + 1
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


def lag_correlation(e, lags):
    """a[b, c, i] = (1/L) sum_t e[b,c,t] e[b,c,t+lags[i]]."""
    B, C, L = e.shape
    a = np.zeros((B, C, len(lags)))
    for i, tau in enumerate(lags):
        if tau < L:
            a[:, :, i] = np.sum(e[:, :, :L - tau] * e[:, :, tau:], axis=2) / L
    return a


def standardise(a):
    """Per (example, channel): subtract the mean over the lag axis and divide
    by the standard deviation (population, floored by EPS)."""
    mu = a.mean(axis=2, keepdims=True)
    d = a - mu
    sd = np.sqrt((d * d).mean(axis=2, keepdims=True) + EPS)
    return d / sd, sd


def standardise_backward(gn, n, sd):
    """Gradient through standardise given dL/dn, the output n and the sd."""
    return (gn - gn.mean(axis=2, keepdims=True) - n * (gn * n).mean(axis=2, keepdims=True)) / sd


def fold_trials(edges, n_trial: int, bin_days: float):
    """Trial periods (in bins) of every window: n_trial log-spaced points at
    the centres of n_trial equal log-steps of [edges[w], edges[w+1])."""
    edges = np.asarray(edges, dtype=np.float64)
    frac = (np.arange(n_trial) + 0.5) / n_trial
    return edges[:-1, None] * (edges[1:, None] / edges[:-1, None]) ** frac[None, :] / bin_days


def fold_step(T: float) -> int:
    """32.32 fixed-point step of a trial period of T bins (round half up)."""
    return int(np.floor(4294967296.0 * float(T) + 0.5))


def fold_pool(e, trials):
    """Coarse fold of each event series at every trial period.  For trial T
    (bins) with fixed-point step R, phase phi in [0, min(L, ceil(R/2^32)))
    sums e over the transit positions phi + ((k R + 2^31) >> 32), k = 0, 1,
    ..., inside the series; the score is that sum over sqrt(number of
    terms).  Per window: the maximum score over its trials and phases (ties:
    the first trial, then the smallest phase).  Returns g [B][W][E] and the
    winning (trial, phase) [B][W][E][2]."""
    B, E, L = e.shape
    W, S = trials.shape
    g = np.zeros((B, W, E))
    arg = np.zeros((B, W, E, 2), dtype=np.int64)
    for w in range(W):
        best = np.full((B, E), -np.inf)
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
                sc = e[:, :, pos].sum(axis=2) / np.sqrt(len(pos))
                better = sc > best
                best = np.where(better, sc, best)
                arg[:, w, :, 0] = np.where(better, s_, arg[:, w, :, 0])
                arg[:, w, :, 1] = np.where(better, ph, arg[:, w, :, 1])
        g[:, w, :] = np.where(np.isfinite(best), best, 0.0)
        arg[:, w, :, 0] = np.where(np.isfinite(best), arg[:, w, :, 0], -1)
    return g, arg


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


def windows_for(n_windows: int, p_lo: float, p_hi: float, bin_days: float):
    """Integer lag ranges [lo, hi] (bins) of n_windows log-spaced period
    windows over [p_lo, p_hi] days, and each window's position q in [0, 1]."""
    edges = p_lo * (p_hi / p_lo) ** (np.arange(n_windows + 1) / n_windows)
    lo = np.maximum(1, np.round(edges[:-1] / bin_days)).astype(np.int64)
    hi = np.maximum(lo, np.round(edges[1:] / bin_days).astype(np.int64))
    q = (np.arange(n_windows) + 0.5) / n_windows
    return lo, hi, q, edges


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    a = (a + 0x7FFF + ((a >> 16) & 1)) & 0xFFFF0000
    return a.astype(np.uint32).view(np.float32).astype(np.float64)


def _q(x, on):
    return bf16(x) if on else x


def forward(p: dict, x, win_lo, win_hi, win_q, n_layers: int = 5, keep: bool = False, bf16_trunk: bool = False,
            trials=None):
    """bf16_trunk: round the convolution inputs, weights and outputs to
    bfloat16 (the storage precision of the device trunk); the arithmetic
    stays FP64.  trials: None for lag-correlation pooling over the windows'
    lag ranges; else [W][S] trial periods in bins for fold pooling, with a
    linear event projection and features (window max, q)."""
    h = [_q(x, bf16_trunk)]
    for l in range(n_layers):
        y = np.maximum(conv1d(h[-1], _q(p[f"W{l}"], bf16_trunk), p[f"b{l}"]), 0.0)
        h.append(_q(y, bf16_trunk))
    pre_e = np.einsum("ec,bcl->bel", p["P"], h[-1]) + p["p"][None, :, None]
    if trials is not None:
        e = pre_e
        g, arg = fold_pool(e, np.asarray(trials, dtype=np.float64))
        B, W = g.shape[:2]
        f = np.concatenate([g, np.broadcast_to(win_q[None, :, None], (B, W, 1))], axis=2)
        pre_r = np.einsum("hf,bwf->bwh", p["U"], f) + p["u"]
        r = np.maximum(pre_r, 0.0)
        z = np.einsum("h,bwh->bw", p["v"], r) + p["v0"][0]
        if not keep:
            return z
        return z, dict(h=h, pre_e=pre_e, e=e, arg=arg, f=f, pre_r=pre_r, r=r, bf16_trunk=bf16_trunk,
                       trials=np.asarray(trials, dtype=np.float64))
    e = np.maximum(pre_e, 0.0)
    lags = np.arange(int(win_lo.min()), int(win_hi.max()) + 1)
    a = lag_correlation(e, lags)
    an, sd = standardise(a)
    B, E, _ = a.shape
    W = len(win_lo)
    g = np.zeros((B, W, E))
    m = np.zeros((B, W, E))
    arg = np.zeros((B, W, E), dtype=np.int64)
    for w in range(W):
        sl = slice(win_lo[w] - lags[0], win_hi[w] - lags[0] + 1)
        seg = an[:, :, sl]
        arg[:, w, :] = np.argmax(seg, axis=2) + win_lo[w]  # absolute lag of the first maximum
        g[:, w, :] = np.max(seg, axis=2)
        m[:, w, :] = np.mean(seg, axis=2)
    f = np.concatenate([g, m, np.broadcast_to(win_q[None, :, None], (B, W, 1))], axis=2)
    pre_r = np.einsum("hf,bwf->bwh", p["U"], f) + p["u"]
    r = np.maximum(pre_r, 0.0)
    z = np.einsum("h,bwh->bw", p["v"], r) + p["v0"][0]
    if not keep:
        return z
    cache = dict(h=h, pre_e=pre_e, e=e, lags=lags, a=a, an=an, sd=sd, arg=arg, f=f, pre_r=pre_r, r=r,
                 bf16_trunk=bf16_trunk)
    return z, cache


def bce_loss(z, y, pos_weight: float = 1.0):
    """Mean over (b, w) of the weighted binary cross-entropy with logits."""
    w = np.where(y > 0.5, pos_weight, 1.0)
    l = np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z)))
    loss = np.sum(w * l) / z.size
    gz = w * (1.0 / (1.0 + np.exp(-z)) - y) / z.size
    return loss, gz


def backward(p: dict, cache: dict, gz, win_lo, win_hi, n_layers: int = 5) -> dict:
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
    h = cache["h"]
    if "trials" in cache:
        L = cache["e"].shape[2]
        gpre_e = fold_pool_backward(gf[:, :, :E], cache["arg"], cache["trials"], L)
        return _trunk_backward(p, g, h, gpre_e, cache, n_layers)
    gg, gm = gf[:, :, :E], gf[:, :, E:2 * E]
    a, lags, arg, e = cache["a"], cache["lags"], cache["arg"], cache["e"]
    B, _, L = e.shape
    ga = np.zeros_like(a)
    for w in range(len(win_lo)):
        lo, hi = win_lo[w] - lags[0], win_hi[w] - lags[0] + 1
        ga[:, :, lo:hi] += gm[:, w, :, None] / (hi - lo)
        for b in range(B):
            for c in range(E):
                ga[b, c, arg[b, w, c] - lags[0]] += gg[b, w, c]
    ga = standardise_backward(ga, cache["an"], cache["sd"])
    ge = np.zeros_like(e)
    for i, tau in enumerate(lags):
        if tau < L:
            coef = ga[:, :, i:i + 1] / L
            ge[:, :, :L - tau] += coef * e[:, :, tau:]
            ge[:, :, tau:] += coef * e[:, :, :L - tau]
    gpre_e = ge * (cache["pre_e"] > 0)
    return _trunk_backward(p, g, h, gpre_e, cache, n_layers)


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
