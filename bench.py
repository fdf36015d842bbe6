"""Benchmark of the transit search on one MI355X.

One step = one pass of the whole search over one light curve already resident
in HBM: template resampling, light-curve resampling, linear search, periodic
search (fold + per-period argmax) and the best period.  Workload: one 90-d
light curve at 20-s cadence (369 360 observations, AR(1) red + white noise,
pre-whitened, 5% gaps, two injected transits), 20 log-spaced durations
0.5-15 h, 50 000 log-spaced periods 0.5-45 d; synthetic, seeded.

Metric: light-curve points x trial periods per second, linear + periodic
(N_obs * K / step time), and the learned proposal's recall of the plain
search's detections above SNR 7 with its speedup (held-out curves of the
learned-proposal workload).  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VECTOR_PEAK_TFLOPS = 157.3
PROFILE_COUNTERS = os.path.join(ROOT, "profiles", "fold_high_cadence_counters.json")
PROFILE_PIPELINE = os.path.join(ROOT, "profiles", "fold_high_cadence_pipeline_counters.json")
# Vector-memory load path of one CU: a wave load of 16 bytes per lane (1 KB)
# keeps the address unit busy 16 cycles (its busy counter), i.e. 64 B per cycle.
L1_PEAK_GBS = 64.0 * 256 * 2.4
FOLD_SOURCES = [os.path.join(ROOT, "paper_2503_20875_amd", "csrc", name) for name in ("fold.hip", "stages.h")]
PROPOSAL_WEIGHTS = os.path.join(ROOT, "paper_2503_20875_amd", "weights", "proposal.npz")


def strip_comments(src: str) -> str:
    """C++ source without its comments and blank lines (string and character
    literals are kept as they are)."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            j = src.find("\n", i)
            i = n if j < 0 else j
        elif src.startswith("/*", i):
            j = src.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return "\n".join(line.rstrip() for line in "".join(out).splitlines() if line.strip())


def fold_source_hash() -> str:
    """Hash of the code the fold kernel is compiled from, comments excluded
    (counter figures are only reported for the kernel they were taken on)."""
    h = hashlib.sha256()
    for path in FOLD_SOURCES:
        with open(path, encoding="utf-8") as fh:
            h.update(strip_comments(fh.read()).encode())
    return h.hexdigest()[:16]


def algorithmic_work(wl, grid):
    """Element visits of the fold (sum over periods of allowed durations x I),
    fold bytes (8 B per visit + 20 B per period record) and linear FLOP
    (4 per window-point visit: two FMAs)."""
    durs = np.asarray(wl.durations)
    J_k = np.array([np.count_nonzero(durs < P) for P in wl.periods], dtype=np.int64)
    visits = int(J_k.sum()) * int(grid.n_t0)
    fold_bytes = 8 * visits + 20 * len(wl.periods)
    c, dt = grid.cadence, grid.t0_step
    # points per window: floor(te/c) - ceil(ts/c) + 1 ~ D/c (exact count summed below)
    lin_points = 0
    i = np.arange(grid.n_t0, dtype=np.float64)
    t_end = (grid.n - 1) * c
    for D in durs:
        ts = i * dt - 0.5 * D
        te = ts + D
        ok = (ts >= 0) & (te <= t_end)
        lo = np.ceil(ts[ok] / c)
        hi = np.floor(te[ok] / c)
        lin_points += int(np.sum(np.maximum(hi - lo + 1, 0)))
    return dict(fold_visits=visits, fold_bytes=fold_bytes, linear_points=lin_points,
                linear_flop=4 * lin_points)


def cpu_baseline(wl, stride: int = 10):
    """The FP64 oracle, as it is, on a bounded sample: full resample + linear
    search, fold over every `stride`-th period, extrapolated linearly in fold
    element visits to the full period grid."""
    import oracle
    g = oracle.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, wl.n_model)
    model = oracle.template(wl.dense, wl.n_model)
    t0 = time.perf_counter()
    flux, ivar = oracle.resample(g, wl.t, wl.f, wl.sigma)
    lin = oracle.linear(g, flux, ivar, model)
    t_lin = time.perf_counter() - t0
    sel = np.arange(0, len(wl.periods), stride)
    t0 = time.perf_counter()
    oracle.periodic(g, lin, wl.periods, sel=sel)
    t_fold = time.perf_counter() - t0
    durs = np.asarray(wl.durations)
    jk = np.array([np.count_nonzero(durs < P) for P in wl.periods], dtype=np.float64)
    scale = jk.sum() / jk[sel].sum()
    t_full = t_lin + t_fold * scale
    value = wl.n_obs * len(wl.periods) / t_full
    return dict(value=value, unit="LC points x trial periods / s", cores=oracle.max_threads(), kind="oracle",
                sample=(f"resample + linear search in full ({t_lin:.2f} s), fold over every {stride}th period "
                        f"({len(sel)} of {len(wl.periods)}, {t_fold:.2f} s) extrapolated x{scale:.1f} in fold "
                        f"element visits; estimated full search {t_full:.1f} s"),
                seconds_measured=round(t_lin + t_fold, 2))


def batched_block(n_curves: int = 32, seed: int = 20250328) -> dict:
    """Batched search over survey curves of uneven length (5 000-120 000
    points at 2-min cadence, 16 durations, per-curve duty-cycle period grids
    over 0.5-min(40, T/2) d): one eager pass, then the same batch captured in
    a HIP graph and replayed, both timed with HIP events; throughput is
    sum over curves of N_obs x K_c per second.  Long gapped curves fold
    more epochs per point than the contiguous single-curve workload, so the
    algorithmic fold bytes per second (same definition as the single-curve
    roofline, whole batch time including the linear stages) are reported
    beside it as the comparable rate."""
    import torch
    import paper_2503_20875_amd as cm
    from synthlc import workloads as W
    curves = W.batched_survey(n_curves, seed=seed)
    grids = [cm.grid_plan(c.t[0], c.t[-1], c.cadence, c.durations, 0.0, c.n_model) for c in curves]
    oo = np.concatenate([[0], np.cumsum([c.n_obs for c in curves])])
    po = np.concatenate([[0], np.cumsum([len(c.periods) for c in curves])])
    dev = "cuda"
    t = torch.as_tensor(np.concatenate([c.t for c in curves]), device=dev)
    f = torch.as_tensor(np.concatenate([c.f for c in curves]), device=dev)
    s_ = torch.as_tensor(np.concatenate([c.sigma for c in curves]), device=dev)
    p = torch.as_tensor(np.concatenate([c.periods for c in curves]), device=dev)
    model = cm.template_resample(torch.as_tensor(curves[0].dense, device=dev), curves[0].n_model)
    plan = cm.batch_plan(grids, oo, po)
    work = cm.batch_workspace(plan)
    out = cm.batch_search(plan, t, f, s_, model, p, work=work)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    e[0].record()
    cm.batch_search(plan, t, f, s_, model, p, work=work, out=out)
    e[1].record()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            cm.batch_search(plan, t, f, s_, model, p, work=work, out=out)
    torch.cuda.current_stream().wait_stream(side)
    e[2].record()
    g.replay()
    e[3].record()
    torch.cuda.synchronize()
    work_units = float(sum(c.n_obs * len(c.periods) for c in curves))
    fold_bytes = float(sum(algorithmic_work(c, gr)["fold_bytes"] for c, gr in zip(curves, grids)))
    ms_eager, ms_graph = e[0].elapsed_time(e[1]), e[2].elapsed_time(e[3])
    sec = min(ms_eager, ms_graph) / 1e3
    return {"workload": f"{n_curves} survey curves, {int(oo[-1])} observations, {int(po[-1])} trial periods in all",
            "n_launches": plan.info["n_launches"], "ms_eager": ms_eager, "ms_graph_replay": ms_graph,
            "value": work_units / sec, "unit": "LC points x trial periods / s",
            "fold_algorithmic_bytes": fold_bytes, "fold_algorithmic_GBps": fold_bytes / sec / 1e9,
            "status": int(out["status"].item())}


PROPOSAL_WEIGHTS_LONG = os.path.join(ROOT, "paper_2503_20875_amd", "weights", "proposal_long.npz")


def learned_long_block(wl, top_k: int = 64) -> dict:
    """The learned form on the Earth-analogue curve: the proposal trained
    for two-year, 25-s curves picks the top_k of 512 windows over 1-400 d
    and the periodic search folds their periods only; timed (downsample,
    network, window selection, restricted fold, best) against the full
    periodic search on the same fold-ready array, one warm-up each."""
    if not os.path.exists(PROPOSAL_WEIGHTS_LONG):
        return {"status": "no trained long-baseline proposal weights in the tree"}
    import torch
    from paper_2503_20875_amd.learned import load_weights
    from paper_2503_20875_amd.train_proposal import make_pipeline
    net, meta = load_weights(PROPOSAL_WEIGHTS_LONG)
    pipe = make_pipeline(workload="long")
    fold = pipe.linear(torch.as_tensor(wl.t, device="cuda"), torch.as_tensor(wl.f, device="cuda"),
                       torch.as_tensor(wl.sigma, device="cuda"))
    pipe.plain(fold)
    pipe.search(net, fold, top_k)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    e[0].record()
    bp = pipe.plain(fold)
    e[1].record()
    e[2].record()
    rec, _, _, n_sub = pipe.search(net, fold, top_k)
    e[3].record()
    torch.cuda.synchronize()
    ms_plain, ms_learned = e[0].elapsed_time(e[1]), e[2].elapsed_time(e[3])
    return {"top_k": top_k, "periods_folded_fraction": n_sub / pipe.K, "plain_ms": ms_plain,
            "learned_ms": ms_learned, "speedup": ms_plain / ms_learned,
            "same_best": bool(rec is not None and rec["k"] == bp["k"]), "best_period": bp["period"],
            "trained_on": {k: meta.get(k) for k in ("n_train", "epochs", "n_trial", "seed")}}


def long_baseline_block(tunings=((8, 8, 4, 2),), reps: int = 2) -> dict:
    """The Earth-analogue curve (730.5 d at 25 s: 2 524 608 points, J = 30,
    I = 1 755 200, K = 399 404): a 421 MB fold-ready array, larger than the
    256 MB Infinity Cache (the concurrent workgroups sweep one 14 MB duration
    row at a time).  Resample + linear search, then the periodic search under
    each tuning (one untimed launch, then `reps` timed ones), with HIP events;
    algorithmic fold bytes over the mean launch time against the HBM peak.
    Also the monotransit-only search (resample + linear search + the five
    strongest single events), timed once after a warm-up."""
    import torch
    import paper_2503_20875_amd as cm
    from synthlc import workloads as W
    wl = W.long_baseline()
    dev = "cuda"
    grid = cm.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, 0.0, wl.n_model)
    K = len(wl.periods)
    t_d, f_d, s_d = (torch.as_tensor(a, device=dev) for a in (wl.t, wl.f, wl.sigma))
    per_d = torch.as_tensor(wl.periods, device=dev)
    fold = torch.empty((grid.n_dur, grid.n_t0, 2), dtype=torch.float32, device=dev)
    work = torch.empty(cm.periodic_workspace(grid, K), dtype=torch.uint8, device=dev)
    model = cm.template_resample(torch.as_tensor(wl.dense, device=dev), wl.n_model)

    def linear():
        flux, ivar, _ = cm.resample(grid, t_d, f_d, s_d, status=False)
        cm.linear_search(grid, flux, ivar, model, fold=fold)

    linear()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    linear()
    e1.record()
    torch.cuda.synchronize()
    lin_ms = e0.elapsed_time(e1)
    before = cm.get_tuning()
    per = None
    fold_ms = {}
    try:
        for tun in tunings:
            cm.set_tuning(*tun)
            per = cm.periodic_search(grid, fold, per_d, work=work, out=per)
            ms = []
            for _ in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                cm.periodic_search(grid, fold, per_d, work=work, out=per)
                b.record()
                b.synchronize()
                ms.append(a.elapsed_time(b))
            fold_ms[",".join(map(str, tun))] = sum(ms) / len(ms)
    finally:
        cm.set_tuning(**before)
    rec = cm.best_record(cm.best(grid, per_d, per))
    # monotransit-only search: resample + linear search + the 5 strongest single events
    ev_out = cm.single_events(grid, fold, 5)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    linear()
    cm.single_events(grid, fold, 5, out=ev_out)
    b.record()
    b.synchronize()
    mono_ms = a.elapsed_time(b)
    events = cm.event_records(ev_out)
    alg = algorithmic_work(wl, grid)
    fastest = min(fold_ms, key=fold_ms.get)
    gbps = alg["fold_bytes"] / (fold_ms[fastest] / 1e3) / 1e9
    learned = learned_long_block(wl)
    return {"workload": (f"long baseline: {wl.n_obs} points at 25 s over 730.5 d, J = {grid.n_dur}, "
                         f"I = {grid.n_t0}, K = {K}; fold-ready array {grid.n_dur * grid.n_t0 * 8 / 1e6:.0f} MB"),
            "linear_ms": lin_ms, "fold_ms_by_tuning": fold_ms, "fastest_tuning": fastest,
            "fold_algorithmic_bytes": alg["fold_bytes"], "fold_effective_GBps": gbps,
            "frac_of_hbm_peak": gbps / HBM_PEAK_GBS,
            "search_ms": lin_ms + fold_ms[fastest],
            "points_x_periods_per_s": wl.n_obs * K / ((lin_ms + fold_ms[fastest]) / 1e3),
            "best": {"period": rec["period"], "snr": rec["snr"], "duration": rec["duration"]},
            "monotransit_search_ms": mono_ms,
            "learned": learned,
            "single_events": [{"t0_abs": e["t0_abs"], "duration": e["duration"], "snr": e["snr"]} for e in events[:3]]}


def keplerian_block(rho=(0.5, 3.0), k_max: float = 0.2, b_max: float = 0.9, reps: int = 2) -> dict:
    """The paper's default duration filter on the benchmark curve: the fold
    over each period's Keplerian durations only (circular orbits around
    stars of density rho g/cm^3, radius ratio <= k_max, impact parameter
    <= b_max), timed against the unfiltered fold on the same fold-ready
    array; and the optimally sampled period grid the paper's default would
    use for this span at the solar density (oversampling 3), with its
    periods x durations fold time."""
    import torch
    import paper_2503_20875_amd as cm
    from synthlc import workloads as W
    wl = W.high_cadence()
    dev = "cuda"
    grid = cm.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, 0.0, wl.n_model)
    model = cm.template_resample(torch.as_tensor(wl.dense, device=dev), wl.n_model)
    flux, ivar, _ = cm.resample(grid, torch.as_tensor(wl.t, device=dev), torch.as_tensor(wl.f, device=dev),
                                torch.as_tensor(wl.sigma, device=dev), status=False)
    fold = cm.linear_search(grid, flux, ivar, model)

    def timed(periods, jrange=None, stride=None):
        K = len(periods)
        per_d = torch.as_tensor(periods, device=dev)
        jr_d = None if jrange is None else torch.as_tensor(jrange, device=dev)
        work = torch.empty(max(cm.periodic_workspace(grid, K), 1), dtype=torch.uint8, device=dev)
        out = cm.periodic_search(grid, fold, per_d, jrange=jr_d, work=work, stride=stride)
        ms = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            cm.periodic_search(grid, fold, per_d, jrange=jr_d, work=work, out=out, stride=stride)
            b.record()
            b.synchronize()
            ms.append(a.elapsed_time(b))
        return sum(ms) / len(ms), cm.best_record(cm.best(grid, per_d, out))

    durs = np.asarray(wl.durations)
    allowed = np.array([np.count_nonzero(durs < P) for P in wl.periods])
    jr = cm.keplerian_jrange(wl.periods, durs, rho[0], rho[1], k_max, b_max)
    kept = np.clip(np.minimum(jr[:, 1], allowed - 1) - jr[:, 0] + 1, 0, None)
    ms_all, b_all = timed(wl.periods)
    ms_kep, b_kep = timed(wl.periods, jr)
    span = wl.t[-1] - wl.t[0]
    ofir = cm.period_grid(span, float(wl.periods[0]), float(wl.periods[-1]), cm.SOLAR_DENSITY, 3.0)
    jr_ofir = cm.keplerian_jrange(ofir, durs, rho[0], rho[1], k_max, b_max)
    ms_ofir, b_ofir = timed(ofir, jr_ofir)
    # the duration-scaled epoch grid (reference-time step 1% of each duration)
    st = cm.epoch_strides(grid, 0.01)
    ms_st, b_st = timed(wl.periods, stride=st)
    ms_st_all, b_st_all = timed(ofir, jr_ofir, stride=st)
    return {"workload": f"90 d at 20 s, J = {len(durs)}, K = {len(wl.periods)} duty-cycle periods 0.5-45 d",
            "filter": {"rho_g_cm3": list(rho), "k_max": k_max, "b_max": b_max},
            "fold_visits_kept": float(kept.sum() / allowed.sum()),
            "fold_ms_all_durations": ms_all, "fold_ms_keplerian": ms_kep,
            "best_all": {"period": b_all["period"], "snr": b_all["snr"], "duration": b_all["duration"]},
            "best_keplerian": {"period": b_kep["period"], "snr": b_kep["snr"], "duration": b_kep["duration"]},
            "optimal_grid": {"n_periods": int(len(ofir)), "fold_ms_keplerian": ms_ofir,
                             "best": {"period": b_ofir["period"], "snr": b_ofir["snr"]}},
            "duration_scaled_epochs": {"fraction": 0.01, "strides": st.tolist(),
                                       "fold_visits_kept": float(np.sum(allowed_rows(durs, wl.periods) / st[None, :])
                                                                 / allowed.sum()),
                                       "fold_ms_all_durations": ms_st,
                                       "best": {"period": b_st["period"], "snr": b_st["snr"]},
                                       "with_optimal_grid_and_filter_ms": ms_st_all,
                                       "best_with_optimal_grid_and_filter": {"period": b_st_all["period"],
                                                                             "snr": b_st_all["snr"]}}}


def allowed_rows(durs, periods):
    """[K][J] 1 where duration j is shorter than period k (the rows a fold
    evaluates), else 0."""
    return (np.asarray(durs)[None, :] < np.asarray(periods)[:, None]).astype(np.float64)


BF16_MFMA_PEAK_TFLOPS = 2500.0


def net_block(batch: int = 32, length: int = 8192, reps: int = 10) -> dict:
    """MFMA roofline of the proposal network's 64-channel convolution (the
    dominant kernel of training): forward and backward (weights and input)
    of one 64 -> 64 channel, 9-tap layer over batch x length positions,
    timed with HIP events, against the dense BF16 MFMA peak; plus one full
    training step (forward, backward, Adam) of the network."""
    import torch
    from paper_2503_20875_amd import proposal as P
    g = torch.Generator(device="cpu").manual_seed(7)
    x = torch.rand((batch, length, 64), generator=g).to("cuda", torch.bfloat16)
    w = (torch.randn((64, 576), generator=g) * 0.06).to("cuda", torch.bfloat16)
    bias = torch.zeros(64, device="cuda")
    dy = torch.randn((batch, length, 64), generator=g).to("cuda")
    y = P.conv1d_fwd(x, w, bias)
    P.conv1d_bwd(dy, y, x, w)
    flop_fwd = 2.0 * 64 * 64 * 9 * length * batch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    for _ in range(reps):
        P.conv1d_fwd(x, w, bias)
    ev[1].record()
    ev[2].record()
    for _ in range(reps):
        P.conv1d_bwd(dy, y, x, w)
    ev[3].record()
    torch.cuda.synchronize()
    ms_f = ev[0].elapsed_time(ev[1]) / reps
    ms_b = ev[2].elapsed_time(ev[3]) / reps
    tf_f = flop_fwd / (ms_f / 1e3) / 1e12
    tf_b = 2 * flop_fwd / (ms_b / 1e3) / 1e12  # weight and input gradients
    # one training step of the whole network on random inputs
    net = P.ProposalNet()
    win = P.Windows.log_spaced(512, 1.0, 100.0, 111.1 / length)
    xin = torch.rand((batch, length, 16), generator=g).to("cuda", torch.bfloat16)
    lab = torch.zeros((batch, 512), device="cuda")
    lab[:, 100] = 1.0
    for _ in range(2):
        net.forward(xin, win)
        net.backward(lab, pos_weight=32.0)
        net.adam()
    ev[0].record()
    for _ in range(3):
        net.forward(xin, win)
        net.backward(lab, pos_weight=32.0)
        net.adam()
    ev[1].record()
    torch.cuda.synchronize()
    step_ms = ev[0].elapsed_time(ev[1]) / 3
    return {"kernel": "conv_fwd_kernel / conv_bwd (64 -> 64 channels, 9 taps, bf16 MFMA, FP32 accumulation)",
            "bound": "mfma", "achieved": tf_f, "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": tf_f / BF16_MFMA_PEAK_TFLOPS, "backward_achieved": tf_b,
            "backward_frac": tf_b / BF16_MFMA_PEAK_TFLOPS, "fwd_ms": ms_f, "bwd_ms": ms_b,
            "shape": f"batch {batch} x {length} positions", "algorithmic_flop_fwd": flop_fwd,
            "train_step_ms": step_ms, "train_examples_per_s": batch / (step_ms / 1e3)}


def learned_block(n_curves: int, seed: int = 20250402, target: float = 0.99) -> dict:
    """Learned proposal versus the plain periodic search on held-out curves of
    the learned-proposal workload (80 000 points at 2-min cadence, half with
    one planet; seeds disjoint from the training set).  Half the curves
    (calibration, run at the default K = 64 windows without fallback) fix two
    operating points that keep `target` of the plain detections above SNR 7:
    the smallest K whose top-K windows hold them (proposal only), and the
    smallest restricted-SNR threshold of the full-fold fallback at K = 64.
    The other half (test) runs both and reports recall and the device-time
    speedup over the full fold, fallback runs included."""
    if not os.path.exists(PROPOSAL_WEIGHTS):
        return {"status": "no trained proposal weights in the tree"}
    from paper_2503_20875_amd.learned import evaluate, fallback_threshold, k_for_recall, load_weights
    from paper_2503_20875_amd.train_proposal import make_pipeline
    from synthlc import workloads as W
    net, meta = load_weights(PROPOSAL_WEIGHTS)
    pipe = make_pipeline()
    n_cal = n_curves // 2
    rng_cal, rng_test = np.random.default_rng(seed), np.random.default_rng(seed + 1)
    cal = evaluate(pipe, net, [W.learned_curve(rng_cal) for _ in range(n_cal)])
    k_target = k_for_recall(cal["ranks"], target, pipe.windows.n)
    tau = fallback_threshold(cal["rows"], target)
    test_curves = [W.learned_curve(rng_test) for _ in range(n_curves - n_cal)]
    test_k = evaluate(pipe, net, test_curves, top_k=k_target)
    test_fb = evaluate(pipe, net, test_curves, fallback_snr=tau)
    batched = learned_batched(pipe, net, test_curves, test_k, k_target)

    def point(r):
        return {"recall_at_snr7": r["recall"], "n_detections": r["n_detections"], "n_recalled": r["n_recalled"],
                "recall_true_detections": r["recall_true"], "n_true_detections": r["n_true_detections"],
                "plain_ms_per_curve": r["plain_ms_per_curve"], "learned_ms_per_curve": r["learned_ms_per_curve"],
                "speedup": r["speedup"], "periods_folded_fraction": r["periods_folded_fraction"],
                "fallback_fraction": r["fallback_fraction"]}

    return {
        "workload": (f"{n_curves} held-out curves ({n_cal} calibration + {n_curves - n_cal} test), "
                     f"{W.LEARNED_N_POINTS} points at 120 s, 16 durations 0.5-10 h, K = {pipe.K} periods "
                     f"1-100 d, {pipe.windows.n} log windows"),
        "target_recall": target,
        "calibration": {"k64_recall": cal["recall"], "n_detections": cal["n_detections"],
                        "k64_speedup": cal["speedup"], "k_for_target": k_target,
                        "fallback_snr_for_target": tau if np.isfinite(tau) else None},
        "proposal_only": {"k_windows": k_target, **point(test_k)},
        "proposal_with_fallback": {"k_windows": pipe.cfg.top_k, "fallback_snr": tau if np.isfinite(tau) else None,
                                   **point(test_fb)},
        "batched": batched,
        "trained_on": {k: meta.get(k) for k in ("n_train", "epochs", "batch", "lr", "seed")},
    }


def learned_batched(pipe, net, curves, ref, k_target: int) -> dict:
    """The learned and plain searches over the test curves as one batch: the
    fold-ready arrays of all curves are resident, then the plain periodic
    searches run back to back against `Pipeline.search_batch` (features, one
    network forward over the batch, top-K, restricted searches) at K = 64
    and at the calibrated K; device time over the whole batch.  Recall is
    checked against the plain records of the same batch."""
    import torch
    folds = [pipe.linear(torch.as_tensor(t, device="cuda"), torch.as_tensor(f, device="cuda"),
                         torch.as_tensor(s, device="cuda")) for t, f, s, _ in curves]
    pipe.plain(folds[0])
    pipe.search_batch(net, folds[:2], 64)
    torch.cuda.synchronize()

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        out = fn()
        b.record()
        b.synchronize()
        return out, a.elapsed_time(b)

    plain, ms_plain = timed(lambda: [pipe.plain(f) for f in folds])
    out = {"n_curves": len(folds), "plain_ms": ms_plain}
    for name, k in (("k64", 64), ("k_target", k_target)):
        res, ms = timed(lambda: pipe.search_batch(net, folds, k))
        det = [i for i, p in enumerate(plain) if p["k"] >= 0 and p["snr"] > 7.0]
        hit = [i for i in det if res[i][0] is not None and res[i][0]["k"] == plain[i]["k"]]
        out[name] = {"top_k": k, "learned_ms": ms, "speedup": ms_plain / ms, "n_detections": len(det),
                     "n_recalled": len(hit), "recall": len(hit) / len(det) if det else None,
                     "periods_folded_fraction": sum(r[1] for r in res) / (len(folds) * pipe.K)}
    del folds
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="high_cadence", choices=["high_cadence", "tiny", "long_baseline"])
    ap.add_argument("--no-long-baseline", action="store_true",
                    help="skip the long-baseline (2 yr at 25 s) fold measurement")
    ap.add_argument("--no-extras", action="store_true",
                    help="time the benchmark steps only (no filter, long-baseline, network, batched, learned or "
                         "CPU measurements), e.g. for kernel traces of the headline search")
    ap.add_argument("--mode", default="full", choices=["full", "fold", "copy", "net"],
                    help="full: the benchmark; fold: setup once, then --steps fold launches only "
                         "(for counter runs); copy: a plain device copy of --copy-mib MiB, --steps "
                         "times (calibrates the HBM byte counters); net: the proposal network's "
                         "convolution roofline only (for kernel traces and MFMA counters)")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--batch-curves", type=int, default=32,
                    help="survey curves of the batched-search measurement (0: skip)")
    ap.add_argument("--fold-tuning", default="",
                    help="period block, workgroups per CU, units per workgroup, variant (e.g. 4,8,4,0); "
                         "default: the library's")
    ap.add_argument("--learned-curves", type=int, default=128,
                    help="held-out curves for the learned-versus-plain comparison (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the search has no "
              "multi-GPU path in this build.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2503_20875_amd as cm
    from synthlc import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.mode == "copy":
        n = args.copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(args.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_read_per_launch": 4 * n, "bytes_written_per_launch": 4 * n,
                          "launches": args.steps}), flush=True)
        return
    if args.mode == "net":
        print(json.dumps({"mode": "net", **net_block()}), flush=True)
        return
    if args.fold_tuning:
        cm.set_tuning(*(int(v) for v in args.fold_tuning.split(",")))
    wl = W.WORKLOADS[args.workload]()
    dev = "cuda"
    t_d = torch.as_tensor(wl.t, device=dev)
    f_d = torch.as_tensor(wl.f, device=dev)
    s_d = torch.as_tensor(wl.sigma, device=dev)
    dense_d = torch.as_tensor(wl.dense, device=dev)
    per_d = torch.as_tensor(wl.periods, device=dev)
    grid = cm.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, 0.0, wl.n_model)
    K = len(wl.periods)
    # every buffer allocated up front: the timed region only launches kernels
    fold = torch.empty((grid.n_dur, grid.n_t0, 2), dtype=torch.float32, device=dev)
    work = torch.empty(cm.periodic_workspace(grid, K), dtype=torch.uint8, device=dev)
    per = dict(lr=torch.empty(K, dtype=torch.float32, device=dev),
               epoch=torch.empty(K, dtype=torch.int32, device=dev),
               dur=torch.empty(K, dtype=torch.int32, device=dev),
               depth=torch.empty(K, dtype=torch.float32, device=dev),
               depth_var=torch.empty(K, dtype=torch.float32, device=dev))
    best = torch.empty(96, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    ev = {k: [] for k in ("start", "lin", "fold0", "fold1", "end")}

    def step(record: bool):
        e = {k: torch.cuda.Event(enable_timing=True) for k in ev} if record else None
        if record:
            e["start"].record(stream)
        model = cm.template_resample(dense_d, wl.n_model)
        flux, ivar, _ = cm.resample(grid, t_d, f_d, s_d, status=False)
        cm.linear_search(grid, flux, ivar, model, fold=fold)
        if record:
            e["lin"].record(stream)
            e["fold0"].record(stream)
        cm.periodic_search(grid, fold, per_d, work=work, out=per)
        if record:
            e["fold1"].record(stream)
        cm.best(grid, per_d, per, out=best)
        if record:
            e["end"].record(stream)
            for k in ev:
                ev[k].append(e[k])

    if args.mode == "fold":
        model = cm.template_resample(dense_d, wl.n_model)
        flux, ivar, _ = cm.resample(grid, t_d, f_d, s_d, status=False)
        cm.linear_search(grid, flux, ivar, model, fold=fold)
        for _ in range(args.steps):
            cm.periodic_search(grid, fold, per_d, work=work, out=per)
        torch.cuda.synchronize()
        work_alg = algorithmic_work(wl, grid)
        print(json.dumps({"mode": "fold", "launches": args.steps, "workload": args.workload, "tuning": cm.get_tuning(),
                          "fold_source_sha256_16": fold_source_hash(),
                          "algorithmic_bytes_per_launch": work_alg["fold_bytes"]}), flush=True)
        return

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_steps = [ev["start"][i].elapsed_time(ev["end"][i]) for i in range(args.steps)]
    ms_lin = [ev["start"][i].elapsed_time(ev["lin"][i]) for i in range(args.steps)]
    ms_fold = [ev["fold0"][i].elapsed_time(ev["fold1"][i]) for i in range(args.steps)]
    ms_step = float(np.mean(ms_steps))
    b = cm.best_record(best)

    work_alg = algorithmic_work(wl, grid)
    fold_s = float(np.mean(ms_fold)) / 1e3
    achieved = work_alg["fold_bytes"] / fold_s / 1e9
    traffic = None
    if os.path.exists(PROFILE_COUNTERS):
        with open(PROFILE_COUNTERS) as fh:
            prof = json.load(fh)
        if prof.get("fold_source_sha256_16") == fold_source_hash() and prof.get("workload") == args.workload:
            traffic = prof.get("hbm_bytes_per_launch")
    ta_busy = None
    if os.path.exists(PROFILE_PIPELINE):
        with open(PROFILE_PIPELINE) as fh:
            pipe = json.load(fh)
        if (pipe.get("fold_source_sha256_16") == fold_source_hash() and pipe.get("workload") == args.workload
                and pipe.get("tuning") == [cm.get_tuning()[k] for k in ("fold_period_block", "fold_wgs_per_cu",
                                                                          "fold_units_per_wg", "fold_variant")]):
            ta_busy = pipe.get("ta_busy_frac")
    lin_s = float(np.mean(ms_lin)) / 1e3
    value = wl.n_obs * K / (ms_step / 1e3)
    out = {
        "metric": "LC points x trials/sec (linear+periodic) on 1 GPU",
        "value": value,
        "unit": "LC points x trial periods / s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"single light curve, 90 d at 20 s cadence, {wl.n_obs} observations "
                         f"(N = {grid.n} resampled), J = {grid.n_dur} durations 0.5-15 h, "
                         f"I = {grid.n_t0} reference times, K = {K} periods 0.5-45 d")
            if args.workload == "high_cadence" else wl.name,
            "n_obs": wl.n_obs, "n_grid": int(grid.n), "n_t0": int(grid.n_t0), "n_durations": int(grid.n_dur),
            "n_periods": K, "n_model": wl.n_model,
        },
        "roofline": {
            "kernel": "fold_kernel (periodic search)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": work_alg["fold_bytes"],
            "avg_launch_ms": fold_s * 1e3,
            "tuning": cm.get_tuning(),
        },
        "roofline_l1": {
            "kernel": "fold_kernel (periodic search)",
            "bound": "vector-memory address unit (cache-resident working set)",
            "achieved": achieved,
            "peak": L1_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / L1_PEAK_GBS,
            "ta_busy_frac": ta_busy,
            "note": "achieved counts 8 B per element visit; transit 0 of a period block is one load for all its "
                    "periods, so the bytes the unit delivers are slightly fewer",
        },
        "roofline_linear": {
            "kernel": "linear_kernel (linear search, all durations)",
            "bound": "alu",
            "achieved": work_alg["linear_flop"] / lin_s / 1e12,
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": work_alg["linear_flop"] / lin_s / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
            "algorithmic_flop": work_alg["linear_flop"],
            "avg_ms_incl_setup": lin_s * 1e3,
        },
        "stages_ms": {"setup_and_linear": lin_s * 1e3, "periodic": fold_s * 1e3,
                      "best": ms_step - lin_s * 1e3 - fold_s * 1e3},
        "wall_s_timed": wall,
        "best": {"period": b["period"], "snr": b["snr"], "depth": b["depth"], "duration": b["duration"]},
    }
    if args.no_extras:
        print(json.dumps(out), flush=True)
        return
    if args.workload == "high_cadence":
        out["keplerian"] = keplerian_block()
        if not args.no_long_baseline:
            out["long_baseline"] = long_baseline_block()
        out["roofline_net"] = net_block()
        if args.batch_curves > 0:
            out["batched"] = batched_block(args.batch_curves)
    if args.learned_curves > 0 and args.workload == "high_cadence":
        out["learned"] = learned_block(args.learned_curves)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
