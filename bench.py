"""Benchmark of the transit search on one MI355X.

One step = one pass of the whole search over one light curve already resident
in HBM: template resampling, light-curve resampling, linear search over every
duration, periodic search (fold + per-period argmax) and the best period.
Default workload: the Earth-analogue batch (two-year curves at 25-s cadence,
2 524 608 points each, white noise 200 ppm, one 100-ppm 13-h transit signal
at P = 365.25 d; 30 log-spaced durations 1-20 h; 399 404 duty-cycle periods
1-400 d); each timed step searches the next curve of the batch.  Synthetic,
seeded.

Metric: light-curve points x trial periods per second, linear + periodic
(N_obs * K / step time).  The line also carries the fold's rooflines (bytes
past L2 from live rocprofv3 counter passes against the HBM peak, and the
algorithmic element-visit rate against the vector-memory address unit), the
linear search's FP32 rate, the rate with the host transfers included, the
FP64 oracle timed on the host's cores, and the secondary measurements (the
90-day high-cadence curve, default grids, batched survey, proposal network,
learned proposal recall at SNR > 7).  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import ctypes
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
# Vector-memory load path of one CU: a wave load of 16 bytes per lane (1 KB)
# keeps the address unit busy 16 cycles (its busy counter), i.e. 64 B per cycle.
ADDRESS_UNIT_PEAK_GBS = 64.0 * 256 * 2.4
LONG_SEED = 20250329  # seed of curve 0 of the Earth-analogue batch
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


def algorithmic_work(wl, grid, linear: bool = True):
    """Element visits of the fold (sum over periods of allowed durations x I),
    fold bytes (8 B per visit + 20 B per period record) and, unless
    linear=False, linear FLOP (4 per window-point visit: two FMAs)."""
    durs = np.asarray(wl.durations)
    J_k = np.searchsorted(np.sort(durs), np.asarray(wl.periods), side="left")  # durations below each P
    visits = int(J_k.sum()) * int(grid.n_t0)
    fold_bytes = 8 * visits + 20 * len(wl.periods)
    if not linear:
        return dict(fold_visits=visits, fold_bytes=fold_bytes)
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


def batched_block(n_curves: int = 64, seed: int = 20250328, n_min: int = 5000, n_max: int = 120000,
                  compare: bool = True, workers: int = 1) -> dict:
    """Batched survey: a length-stratified subset of the survey workload
    (curve k has the midpoint length of the k-th of n_curves strata of
    5 000-120 000 points at 2-min cadence; 16 durations 0.5-10 h; per-curve
    duty-cycle period grids over 0.5-min(40, T/2) d), searched by the
    persistent work-queue launch, eagerly and as a replayed HIP graph, both
    timed with HIP events; then the same curves as back-to-back single-curve
    searches (resample, linear search, periodic search, best per curve) for
    comparison.  Throughput is sum over curves of N_obs x K_c per second.
    compare=False times one eager batch only (no warm-up call, graph replay
    or single-curve calls), for surveys that take minutes; while it runs the
    per-curve done flags are read on a side stream every 15 s and logged.
    workers > 1 generates the curves in a forked process pool, so it must
    run before anything initialises the GPU."""
    import torch
    import paper_2503_20875_amd as cm
    from synthlc import workloads as W
    curves = W.survey_subset(n_curves, seed=seed, n_min=n_min, n_max=n_max, workers=workers,
                             progress=lambda k: log(f"batched survey: {k}/{n_curves} curves generated"))
    log(f"batched survey: {n_curves} curves generated")
    torch.cuda.init()
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
    log(f"batched survey: inputs resident, plan and workspace made ({plan.info['n_items']} queue items)")
    work_units = float(sum(c.n_obs * len(c.periods) for c in curves))
    fold_bytes = float(sum(algorithmic_work(c, gr, linear=False)["fold_bytes"] for c, gr in zip(curves, grids)))
    workload = (f"{n_curves} length-stratified survey curves ({n_min}-{n_max} points at 2 min), "
                f"{int(oo[-1])} observations, {int(po[-1])} trial periods in all")
    if not compare:
        torch.cuda.synchronize()
        log("batched survey: one timed batch")
        side = torch.cuda.Stream()
        done_host = torch.empty(n_curves, dtype=torch.int32, pin_memory=True)
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record()
        out = cm.batch_search(plan, t, f, s_, model, p, work=work)
        e[1].record()
        while not e[1].query():
            time.sleep(15.0)
            with torch.cuda.stream(side):
                done_host.copy_(out["done"], non_blocking=True)
            side.synchronize()
            log(f"batched survey: {int((done_host == 1).sum())}/{n_curves} curves done")
        torch.cuda.synchronize()
        sec = e[0].elapsed_time(e[1]) / 1e3
        return {"workload": workload, "n_launches": plan.info["n_launches"], "n_items": plan.info["n_items"],
                "workspace_bytes": plan.info["workspace_bytes"], "ms_eager": sec * 1e3,
                "value": work_units / sec, "unit": "LC points x trial periods / s",
                "fold_algorithmic_bytes": fold_bytes, "fold_algorithmic_GBps": fold_bytes / sec / 1e9,
                "status": int(out["status"].item()), "curves_done": int((out["done"] == 1).sum().item())}
    out = cm.batch_search(plan, t, f, s_, model, p, work=work)
    torch.cuda.synchronize()
    log(f"batched survey: first search done, status {int(out['status'].item())}")
    e = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
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
    log("batched survey: eager and graph-replayed searches timed")
    status = int(out["status"].item())
    n_done = int((out["done"] == 1).sum().item())
    best_batch = out["best"].cpu().numpy()
    del g, work
    # the same curves as single-curve searches back to back (device-resident inputs)
    bufs = []
    for c, gr in zip(curves, grids):
        K = len(c.periods)
        bufs.append((tuple(torch.as_tensor(a, device=dev) for a in (c.t, c.f, c.sigma)),
                     torch.as_tensor(c.periods, device=dev), search_buffers(cm, torch, gr, max(K, 1))))

    def singles():
        for (c, gr), ((td, fd, sd), pd, b) in zip(zip(curves, grids), bufs):
            flux, ivar, _ = cm.resample(gr, td, fd, sd, status=False)
            cm.linear_search(gr, flux, ivar, model, fold=b["fold"])
            if len(c.periods):
                cm.periodic_search(gr, b["fold"], pd, work=b["work"], out=b["per"])
                cm.best(gr, pd, b["per"], out=b["best"])

    singles()
    torch.cuda.synchronize()
    log("batched survey: single-curve searches warmed up")
    e[4].record()
    singles()
    e[5].record()
    torch.cuda.synchronize()
    same = all(np.array_equal(best_batch[i], b[2]["best"].cpu().numpy())
               for i, (c, b) in enumerate(zip(curves, bufs)) if len(c.periods))
    del bufs
    torch.cuda.empty_cache()
    ms_eager, ms_graph, ms_single = e[0].elapsed_time(e[1]), e[2].elapsed_time(e[3]), e[4].elapsed_time(e[5])
    sec = min(ms_eager, ms_graph) / 1e3
    return {"workload": workload,
            "n_launches": plan.info["n_launches"], "n_items": plan.info["n_items"],
            "ms_eager": ms_eager, "ms_graph_replay": ms_graph, "ms_single_curve_calls": ms_single,
            "speedup_over_single_curve_calls": ms_single / min(ms_eager, ms_graph),
            "value": work_units / sec, "unit": "LC points x trial periods / s",
            "fold_algorithmic_bytes": fold_bytes, "fold_algorithmic_GBps": fold_bytes / sec / 1e9,
            "status": status, "curves_done": n_done, "best_equal_to_single_calls": bool(same)}


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


def monotransit_block(wl) -> dict:
    """The monotransit-only search on one curve: resampling, the linear search
    and the five strongest single events, timed once after a warm-up."""
    import torch
    import paper_2503_20875_amd as cm
    grid = cm.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, 0.0, wl.n_model)
    t_d, f_d, s_d = (torch.as_tensor(a, device="cuda") for a in (wl.t, wl.f, wl.sigma))
    model = cm.template_resample(torch.as_tensor(wl.dense, device="cuda"), wl.n_model)
    fold = torch.empty((grid.n_dur, grid.n_t0, 2), dtype=torch.float32, device="cuda")

    def run(out=None):
        flux, ivar, _ = cm.resample(grid, t_d, f_d, s_d, status=False)
        cm.linear_search(grid, flux, ivar, model, fold=fold)
        return cm.single_events(grid, fold, 5, out=out)

    ev_out = run()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    run(ev_out)
    b.record()
    b.synchronize()
    events = cm.event_records(ev_out)
    return {"ms": a.elapsed_time(b),
            "single_events": [{"t0_abs": e["t0_abs"], "duration": e["duration"], "snr": e["snr"]}
                              for e in events[:3]]}


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
    one planet; seeds disjoint from the training set).  Two operating points
    keep `target` of the plain detections above SNR 7: the smallest K whose
    top-K windows hold them (proposal only), and the smallest restricted-SNR
    threshold of the full-fold fallback at K = 64.  They come from the
    weights' metadata when eval_proposal stored them (calibrated on a larger
    held-out set), else from the first half of these curves.  The test
    curves run K = 64 and both operating points and report recall and the
    device-time speedup over the full fold, fallback runs included."""
    if not os.path.exists(PROPOSAL_WEIGHTS):
        return {"status": "no trained proposal weights in the tree"}
    from paper_2503_20875_amd.learned import evaluate, fallback_threshold, k_for_recall, load_weights
    from paper_2503_20875_amd.train_proposal import make_pipeline
    from synthlc import workloads as W
    net, meta = load_weights(PROPOSAL_WEIGHTS)
    pipe = make_pipeline()
    rng_cal, rng_test = np.random.default_rng(seed), np.random.default_rng(seed + 1)
    if meta.get("calibrated_k"):
        # operating points calibrated on a larger held-out set (stored with the
        # weights by eval_proposal); every curve here is a test curve
        n_cal = 0
        k_target = int(meta["calibrated_k"])
        tau = meta.get("calibrated_fallback_snr")
        tau = float("-inf") if tau is None else float(tau)
        cal = None
    else:
        n_cal = n_curves // 2
        cal = evaluate(pipe, net, [W.learned_curve(rng_cal) for _ in range(n_cal)])
        k_target = k_for_recall(cal["ranks"], target, pipe.windows.n)
        tau = fallback_threshold(cal["rows"], target)
    test_curves = [W.learned_curve(rng_test) for _ in range(n_curves - n_cal)]
    test_k64 = evaluate(pipe, net, test_curves, top_k=64)
    test_k = evaluate(pipe, net, test_curves, top_k=k_target, plain=test_k64["plain"])
    test_fb = evaluate(pipe, net, test_curves, fallback_snr=tau, plain=test_k64["plain"])
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
        "calibration": ({"source": meta["calibration"], "k_for_target": k_target,
                         "fallback_snr_for_target": tau if np.isfinite(tau) else None} if cal is None else
                        {"k64_recall": cal["recall"], "n_detections": cal["n_detections"],
                         "k64_speedup": cal["speedup"], "k_for_target": k_target,
                         "fallback_snr_for_target": tau if np.isfinite(tau) else None}),
        "proposal_k64": {"k_windows": 64, **point(test_k64)},
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


def log(msg: str) -> None:
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


# --------------------------------------------------------------- counters
COUNTER_TIMEOUT_S = 240


def _under_profiler() -> bool:
    """True when this process already runs under rocprofv3 (a nested counter
    pass would not work)."""
    pre = os.environ.get("LD_PRELOAD", "")
    return "rocprof" in pre or any(k.startswith("ROCPROF") for k in os.environ)


def read_counter_csv(out_dir: str) -> list:
    """Rows of every rocprofv3 counter-collection CSV under out_dir:
    (dispatch id, kernel name, counter name, value)."""
    import csv
    import glob
    rows = []
    for path in glob.glob(os.path.join(out_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(path, newline="") as fh:
            for r in csv.DictReader(fh):
                rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"])))
    return rows


def per_dispatch(rows, counter: str) -> dict:
    """{dispatch id: (kernel name, summed value)} of one counter."""
    out = {}
    for d, k, c, v in rows:
        if c != counter:
            continue
        name, acc = out.get(d, (k, 0.0))
        out[d] = (name, acc + v)
    return out


def counter_pass(counter: str, workload: str, copy_mib: int, tuning: str) -> dict:
    """One rocprofv3 --pmc pass of `counter` over a child process that runs a
    plain device copy of copy_mib MiB and one fold launch of the workload;
    returns the counter per dispatch of the copy and of the fold (KiB)."""
    import subprocess
    import tempfile
    out_dir = tempfile.mkdtemp(prefix=f"cetra_{counter.lower()}_", dir=os.environ.get("TMPDIR", "/tmp"))
    cmd = ["rocprofv3", "--pmc", counter, "--output-format", "csv", "-d", out_dir, "-o", "run", "--",
           sys.executable, os.path.join(ROOT, "bench.py"), "--mode", "fold", "--workload", workload,
           "--steps", "1", "--copy-mib", str(copy_mib)]
    if tuning:
        cmd += ["--fold-tuning", tuning]
    import signal
    proc = subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, cwd=out_dir,
                            start_new_session=True)
    try:
        text, _ = proc.communicate(timeout=COUNTER_TIMEOUT_S)
    except subprocess.TimeoutExpired:
        os.killpg(proc.pid, signal.SIGKILL)  # the profiler and its child, nothing else
        proc.communicate()
        raise RuntimeError(f"counter pass {counter} exceeded {COUNTER_TIMEOUT_S} s")
    rows = read_counter_csv(out_dir)
    disp = per_dispatch(rows, counter)
    fold = [v for _, (k, v) in sorted(disp.items()) if "fold_kernel" in k]
    copies = [v for _, (k, v) in sorted(disp.items()) if "fold" not in k and ("copy" in k.lower() or "elementwise" in k)]
    if not fold or not copies:
        tail = text.decode(errors="replace")[-600:]
        raise RuntimeError(f"counter pass {counter}: no fold or copy dispatch found (rc {proc.returncode}): {tail}")
    return {"fold_kib": fold, "copy_kib": max(copies), "rc": proc.returncode}


def live_counters(workload: str, tuning: str, copy_mib: int = 1024) -> dict:
    """Bytes the fold moves past L2 per launch, measured now: one rocprofv3
    pass for FETCH_SIZE and one for WRITE_SIZE, each scaled by what the same
    counter reads for a plain copy of copy_mib MiB in the same process (the
    copy reads and writes exactly copy_mib MiB)."""
    copy_bytes = copy_mib * (1 << 20)
    fetch = counter_pass("FETCH_SIZE", workload, copy_mib, tuning)
    write = counter_pass("WRITE_SIZE", workload, copy_mib, tuning)
    f_scale = copy_bytes / (fetch["copy_kib"] * 1024.0)
    w_scale = copy_bytes / (write["copy_kib"] * 1024.0)
    fetch_b = float(np.mean(fetch["fold_kib"])) * 1024.0 * f_scale
    write_b = float(np.mean(write["fold_kib"])) * 1024.0 * w_scale
    return {"source": "live rocprofv3 --pmc passes (FETCH_SIZE, then WRITE_SIZE) over one fold launch of this "
                      "workload, scaled by the same counters over a plain device copy",
            "fetch_kib_per_dispatch": fetch["fold_kib"], "write_kib_per_dispatch": write["fold_kib"],
            "copy_bytes": copy_bytes, "copy_fetch_kib": fetch["copy_kib"], "copy_write_kib": write["copy_kib"],
            "fetch_scale": f_scale, "write_scale": w_scale,
            "fetch_bytes_per_launch": fetch_b, "write_bytes_per_launch": write_b,
            "bytes_per_launch": fetch_b + write_b}


def committed_counters(workload: str, tuning: dict):
    """Counter figures committed under profiles/ for this workload, used only
    while the fold source and tuning still match the ones they were taken on."""
    path = os.path.join(ROOT, "profiles", f"fold_{workload}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        prof = json.load(fh)
    tun = [tuning[k] for k in ("fold_period_block", "fold_wgs_per_cu", "fold_units_per_wg", "fold_variant")]
    if prof.get("fold_source_sha256_16") != fold_source_hash() or prof.get("tuning") != tun:
        return None
    return {"source": f"profiles/fold_{workload}_counters.json (fold source hash and tuning match)",
            "bytes_per_launch": prof["hbm_bytes_per_launch"], "fetch_scale": prof.get("fetch_scale"),
            "write_scale": prof.get("write_scale")}


# ------------------------------------------------------------ host facts
def cpu_facts() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline(wl, fold_stride: int = 4000, st_lin_stride: int = 4000, st_periods: int = 4) -> dict:
    """The FP64 oracle, as it is, on a bounded sample of one curve of the
    workload, on every core OpenMP uses here: resampling and the linear search
    in full, the fold over every fold_stride-th period, extrapolated linearly
    in fold element visits (sum over periods of allowed durations x I) to the
    full grid.  Then the same on one thread: the linear search on every
    st_lin_stride-th element (extrapolated in elements) and the fold over
    st_periods evenly spaced periods (extrapolated in element visits)."""
    import oracle
    g = oracle.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, wl.n_model)
    model = oracle.template(wl.dense, wl.n_model)
    cores = oracle.max_threads()
    durs = np.asarray(wl.durations)
    jk = np.array([np.count_nonzero(durs < P) for P in wl.periods], dtype=np.float64)
    K = len(wl.periods)
    t0 = time.perf_counter()
    flux, ivar = oracle.resample(g, wl.t, wl.f, wl.sigma)
    t_res = time.perf_counter() - t0
    t0 = time.perf_counter()
    lin = oracle.linear(g, flux, ivar, model)
    t_lin = time.perf_counter() - t0
    sel = np.arange(fold_stride // 2, K, fold_stride)
    t0 = time.perf_counter()
    oracle.periodic(g, lin, wl.periods, sel=sel)
    t_fold = time.perf_counter() - t0
    scale = jk.sum() / jk[sel].sum()
    t_full = t_res + t_lin + t_fold * scale
    # one thread
    n_el = g.n_dur * g.n_t0
    idx = np.arange(0, n_el, st_lin_stride, dtype=np.int64)
    sel1 = np.linspace(0, K - 1, st_periods + 2)[1:-1].astype(np.int64)
    try:
        oracle.set_threads(1)
        t0 = time.perf_counter()
        oracle.linear_at(g, flux, ivar, model, idx)
        m_lin1 = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.periodic(g, lin, wl.periods, sel=sel1)
        m_fold1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(cores)
    t_lin1 = m_lin1 * n_el / len(idx)
    t_fold1 = m_fold1 * jk.sum() / jk[sel1].sum()
    t_full1 = t_res + t_lin1 + t_fold1
    units = wl.n_obs * K
    return dict(value=units / t_full, unit="LC points x trial periods / s", cores=cores, kind="oracle",
                sample=(f"one curve of the workload: resampling ({t_res:.2f} s) and the linear search "
                        f"({t_lin:.2f} s) in full, fold over every {fold_stride}th period ({len(sel)} of {K}, "
                        f"{t_fold:.2f} s) extrapolated x{scale:.0f} in fold element visits; estimated full "
                        f"search {t_full:.0f} s"),
                single_thread={"value": units / t_full1, "estimated_full_search_s": t_full1,
                               "sample": (f"linear search on every {st_lin_stride}th element, fold over "
                                          f"{len(sel1)} periods, each extrapolated as above")},
                seconds_measured=round(t_res + t_lin + t_fold + m_lin1 + m_fold1, 1),
                **cpu_facts())


# ------------------------------------------------------------ headline
def search_buffers(cm, torch, grid, K, dev="cuda"):
    return dict(fold=torch.empty((grid.n_dur, grid.n_t0, 2), dtype=torch.float32, device=dev),
                work=torch.empty(max(cm.periodic_workspace(grid, K), 1), dtype=torch.uint8, device=dev),
                per=dict(lr=torch.empty(K, dtype=torch.float32, device=dev),
                         epoch=torch.empty(K, dtype=torch.int32, device=dev),
                         dur=torch.empty(K, dtype=torch.int32, device=dev),
                         depth=torch.empty(K, dtype=torch.float32, device=dev),
                         depth_var=torch.empty(K, dtype=torch.float32, device=dev)),
                best=torch.empty(ctypes.sizeof(cm.BestRecord), dtype=torch.uint8, device=dev))


def timed_search(cm, torch, grid, curves, dense_d, per_d, n_model, bufs, steps: int, warmup: int) -> dict:
    """warmup untimed steps, then `steps` timed ones, step s on curve
    s mod len(curves) (each a (t, f, sigma) triple of device tensors); HIP
    events on the launch stream around every step and around its fold."""
    stream = torch.cuda.current_stream()
    fold, work, per, best = bufs["fold"], bufs["work"], bufs["per"], bufs["best"]
    names = ("start", "lin", "fold1", "end")
    ev = {k: [] for k in names}

    def step(s: int, record: bool):
        t_d, f_d, s_d = curves[s % len(curves)]
        e = {k: torch.cuda.Event(enable_timing=True) for k in names} if record else None
        if record:
            e["start"].record(stream)
        model = cm.template_resample(dense_d, n_model)
        flux, ivar, _ = cm.resample(grid, t_d, f_d, s_d, status=False)
        cm.linear_search(grid, flux, ivar, model, fold=fold)
        if record:
            e["lin"].record(stream)
        cm.periodic_search(grid, fold, per_d, work=work, out=per)
        if record:
            e["fold1"].record(stream)
        cm.best(grid, per_d, per, out=best)
        if record:
            e["end"].record(stream)
            for k in names:
                ev[k].append(e[k])

    for s in range(warmup):
        step(s, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        step(warmup + s, True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_steps = [ev["start"][i].elapsed_time(ev["end"][i]) for i in range(steps)]
    ms_lin = [ev["start"][i].elapsed_time(ev["lin"][i]) for i in range(steps)]
    ms_fold = [ev["lin"][i].elapsed_time(ev["fold1"][i]) for i in range(steps)]
    return dict(ms_step=float(np.mean(ms_steps)), ms_lin=float(np.mean(ms_lin)), ms_fold=float(np.mean(ms_fold)),
                wall=wall, best=cm.best_record(best), last_curve=(warmup + steps - 1) % len(curves))


def pcie_inclusive(cm, torch, grid, host_curve, dense_d, per_d, n_model, bufs, reps: int = 2) -> dict:
    """One step with the host transfers inside: t, f, sigma copied from
    pinned host memory, the search, and the per-period records plus the best
    record copied back to pinned host memory; mean of `reps` after one
    untimed run."""
    t_h, f_h, s_h = (torch.as_tensor(a).pin_memory() for a in host_curve)
    t_d, f_d, s_d = (torch.empty_like(a, device="cuda") for a in (t_h, f_h, s_h))
    per, best = bufs["per"], bufs["best"]
    out_h = {k: torch.empty(v.shape, dtype=v.dtype).pin_memory() for k, v in per.items()}
    best_h = torch.empty(best.shape, dtype=best.dtype).pin_memory()

    def run():
        for d, h in ((t_d, t_h), (f_d, f_h), (s_d, s_h)):
            d.copy_(h, non_blocking=True)
        model = cm.template_resample(dense_d, n_model)
        flux, ivar, _ = cm.resample(grid, t_d, f_d, s_d, status=False)
        cm.linear_search(grid, flux, ivar, model, fold=bufs["fold"])
        cm.periodic_search(grid, bufs["fold"], per_d, work=bufs["work"], out=per)
        cm.best(grid, per_d, per, out=best)
        for k, v in per.items():
            out_h[k].copy_(v, non_blocking=True)
        best_h.copy_(best, non_blocking=True)

    run()
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        run()
        b.record()
        b.synchronize()
        ms.append(a.elapsed_time(b))
    h2d = sum(x.numel() * x.element_size() for x in (t_h, f_h, s_h))
    d2h = sum(v.numel() * v.element_size() for v in out_h.values()) + best_h.numel()
    return {"ms_per_step": float(np.mean(ms)), "h2d_bytes": h2d, "d2h_bytes": d2h}


def high_cadence_block(steps: int = 5, warmup: int = 2) -> dict:
    """The 90-day, 20-s cadence curve (369 360 observations, red + white
    noise, pre-whitened, gaps; 20 durations 0.5-15 h; 50 000 periods
    0.5-45 d): the same timed step as the headline, with its fold rate in
    algorithmic bytes against the address-unit bound (the 70 MB fold-ready
    array is cache-resident), the linear search's FP32 rate, and the
    default-grid measurements on the same curve."""
    import torch
    import paper_2503_20875_amd as cm
    from synthlc import workloads as W
    wl = W.high_cadence()
    grid = cm.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, 0.0, wl.n_model)
    K = len(wl.periods)
    curves = [tuple(torch.as_tensor(a, device="cuda") for a in (wl.t, wl.f, wl.sigma))]
    bufs = search_buffers(cm, torch, grid, K)
    r = timed_search(cm, torch, grid, curves, torch.as_tensor(wl.dense, device="cuda"),
                     torch.as_tensor(wl.periods, device="cuda"), wl.n_model, bufs, steps, warmup)
    alg = algorithmic_work(wl, grid)
    fold_gbps = alg["fold_bytes"] / (r["ms_fold"] / 1e3) / 1e9
    lin_tf = alg["linear_flop"] / (r["ms_lin"] / 1e3) / 1e12
    del bufs
    return {"workload": (f"single light curve, 90 d at 20 s cadence, {wl.n_obs} observations (N = {grid.n}), "
                         f"J = {grid.n_dur} durations 0.5-15 h, I = {grid.n_t0}, K = {K} periods 0.5-45 d"),
            "value": wl.n_obs * K / (r["ms_step"] / 1e3), "unit": "LC points x trial periods / s",
            "ms_per_step": r["ms_step"], "steps": steps,
            "stages_ms": {"setup_and_linear": r["ms_lin"], "periodic": r["ms_fold"],
                          "best": r["ms_step"] - r["ms_lin"] - r["ms_fold"]},
            "roofline_address_unit": {"kernel": "fold_kernel (periodic search)", "achieved": fold_gbps,
                                      "peak": ADDRESS_UNIT_PEAK_GBS, "unit": "GB/s",
                                      "frac": fold_gbps / ADDRESS_UNIT_PEAK_GBS,
                                      "algorithmic_bytes_per_launch": alg["fold_bytes"]},
            "roofline_linear": {"kernel": "linear_kernel", "bound": "alu", "achieved": lin_tf,
                                "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                                "frac": lin_tf / FP32_VECTOR_PEAK_TFLOPS, "algorithmic_flop": alg["linear_flop"],
                                "avg_ms_incl_setup": r["ms_lin"]},
            "best": {"period": r["best"]["period"], "snr": r["best"]["snr"], "depth": r["best"]["depth"],
                     "duration": r["best"]["duration"]},
            "default_grids": keplerian_block()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="long_baseline", choices=["long_baseline", "high_cadence", "tiny"],
                    help="long_baseline (default): the Earth-analogue batch, one curve per step")
    ap.add_argument("--curves", type=int, default=8,
                    help="distinct curves of the Earth-analogue batch the steps cycle through")
    ap.add_argument("--no-extras", action="store_true",
                    help="time the benchmark steps only (no counters, secondary workloads, network, batched, "
                         "learned or CPU measurements), e.g. for kernel traces of the headline search")
    ap.add_argument("--no-counters", action="store_true", help="skip the live rocprofv3 counter passes")
    ap.add_argument("--mode", default="full", choices=["full", "fold", "copy", "net", "batch"],
                    help="full: the benchmark; fold: setup once, then an optional --copy-mib device copy and "
                         "--steps fold launches only (for counter runs); copy: a plain device copy of "
                         "--copy-mib MiB, --steps times; net: the proposal network's convolution roofline only; "
                         "batch: the batched-survey measurement only (--batch-curves curves)")
    ap.add_argument("--copy-mib", type=int, default=0)
    ap.add_argument("--batch-curves", type=int, default=64,
                    help="survey curves of the batched-search measurement (0: skip)")
    ap.add_argument("--batch-points", default="5000,120000",
                    help="length range (points) of the batched-search curves")
    ap.add_argument("--batch-compare", type=int, default=1,
                    help="with --mode batch: 0 times one eager batch only (no graph replay or single-curve "
                         "calls), with progress lines, and generates the curves with 8 processes")
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

    batch_pts = tuple(int(v) for v in args.batch_points.split(","))
    if args.mode == "batch":  # before any GPU call: its curve generator may fork
        print(json.dumps({"mode": "batch", **batched_block(args.batch_curves, n_min=batch_pts[0],
                                                           n_max=batch_pts[1], compare=bool(args.batch_compare),
                                                           workers=1 if args.batch_compare else 8)}),
              flush=True)
        return
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.mode == "copy":
        n = max(args.copy_mib, 1) * (1 << 20) // 4
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
    tuning = cm.get_tuning()
    tuning_str = ",".join(str(tuning[k]) for k in ("fold_period_block", "fold_wgs_per_cu", "fold_units_per_wg",
                                                     "fold_variant"))
    long = args.workload == "long_baseline"
    n_curves = max(1, min(args.curves, args.steps + args.warmup)) if long and args.mode == "full" else 1
    wls = [W.long_baseline(seed=LONG_SEED + c) for c in range(n_curves)] if long else [W.WORKLOADS[args.workload]()]
    wl = wls[0]
    dev = "cuda"
    grid = cm.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, 0.0, wl.n_model)
    K = len(wl.periods)
    for w in wls[1:]:  # the batch shares its time grid and period grid
        assert np.array_equal(w.t, wl.t) and np.array_equal(w.periods, wl.periods)
    curves = [tuple(torch.as_tensor(a, device=dev) for a in (w.t, w.f, w.sigma)) for w in wls]
    dense_d = torch.as_tensor(wl.dense, device=dev)
    per_d = torch.as_tensor(wl.periods, device=dev)
    bufs = search_buffers(cm, torch, grid, K)  # every buffer allocated before timing

    if args.mode == "fold":
        t_d, f_d, s_d = curves[0]
        model = cm.template_resample(dense_d, wl.n_model)
        flux, ivar, _ = cm.resample(grid, t_d, f_d, s_d, status=False)
        cm.linear_search(grid, flux, ivar, model, fold=bufs["fold"])
        if args.copy_mib > 0:
            n = args.copy_mib * (1 << 20) // 4
            src = torch.ones(n, dtype=torch.float32, device=dev)
            dst = torch.empty_like(src)
            dst.copy_(src)
            del src, dst
        for _ in range(args.steps):
            cm.periodic_search(grid, bufs["fold"], per_d, work=bufs["work"], out=bufs["per"])
        torch.cuda.synchronize()
        print(json.dumps({"mode": "fold", "launches": args.steps, "workload": args.workload, "tuning": tuning,
                          "fold_source_sha256_16": fold_source_hash(), "copy_mib": args.copy_mib,
                          "algorithmic_bytes_per_launch": algorithmic_work(wl, grid)["fold_bytes"]}), flush=True)
        return

    log(f"{args.workload}: {n_curves} curve(s) resident, {args.warmup} warm-up + {args.steps} timed steps")
    r = timed_search(cm, torch, grid, curves, dense_d, per_d, wl.n_model, bufs, args.steps, args.warmup)
    log(f"timed steps done: {r['ms_step']:.1f} ms per step")
    alg = algorithmic_work(wl, grid)
    fold_s = r["ms_fold"] / 1e3
    lin_s = r["ms_lin"] / 1e3
    alg_gbps = alg["fold_bytes"] / fold_s / 1e9
    value = wl.n_obs * K / (r["ms_step"] / 1e3)
    b = r["best"]
    if long:
        desc = (f"Earth-analogue batch of 64 curves, one curve per step (steps cycle through {n_curves} of them): "
                f"730.5 d at 25 s, {wl.n_obs} observations (N = {grid.n} resampled), J = {grid.n_dur} durations "
                f"1-20 h, I = {grid.n_t0} reference times, K = {K} periods 1-400 d")
    else:
        desc = (f"{wl.name}: {wl.n_obs} observations (N = {grid.n}), J = {grid.n_dur}, I = {grid.n_t0}, K = {K}")
    out = {
        "metric": "LC points x trials/sec (linear+periodic) on 1 GPU",
        "value": value,
        "unit": "LC points x trial periods / s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "n_obs": wl.n_obs, "n_grid": int(grid.n), "n_t0": int(grid.n_t0),
                   "n_durations": int(grid.n_dur), "n_periods": K, "n_model": wl.n_model,
                   "curves_cycled": n_curves},
    }
    counters, counter_note = None, None
    if not args.no_extras and not args.no_counters and not _under_profiler():
        try:
            log("live counter passes (FETCH_SIZE, WRITE_SIZE)")
            counters = live_counters(args.workload, tuning_str)
        except Exception as exc:  # a missing profiler is reported, never papered over
            counter_note = f"live counter passes failed: {exc}"
    if counters is None:
        counters = committed_counters(args.workload, tuning)
    traffic = counters["bytes_per_launch"] if counters else None
    achieved = traffic / fold_s / 1e9 if traffic else None
    out["roofline"] = {
        "kernel": "fold_kernel (periodic search)",
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS if achieved else None,
        "traffic": traffic,
        "basis": ("achieved = bytes the fold moves past L2 per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated; "
                  "they are served by the Infinity Cache or HBM) / the fold's mean launch time in the timed "
                  "steps; null when no counter figures for this exact fold source exist"),
        "counters": counters if counters else counter_note,
        "algorithmic_bytes_per_launch": alg["fold_bytes"],
        "algorithmic_GBps": alg_gbps,
        "traffic_over_algorithmic": traffic / alg["fold_bytes"] if traffic else None,
        "avg_launch_ms": fold_s * 1e3,
        "tuning": tuning,
        "fold_source_sha256_16": fold_source_hash(),
    }
    out["roofline_address_unit"] = {
        "kernel": "fold_kernel (periodic search)",
        "bound": "vector-memory address unit",
        "achieved": alg_gbps,
        "peak": ADDRESS_UNIT_PEAK_GBS,
        "unit": "GB/s",
        "frac": alg_gbps / ADDRESS_UNIT_PEAK_GBS,
        "derivation": ("peak = 64 B per clock per CU (a 16-byte-per-lane wave load, 1 KB, occupies the unit 16 "
                       "cycles) x 256 CUs x 2.4 GHz; achieved = algorithmic bytes (8 B per element visit + 20 B "
                       "per period) / mean launch time"),
    }
    out["roofline_linear"] = {
        "kernel": "linear_kernel (linear search, all durations)",
        "bound": "alu",
        "achieved": alg["linear_flop"] / lin_s / 1e12,
        "peak": FP32_VECTOR_PEAK_TFLOPS,
        "unit": "TFLOP/s",
        "frac": alg["linear_flop"] / lin_s / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
        "algorithmic_flop": alg["linear_flop"],
        "avg_ms_incl_setup": lin_s * 1e3,
    }
    out["stages_ms"] = {"setup_and_linear": r["ms_lin"], "periodic": r["ms_fold"],
                        "best": r["ms_step"] - r["ms_lin"] - r["ms_fold"]}
    out["wall_s_timed"] = r["wall"]
    out["best"] = {"period": b["period"], "snr": b["snr"], "depth": b["depth"], "duration": b["duration"],
                   "curve": r["last_curve"]}
    if args.no_extras:
        print(json.dumps(out), flush=True)
        return
    log("host-transfer-inclusive step")
    pc = pcie_inclusive(cm, torch, grid, (wl.t, wl.f, wl.sigma), dense_d, per_d, wl.n_model, bufs)
    out["pcie_inclusive"] = {**pc, "value": wl.n_obs * K / (pc["ms_per_step"] / 1e3),
                             "note": "t, f, sigma from pinned host memory and the per-period and best records "
                                     "back to it, inside the timed step"}
    del bufs, curves
    torch.cuda.empty_cache()
    if long:
        log("learned form on the Earth analogue")
        out["learned_long"] = learned_long_block(wl)
        log("monotransit search")
        out["monotransit"] = monotransit_block(wl)
        log("high-cadence curve")
        out["high_cadence"] = high_cadence_block()
    log("proposal network")
    out["roofline_net"] = net_block()
    if args.batch_curves > 0:
        log(f"batched survey ({args.batch_curves} curves)")
        out["batched"] = batched_block(args.batch_curves, n_min=batch_pts[0], n_max=batch_pts[1])
        log("batched short curves (1 024 curves of 5 000-10 000 points)")
        out["batched_short"] = batched_block(1024, seed=30250000, n_min=5000, n_max=10000)
    if args.learned_curves > 0:
        log(f"learned proposal ({args.learned_curves} held-out curves)")
        out["learned"] = learned_block(args.learned_curves)
    if not args.no_cpu_baseline:
        log("FP64 oracle on the host")
        out["cpu_baseline"] = cpu_baseline(wl)
    log("done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
