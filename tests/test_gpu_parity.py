"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on
the same seeded inputs.  Floating point within 1e-5 (floored relative error,
see parity.py); integer outputs (grid indices, argmax) identical outside
near-ties."""

import numpy as np
import pytest

from synthlc import transit, workloads as W

from parity import TOL, check_linear, check_periodic, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_20875_amd as cm
    cm._abi.load()  # raises if the HIP library is not built: no fallback
    return cm


def run_both(cm, ora, wl, t0_step=0.0, jrange=None, subset=None, oracle_sel=None):
    import torch
    print(f"[case] {wl.name} n_obs={wl.n_obs} J={len(wl.durations)} K={len(wl.periods)}", flush=True)
    r = cm.search(wl.t, wl.f, wl.sigma, wl.cadence, wl.durations, wl.periods, wl.dense,
                  n_model=wl.n_model, t0_step=t0_step, public=True, jrange=jrange, subset=subset)
    torch.cuda.synchronize()
    o = ora.search(wl, t0_step=t0_step, jrange=jrange, sel=oracle_sel)
    g = {k: v.cpu().numpy() for k, v in r["periodic"].items()}
    return r, o, g


def lin_arrays(r):
    return r["depth"].cpu().numpy(), r["var"].cpu().numpy(), r["lr"].cpu().numpy()


def fold_at(ora, o):
    return lambda P, i, j: ora.fold_at(o["grid"], o["linear"], P, i, j)


# ------------------------------------------------------------------ setup stages
@pytest.mark.parametrize("n_dense,M", [(4097, 1024), (101, 7), (2, 64), (16385, 4096)])
def test_template_resample_bit_exact(cm, ora, n_dense, M):
    import torch
    dense = transit.dense_template(n_dense) if n_dense > 2 else np.array([0.25, 1.0])
    g = cm.template_resample(torch.as_tensor(dense, device="cuda"), M).cpu().numpy()
    assert np.array_equal(g, ora.template(dense, M))


@pytest.mark.parametrize("seed", [0, 5])
def test_resample_matches_oracle(cm, ora, seed):
    wl = W.small_random(seed, n_obs=3000, dup_frac=0.3)
    grid = cm.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations)
    flux, ivar, st = cm.resample(grid, wl.t, wl.f, wl.sigma)
    og = ora.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations)
    of, oi = ora.resample(og, wl.t, wl.f, wl.sigma)
    assert int(st.item()) == 0
    f, i = flux.cpu().numpy(), ivar.cpu().numpy()
    assert np.array_equal(i > 0, oi > 0)
    assert np.max(rel(i[oi > 0], oi[oi > 0])) < 1e-6
    # FP32 output of an FP64 mean: one rounding
    assert np.max(np.abs(f - of) / np.maximum(np.abs(of), 1e-30)) < 1e-6


def test_resample_flags_unsorted_input(cm):
    wl = W.small_random(1, n_obs=400)
    t = wl.t.copy()
    t[[10, 11]] = t[[11, 10]]
    grid = cm.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations)
    _, _, st = cm.resample(grid, t, wl.f, wl.sigma)
    assert int(st.item()) == 1


def test_loglike0_matches_oracle(cm, ora):
    wl = W.tiny_single()
    grid = cm.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations)
    flux, ivar, _ = cm.resample(grid, wl.t, wl.f, wl.sigma)
    l0 = float(cm.loglike0(grid, flux, ivar).item())
    og = ora.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations)
    of, oi = ora.resample(og, wl.t, wl.f, wl.sigma)
    assert l0 == pytest.approx(ora.loglike0(og, of, oi), rel=1e-6)


# ------------------------------------------------- full search, tiny workload
@pytest.fixture(scope="module")
def tiny_wl():
    return W.tiny_single()


@pytest.fixture(scope="module")
def tiny_pair(cm, ora, tiny_wl):
    return run_both(cm, ora, tiny_wl)


def test_tiny_linear_all_elements(tiny_pair):
    r, o, _ = tiny_pair
    res = check_linear(*lin_arrays(r), o["linear"])
    print("linear", res)
    # fold-ready pairs: (S_fm, S_mm) = (depth/var, 1/var)
    fold = r["fold"].cpu().numpy().astype(np.float64)
    lin = o["linear"]
    ok = np.isfinite(lin["var"])
    assert np.all(fold[~ok] == 0)
    assert np.max(rel(fold[..., 1][ok], 1 / lin["var"][ok])) < TOL
    assert np.max(rel(fold[..., 0][ok], lin["depth"][ok] / lin["var"][ok], lin["aabs"][ok])) < TOL


def test_linear_long_windows_read_from_memory(cm, ora):
    """Windows too long to stage in LDS (46 h at 20 s: the span of 256
    windows exceeds 64 KB) are summed from global memory: every linear
    element and every period against the oracle."""
    wl = W.small_random(3, n_obs=30000, cadence_s=20.0, n_dur=2, n_per=6, p_range=(3.0, 5.0), dur_h=(2.0, 38.0))
    r, o, g = run_both(cm, ora, wl)
    og = o["grid"]
    Wl = cm.get_tuning()["linear_windows"]
    table = 4 * ((wl.n_model + 5) & ~1)
    span_pairs = ((256 * Wl - 1) * og.t0_step + wl.durations[-1]) / og.cadence + 4
    assert span_pairs * 8 + table > 64 * 1024  # the longest duration takes the direct path
    assert (((256 * Wl - 1) * og.t0_step + wl.durations[0]) / og.cadence + 4) * 8 + table < 64 * 1024  # staged
    print("linear", check_linear(*lin_arrays(r), o["linear"]))
    print("periodic", check_periodic(g, o["periodic"], fold_at(ora, o), wl.periods))


@pytest.mark.parametrize("name", ["tiny", "long_windows"])
def test_linear_windows_per_lane_identical(cm, name):
    """One, two or four windows per lane (tiles of 256 to 1 024 reference
    times) give the same fold-ready pairs and public arrays, bit for bit:
    FP32 partial sums cover aligned 32-point blocks whatever the tile, and
    lanes with a null window walk each window alone in the same blocks."""
    import torch
    wl = W.tiny_single() if name == "tiny" else W.small_random(
        3, n_obs=30000, cadence_s=20.0, n_dur=2, n_per=6, p_range=(3.0, 5.0), dur_h=(2.0, 38.0))
    grid = cm.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, 0.0, wl.n_model)
    model = cm.template_resample(torch.as_tensor(wl.dense, device="cuda"), wl.n_model)
    flux, ivar, _ = cm.resample(grid, wl.t, wl.f, wl.sigma)
    out = {}
    try:
        for Wl in (4, 2, 1):
            print(f"[case] {name} linear_windows={Wl}", flush=True)
            cm.set_tuning(linear_windows=Wl)
            res = cm.linear_search(grid, flux, ivar, model, public=True)
            torch.cuda.synchronize()
            out[Wl] = [x.cpu().numpy() for x in res]
    finally:
        cm.reset_tuning()
    for Wl in (2, 1):
        for a, b in zip(out[Wl], out[4]):
            assert np.array_equal(a, b, equal_nan=True), Wl


def test_tiny_periodic_all_periods(ora, tiny_pair, tiny_wl):
    r, o, g = tiny_pair
    res = check_periodic(g, o["periodic"], fold_at(ora, o), tiny_wl.periods)
    print("periodic", res)


def test_tiny_best(cm, ora, tiny_pair, tiny_wl):
    r, o, g = tiny_pair
    b = cm.best_record(r["best_raw"])
    kb = o["best"]
    if b["k"] != kb:  # near-tie across periods
        lo, lg = o["periodic"]["lr"][kb], o["periodic"]["lr"][b["k"]]
        assert (lo - lg) <= TOL * lo
    p = o["periodic"]
    k = b["k"]
    assert b["lr"] == pytest.approx(float(g["lr"][k]))
    assert b["snr"] == pytest.approx(p["z"][k] / np.sqrt(p["zvar"][k]), rel=1e-5)
    assert b["t0"] == pytest.approx(g["epoch"][k] * o["grid"].t0_step)
    assert b["t0_abs"] == pytest.approx(o["grid"].t_origin + b["t0"])
    inj = tiny_wl.injections[0]
    assert abs(b["period"] / inj.period - 1) < 0.01


def test_lr_nonnegative_everywhere(tiny_pair):
    r, _, g = tiny_pair
    assert float(r["lr"].min().item()) >= 0
    assert np.all(g["lr"] >= 0)


# --------------------------------------------------------------- edge cases
def _edge(name, seed=3, **kw):
    wl = W.small_random(seed, **kw)
    wl.name = name
    return wl


def test_edge_ragged_small(cm, ora):
    """Few hundred epochs (not a multiple of the 256-lane tile), irregular."""
    wl = _edge("ragged", n_obs=211, n_dur=3, n_per=17)
    r, o, g = run_both(cm, ora, wl, t0_step=0.0371 * wl.durations[0])
    assert r["grid"].n_t0 % 256 != 0
    check_linear(*lin_arrays(r), o["linear"])
    check_periodic(g, o["periodic"], fold_at(ora, o), wl.periods)


def test_edge_data_shorter_than_windows(cm, ora):
    """Six points spanning 1 h, durations 5-10 h: the padding of half the
    longest duration keeps windows inside the grid, every period is longer
    than the grid, so each period reduces to the linear search's maximum."""
    wl = _edge("short", n_obs=6, n_dur=2, n_per=4, dup_frac=0, gap_frac=0, dur_h=(5.0, 8.0),
               p_range=(2.0, 3.0))
    r, o, g = run_both(cm, ora, wl)
    d, v, l = lin_arrays(r)
    check_linear(d, v, l, o["linear"])
    check_periodic(g, o["periodic"], fold_at(ora, o), wl.periods)
    flat = o["linear"]["lr"].reshape(-1)
    jb, ib = divmod(int(np.argmax(flat)), r["grid"].n_t0)
    assert np.all(g["epoch"] == ib) and np.all(g["dur"] == jb)


def test_edge_all_missing(cm, ora):
    wl = _edge("all-missing", n_obs=300)
    wl.sigma = np.full_like(wl.sigma, np.nan)
    r, o, g = run_both(cm, ora, wl)
    assert float(r["ivar"].abs().max().item()) == 0
    assert np.all(g["epoch"] == -1)
    assert cm.best_record(r["best_raw"])["k"] == -1


def test_edge_box_template_single_duration(cm, ora):
    wl = _edge("box", n_obs=800, n_dur=1, n_per=9)
    wl.n_model = 1
    r, o, g = run_both(cm, ora, wl)
    check_linear(*lin_arrays(r), o["linear"])
    check_periodic(g, o["periodic"], fold_at(ora, o), wl.periods)


def test_edge_periods_shorter_than_durations(cm, ora):
    """D_j < P_k is required: periods below the shortest duration are null,
    intermediate ones only use the shorter durations."""
    wl = _edge("short-periods", n_obs=900, n_dur=4, n_per=10, dur_h=(2.0, 8.0))
    wl.periods = np.sort(np.concatenate([[0.05, 0.09], np.geomspace(0.12, 0.5, 8), [1.3]]))
    r, o, g = run_both(cm, ora, wl)
    assert g["epoch"][0] == -1
    check_periodic(g, o["periodic"], fold_at(ora, o), wl.periods)
    for k, P in enumerate(wl.periods):
        if g["dur"][k] >= 0:
            assert wl.durations[g["dur"][k]] < P


def test_edge_subset_and_jrange(cm, ora):
    wl = _edge("subset", n_obs=1200, n_dur=4, n_per=40)
    rng = np.random.default_rng(0)
    jr = np.stack([rng.integers(0, 2, 40), rng.integers(1, 4, 40)], axis=1).astype(np.int32)
    sub = np.sort(rng.choice(40, 13, replace=False)).astype(np.int64)
    r, o, g = run_both(cm, ora, wl, jrange=jr, subset=sub, oracle_sel=sub)
    check_periodic(g, o["periodic"], fold_at(ora, o), wl.periods, sel=sub)
    rest = np.setdiff1d(np.arange(40), sub)
    assert np.all(g["epoch"][rest] == -1) and np.all(np.isnan(g["depth"][rest]))
    for k in sub:
        if g["dur"][k] >= 0:
            assert jr[k, 0] <= g["dur"][k] <= jr[k, 1]


def test_noiseless_injection_recovered_exactly(cm, ora):
    """Exact injection on the resampled grid: GPU returns depth A and the
    injected (period, epoch, duration) like the oracle."""
    from oracle import bruteforce as bf
    rng = np.random.default_rng(3)
    c = 301.7 / 86400
    n = 2000
    t = np.arange(n) * c + 0.4
    sig = (5e-4 * np.exp(0.3 * rng.normal(size=n))).astype(np.float32)
    durs = np.array([0.9137, 1.7093, 2.6351]) / 24
    periods = np.sort(rng.uniform(0.55, 2.4, 25))
    dense = transit.dense_template(1025)
    M = 256
    step = 0.0537 * durs[0]
    og = ora.grid_plan(t[0], t[-1], c, durs, M, t0_step=step)
    bg = bf.BruteGrid(t[0], t[-1], c, durs, M, t0_step=step)
    model = ora.template(dense, M)
    kstar, jstar = 12, 2
    istar = int(rng.integers(0, bg.epochs_per_period(periods[kstar])))
    A = 2.0 ** -10
    vec = np.zeros(bg.N)
    for x in bg.transit_epochs(istar, periods[kstar]):
        gx = bg.window_model(x, jstar, model)
        if gx is not None:
            vec += A * gx
    f = vec[og.n_pad: og.n_pad + n].astype(np.float32)
    wl = W.Workload("noiseless", t, f, sig, c, durs, periods, dense, n_model=M)
    r, o, g = run_both(cm, ora, wl, t0_step=step)
    assert (g["epoch"][kstar], g["dur"][kstar]) == (istar, jstar)
    assert g["depth"][kstar] == pytest.approx(A, rel=1e-6)
    b = cm.best_record(r["best_raw"])
    assert b["k"] == kstar


# ------------------------------------------- full-size high-cadence workload
def test_high_cadence_full_size_sampled(cm, ora):
    """90 d at 20 s (N = 391 500, I = 435 001, J = 20, K = 50 000) in the
    benchmark's launch configuration.  Linear search: 20 000 sampled elements
    recomputed one by one by the oracle.  Periodic search: 300 sampled periods
    against the oracle's fold over its own full linear search."""
    import torch
    wl = W.high_cadence()
    print(f"[case] {wl.name}", flush=True)
    r = cm.search(wl.t, wl.f, wl.sigma, wl.cadence, wl.durations, wl.periods, wl.dense, public=True)
    torch.cuda.synchronize()
    og = ora.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, wl.n_model)
    model = ora.template(wl.dense, wl.n_model)
    of, oi = ora.resample(og, wl.t, wl.f, wl.sigma)
    rng = np.random.default_rng(1)
    idx = rng.integers(0, og.n_dur * og.n_t0, 20000)
    samp = ora.linear_at(og, of, oi, model, idx)
    d, v, l = (a.reshape(-1)[idx] for a in lin_arrays(r))
    res = check_linear(d, v, l, samp)
    print("linear sample", res)
    lin = ora.linear(og, of, oi, model)
    sel = np.unique(np.concatenate([rng.choice(len(wl.periods), 280, replace=False),
                                    np.arange(0, 50000, 2500)]))
    per = ora.periodic(og, lin, wl.periods, sel=sel)
    g = {k: v.cpu().numpy() for k, v in r["periodic"].items()}
    res = check_periodic(g, per, lambda P, i, j: ora.fold_at(og, lin, P, i, j), wl.periods, sel=sel)
    print("periodic sample", res)
    # the duration-scaled epoch grid (1% of each duration) on the same arrays
    st = cm.epoch_strides(r["grid"], 0.01)
    per_s = cm.periodic_search(r["grid"], r["fold"], wl.periods, stride=st)
    gs = {k: v.cpu().numpy() for k, v in per_s.items()}
    ps = ora.periodic(og, lin, wl.periods, sel=sel, stride=st)
    print("strided sample", check_periodic(gs, ps, lambda P, i, j: ora.fold_at(og, lin, P, i, j), wl.periods,
                                           sel=sel))
    check_on_coarse_grid(gs, st)
    b = cm.best_record(r["best_raw"])
    # one of the two injected signals (17.1 d or 3.2 d), or an alias, is the strongest
    assert min(abs(b["period"] / (P * f) - 1) for P in (17.1, 3.2) for f in (0.5, 1, 2)) < 0.01
    alt = ora.fold_at(og, lin, b["period"], b["epoch"], b["dur"])
    assert b["lr"] == pytest.approx(alt[0], rel=TOL)


def test_long_baseline_full_size_sampled(cm, ora):
    """Earth analogue, 730.5 d at 25 s (2 524 608 points, I = 1 755 200,
    J = 30, K = 399 404; the fold-ready array is 421 MB) in the benchmark's
    launch configuration.  Linear search: 20 000 sampled elements recomputed
    one by one by the oracle.  Periodic search: 48 sampled periods, the
    periods around the injected 365.25 d and its half, and the shortest and
    longest, against the oracle's fold over its own full linear search; the
    best period is the injected one."""
    import torch
    wl = W.long_baseline()
    print(f"[case] {wl.name} K={len(wl.periods)}", flush=True)
    r = cm.search(wl.t, wl.f, wl.sigma, wl.cadence, wl.durations, wl.periods, wl.dense, public=True)
    torch.cuda.synchronize()
    og = ora.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, wl.n_model)
    model = ora.template(wl.dense, wl.n_model)
    of, oi = ora.resample(og, wl.t, wl.f, wl.sigma)
    rng = np.random.default_rng(2)
    idx = rng.integers(0, og.n_dur * og.n_t0, 20000)
    samp = ora.linear_at(og, of, oi, model, idx)
    d, v, l = (a.reshape(-1)[idx] for a in lin_arrays(r))
    print("linear sample", check_linear(d, v, l, samp), flush=True)
    lin = ora.linear(og, of, oi, model)
    K = len(wl.periods)
    near = [np.searchsorted(wl.periods, P) + o for P in (365.25, 182.625) for o in (-2, -1, 0, 1)]
    sel = np.unique(np.concatenate([rng.choice(K, 48, replace=False), near, [0, 1, K - 2, K - 1]]))
    per = ora.periodic(og, lin, wl.periods, sel=sel)
    g = {k: v.cpu().numpy() for k, v in r["periodic"].items()}
    res = check_periodic(g, per, lambda P, i, j: ora.fold_at(og, lin, P, i, j), wl.periods, sel=sel)
    print("periodic sample", res)
    b = cm.best_record(r["best_raw"])
    assert abs(b["period"] / 365.25 - 1) < 0.002
    alt = ora.fold_at(og, lin, b["period"], b["epoch"], b["dur"])
    assert b["lr"] == pytest.approx(alt[0], rel=TOL)


@pytest.mark.parametrize("cfg", [(8, 8, 4, 0), (4, 8, 16, 0), (16, 8, 4, 0), (4, 8, 4, 2), (8, 8, 4, 2),
                                 (16, 8, 4, 2), (8, 2, 1, 2)])
def test_fold_variants_identical(cm, ora, tiny_pair, tiny_wl, cfg):
    """Both fold variants, period blocks 4 to 16: the same
    per-period records, bit for bit (the FP32 ranking sums are accumulated in
    the same order), and parity with the oracle."""
    import torch
    r, o, g = tiny_pair
    cm.set_tuning(*cfg)
    try:
        per = cm.periodic_search(r["grid"], r["fold"], tiny_wl.periods)
        torch.cuda.synchronize()
    finally:
        cm.reset_tuning()
    h = {k: v.cpu().numpy() for k, v in per.items()}
    for k in ("lr", "epoch", "dur", "depth", "depth_var"):
        assert np.array_equal(h[k], g[k], equal_nan=True), (cfg, k)
    check_periodic(h, o["periodic"], fold_at(ora, o), tiny_wl.periods)


def mixed_periods(seed=11):
    """Periods that drive every path of the fold on the tiny grid
    (27.4 d, durations 0.5-6 h): 160 close periods of 0.12-0.3 d (90-230
    transits, several FP32 chunks, narrow windows that fit a wave's LDS
    buffer; the shortest exclude the longer durations), 120 periods of
    0.5-13 d (windows that outgrow the buffer after a few transits), and 40
    in random order (period blocks with widely different steps)."""
    rng = np.random.default_rng(seed)
    short = 1.0 / np.linspace(1 / 0.12, 1 / 0.3, 160)[::-1]
    mid = 1.0 / np.linspace(1 / 0.5, 1 / 13.0, 120)[::-1]
    loose = rng.uniform(0.15, 13.0, 40)
    return np.concatenate([short, mid, loose])


@pytest.mark.parametrize("B", [4, 8, 16])
def test_fold_variants_identical_mixed_periods(cm, ora, tiny_pair, B):
    """Every fold variant returns the records of the default variant bit for
    bit on mixed periods with a duration-range restriction, and those
    records match the oracle."""
    import torch
    r, o, _ = tiny_pair
    periods = mixed_periods()
    K = len(periods)
    rng = np.random.default_rng(5)
    jr = np.stack([rng.integers(0, 3, K), rng.integers(4, 8, K)], axis=1).astype(np.int32)
    print(f"[case] mixed periods K={K} B={B}", flush=True)
    out = {}
    try:
        for v in (2, 0):
            cm.set_tuning(B, 8, 4, v)
            per = cm.periodic_search(r["grid"], r["fold"], periods, jrange=jr)
            torch.cuda.synchronize()
            out[v] = {k: x.cpu().numpy() for k, x in per.items()}
    finally:
        cm.reset_tuning()
    for v in (0,):
        for k in ("lr", "epoch", "dur", "depth", "depth_var"):
            assert np.array_equal(out[v][k], out[2][k], equal_nan=True), (B, v, k)
    if B == 8:
        op = ora.periodic(o["grid"], o["linear"], periods, jrange=jr)
        for v in (0, 2):
            check_periodic(out[v], op, fold_at(ora, o), periods)
            for k in range(K):
                if out[v]["dur"][k] >= 0:
                    assert jr[k, 0] <= out[v]["dur"][k] <= jr[k, 1]


def check_on_coarse_grid(h, st):
    for k in range(len(h["epoch"])):
        if h["epoch"][k] >= 0:
            assert h["epoch"][k] % st[h["dur"][k]] == 0, (k, h["epoch"][k], h["dur"][k])


@pytest.mark.parametrize("B", [4, 8, 16])
def test_strided_fold_matches_oracle(cm, ora, tiny_pair, tiny_wl, B):
    """Duration-scaled epoch grid (strides 1 to 34, one far above any
    period's epoch count) against the oracle on the same grid, for every
    period block; unit strides return the plain search bit for bit."""
    import torch
    r, o, g = tiny_pair
    J = o["grid"].n_dur
    st = np.array([1, 2, 3, 5, 8, 13, 34, 10**6][:J], dtype=np.int32)
    print(f"[case] strided tiny B={B} strides={st.tolist()}", flush=True)
    cm.set_tuning(B, 8, 4, 2)
    try:
        per = cm.periodic_search(r["grid"], r["fold"], tiny_wl.periods, stride=st)
        ones = cm.periodic_search(r["grid"], r["fold"], tiny_wl.periods, stride=np.ones(J, dtype=np.int32))
        torch.cuda.synchronize()
    finally:
        cm.reset_tuning()
    h = {k: v.cpu().numpy() for k, v in per.items()}
    op = ora.periodic(o["grid"], o["linear"], tiny_wl.periods, stride=st)
    print("strided", check_periodic(h, op, fold_at(ora, o), tiny_wl.periods))
    check_on_coarse_grid(h, st)
    assert np.any(h["dur"] >= 1)  # winners on strided rows too
    h1 = {k: v.cpu().numpy() for k, v in ones.items()}
    for k in h1:
        assert np.array_equal(h1[k], g[k], equal_nan=True), k


def test_strided_fold_mixed_periods_and_ranges(cm, ora, tiny_pair):
    """Strided fold on the mixed period set with duration-range
    restrictions and a subset of the periods, against the oracle."""
    import torch
    r, o, _ = tiny_pair
    periods = mixed_periods()
    K = len(periods)
    rng = np.random.default_rng(9)
    jr = np.stack([rng.integers(0, 3, K), rng.integers(4, 8, K)], axis=1).astype(np.int32)
    sub = np.sort(rng.choice(K, K // 2, replace=False))
    st = cm.epoch_strides(r["grid"], 0.04)
    assert st.max() > 1
    print(f"[case] strided mixed periods K={K} strides={st.tolist()}", flush=True)
    per = cm.periodic_search(r["grid"], r["fold"], periods, jrange=jr, subset=sub, stride=st)
    torch.cuda.synchronize()
    h = {k: v.cpu().numpy() for k, v in per.items()}
    op = ora.periodic(o["grid"], o["linear"], periods, jrange=jr, sel=sub, stride=st)
    print("strided mixed", check_periodic(h, op, fold_at(ora, o), periods, sel=sub))
    check_on_coarse_grid(h, st)
    rest = np.setdiff1d(np.arange(K), sub)
    assert np.all(h["epoch"][rest] == -1)


def test_strided_fold_rejects_bad_strides(cm, tiny_pair, tiny_wl):
    r, o, _ = tiny_pair
    J = o["grid"].n_dur
    with pytest.raises(cm.CetraError, match="stride"):
        cm.periodic_search(r["grid"], r["fold"], tiny_wl.periods, stride=np.zeros(J, dtype=np.int32))
    with pytest.raises(ValueError):
        cm.periodic_search(r["grid"], r["fold"], tiny_wl.periods, stride=np.ones(J + 1, dtype=np.int32))


def test_keplerian_duration_filter(cm, ora, tiny_wl):
    """The fold restricted to each period's Keplerian durations (Sun-like
    densities 0.5-3 g/cm^3, k <= 0.2, b <= 0.9): the library's ranges equal
    the grid oracle's, and the records match the oracle's fold under the
    same ranges.  Periods whose range is empty get the null record."""
    from oracle import grids as og
    wl = tiny_wl
    jr = cm.keplerian_jrange(wl.periods, wl.durations, 0.5, 3.0, 0.2, 0.9)
    assert np.array_equal(jr, og.keplerian_jrange(wl.periods, wl.durations, 0.5, 3.0, 0.2, 0.9))
    assert np.any(jr[:, 0] > 0) and np.any(jr[:, 1] < len(wl.durations) - 1)
    r, o, g = run_both(cm, ora, wl, jrange=jr)
    check_periodic(g, o["periodic"], fold_at(ora, o), wl.periods)
    for k in range(len(wl.periods)):
        if g["dur"][k] >= 0:
            assert jr[k, 0] <= g["dur"][k] <= jr[k, 1]
        else:
            assert jr[k, 0] > jr[k, 1] or wl.durations[jr[k, 0]] >= wl.periods[k]


def test_period_range_edges_match_oracle(cm, ora):
    """Periods below the reference-time step (some longer than the shortest
    duration), non-finite or non-positive periods get the null record on both
    sides; a period of exactly one step and periods of at least I steps (one
    transit per epoch, up to 1e30 d) are evaluated identically."""
    wl = W.small_random(5, n_obs=600, n_dur=3, n_per=4, p_range=(0.5, 1.0), dur_h=(0.6, 2.0))
    step = 1.7 * wl.durations[0]
    g0 = ora.grid_plan(wl.t[0], wl.t[-1], wl.cadence, wl.durations, wl.n_model, t0_step=step)
    span = g0.n_t0 * step
    wl.periods = np.array([0.5 * step, step * (1 - 1e-9), 1.2 * wl.durations[0], float("nan"), float("inf"),
                           -1.0, 0.0, step, span * 1.0000001, span * 4.0, 1e30, 0.7, 0.9])
    r, o, g = run_both(cm, ora, wl, t0_step=step)
    assert np.all(g["epoch"][:7] == -1) and np.all(g["lr"][:7] == 0) and np.all(np.isinf(g["depth_var"][:7]))
    assert np.all(g["epoch"][7:] >= 0)
    check_periodic(g, o["periodic"], fold_at(ora, o), wl.periods)
