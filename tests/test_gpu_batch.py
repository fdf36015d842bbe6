"""Batched search (one persistent work-queue launch): results bit-identical
to single-curve calls on a batch with edge cases (a two-point curve, a curve
with every point missing, a curve without periods), whatever the queue order
or period block, on every replay of a captured HIP graph, and after a
cancelled search is resumed; per-curve parity with the FP64 oracle; host-set
failure conditions (a workspace without the plan's tables, unsorted times)
end in status bits, never in a hang."""

import threading
import time

import numpy as np
import pytest

from synthlc import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2503_20875_amd as cm
    cm._abi.load()
    return cm


def make_batch(n=10, seed=7, thin=25):
    curves = W.batched_survey(n, seed=seed, n_min=2000, n_max=15000)
    for c in curves:
        c.periods = c.periods[::thin].copy()
    # edge cases: a 2-point curve, an all-missing curve, a curve with no periods
    tiny = curves[1]
    tiny.t, tiny.f, tiny.sigma = tiny.t[:2].copy(), tiny.f[:2].copy(), tiny.sigma[:2].copy()
    curves[2].sigma = np.full_like(curves[2].sigma, np.nan)
    curves[3].periods = np.zeros(0)
    return curves


def pack(cm, curves):
    grids = [cm.grid_plan(c.t[0], c.t[-1], c.cadence, c.durations, 0.0, c.n_model) for c in curves]
    obs_off = np.concatenate([[0], np.cumsum([c.n_obs for c in curves])])
    per_off = np.concatenate([[0], np.cumsum([len(c.periods) for c in curves])])
    t = np.concatenate([c.t for c in curves])
    f = np.concatenate([c.f for c in curves])
    s = np.concatenate([c.sigma for c in curves])
    p = np.concatenate([c.periods for c in curves]) if per_off[-1] else np.zeros(1)
    return grids, obs_off, per_off, t, f, s, p


def single_results(cm, curves, model):
    import torch
    out = []
    print(f"[single] {len(curves)} curves", flush=True)
    for c in curves:
        r = {}
        if len(c.periods):
            res = cm.search(c.t, c.f, c.sigma, c.cadence, c.durations, c.periods, c.dense, n_model=c.n_model)
            torch.cuda.synchronize()
            r = {k: v.cpu().numpy() for k, v in res["periodic"].items()}
            r["best"] = cm.best_record(res["best_raw"])
        out.append(r)
    return out


def batch_results(cm, plan, curves, packed, model, **kw):
    import torch
    grids, obs_off, per_off, t, f, s, p = packed
    print(f"[batch] curves={plan.n_curves} launches={plan.info['n_launches']} kw={sorted(kw)}", flush=True)
    o = cm.batch_search(plan, t, f, s, model, p, **kw)
    torch.cuda.synchronize()
    print(f"[batch] done status={int(o['status'].item())}", flush=True)
    return o


def records(o):
    return {k: v.cpu().numpy() for k, v in o.items() if k not in ("best", "status", "done")}


def compare(cm, o, single, per_off):
    h = records(o)
    bests = cm.best_records(o["best"])
    assert np.all(o["done"].cpu().numpy() == 1)
    for ci, r in enumerate(single):
        sl = slice(per_off[ci], per_off[ci + 1])
        if not r:
            assert bests[ci]["k"] == -1
            continue
        for k in ("lr", "epoch", "dur", "depth", "depth_var"):
            assert np.array_equal(h[k][sl], r[k], equal_nan=True), (ci, k)
        b, sb = bests[ci], r["best"]
        for k in ("k", "epoch", "dur", "lr", "depth", "depth_var", "snr", "t0", "t0_abs", "period"):
            assert (b[k] == sb[k]) or (np.isnan(b[k]) and np.isnan(sb[k])), (ci, k, b[k], sb[k])


@pytest.fixture(scope="module")
def setup(cm):
    import torch
    curves = make_batch()
    model = cm.template_resample(torch.as_tensor(curves[0].dense, device="cuda"), curves[0].n_model)
    packed = pack(cm, curves)
    single = single_results(cm, curves, model)
    return curves, model, packed, single


def test_batch_equals_single_bitwise(cm, setup):
    curves, model, packed, single = setup
    grids, obs_off, per_off = packed[:3]
    plan = cm.batch_plan(grids, obs_off, per_off)
    assert plan.info["n_launches"] == 2
    o = batch_results(cm, plan, curves, packed, model)
    assert int(o["status"].item()) == 0
    compare(cm, o, single, per_off)


@pytest.mark.parametrize("shuffle,block,pop", [(12345, 0, 0), (0, 4, 1), (777, 4, 3), (0, 0, 64)])
def test_batch_order_and_block_do_not_change_results(cm, setup, shuffle, block, pop):
    """A seeded queue order, another period block or another run length per
    queue pop interleaves the curves' items differently; every record stays
    bit-identical."""
    curves, model, packed, single = setup
    grids, obs_off, per_off = packed[:3]
    plan = cm.batch_plan(grids, obs_off, per_off, period_block=block, shuffle_seed=shuffle, pop_items=pop)
    o = batch_results(cm, plan, curves, packed, model)
    assert int(o["status"].item()) == 0
    compare(cm, o, single, per_off)


def test_batch_graph_replay(cm, setup):
    """Capture the whole batch in a HIP graph; every replay, with eager work
    in between, equals the single-curve results."""
    import torch
    curves, model, packed, single = setup
    grids, obs_off, per_off, t, f, s, p = packed
    plan = cm.batch_plan(grids, obs_off, per_off)
    td, fd, sd, pd = (torch.as_tensor(x, device="cuda") for x in (t, f, s, p))
    work = cm.batch_workspace(plan)
    o = cm.batch_search(plan, td, fd, sd, model, pd, work=work)
    torch.cuda.synchronize()
    assert int(o["status"].item()) == 0
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            cm.batch_search(plan, td, fd, sd, model, pd, work=work, out=o)
    torch.cuda.current_stream().wait_stream(side)
    for rep in range(3):
        for k in ("lr", "depth"):
            o[k].fill_(-7.0)
        o["status"].fill_(5)
        print(f"[batch] graph replay {rep}", flush=True)
        g.replay()
        torch.cuda.synchronize()
        assert int(o["status"].item()) == 0
        compare(cm, o, single, per_off)
        _ = (torch.randn(1000, device="cuda") ** 2).sum().item()  # eager work between replays


def test_batch_matches_oracle(cm, ora, setup):
    """Every curve of the batch, edge cases included, against the FP64
    oracle run on that curve alone: per-period records to the parity bar
    (floored 1e-5, argmax identical outside near-ties) and the best period."""
    import sys
    import os
    sys.path.insert(0, os.path.dirname(__file__))
    from parity import TOL, check_periodic
    curves, model, packed, _ = setup
    grids, obs_off, per_off = packed[:3]
    plan = cm.batch_plan(grids, obs_off, per_off)
    o = batch_results(cm, plan, curves, packed, model)
    assert int(o["status"].item()) == 0
    h = records(o)
    bests = cm.best_records(o["best"])
    for ci, c in enumerate(curves):
        print(f"[oracle] curve {ci}: n_obs={c.n_obs} K={len(c.periods)}", flush=True)
        ref = ora.search(c)
        sl = slice(per_off[ci], per_off[ci + 1])
        if len(c.periods) == 0:
            assert bests[ci]["k"] == -1
            continue
        g = {k: h[k][sl] for k in ("lr", "epoch", "dur", "depth", "depth_var")}
        res = check_periodic(g, ref["periodic"], lambda P, i, j: ora.fold_at(ref["grid"], ref["linear"], P, i, j),
                             c.periods)
        b = bests[ci]
        if ref["best"] < 0:
            assert b["k"] == -1
            continue
        if b["k"] != ref["best"]:  # near-tie across periods
            lr_o = ref["periodic"]["lr"]
            gap = (lr_o[ref["best"]] - lr_o[b["k"]]) / lr_o[ref["best"]]
            assert gap <= TOL, (ci, b["k"], ref["best"], gap)
        assert b["lr"] == pytest.approx(ref["periodic"]["lr"][b["k"]], rel=TOL)
        print(f"[oracle] curve {ci}: {res}", flush=True)


def test_batch_cancel_then_resume(cm):
    """The plan's pinned-host cancel flag: set before the search, nothing
    runs; set by a host thread while it runs, the launch stops early with
    some curves done; a resumed search then completes the rest, and every
    record equals the uncancelled search's."""
    import torch
    curves = W.batched_survey(24, seed=31, n_min=20000, n_max=60000)
    model = cm.template_resample(torch.as_tensor(curves[0].dense, device="cuda"), curves[0].n_model)
    grids, obs_off, per_off, t, f, s, p = pack(cm, curves)
    td, fd, sd, pd = (torch.as_tensor(x, device="cuda") for x in (t, f, s, p))
    plan = cm.batch_plan(grids, obs_off, per_off)
    work = cm.batch_workspace(plan)
    flag = plan.cancel_flag()
    flag[0] = 0
    print("[cancel] reference search", flush=True)
    t0 = time.perf_counter()
    ref = cm.batch_search(plan, td, fd, sd, model, pd, work=work)
    torch.cuda.synchronize()
    ms_ref = (time.perf_counter() - t0) * 1e3
    assert int(ref["status"].item()) == 0 and np.all(ref["done"].cpu().numpy() == 1)
    want = records(ref)
    want_best = ref["best"].cpu().numpy()
    # cancelled before it starts: no curve is searched
    flag[0] = 1
    print("[cancel] pre-set flag", flush=True)
    o = cm.batch_search(plan, td, fd, sd, model, pd, work=work)
    torch.cuda.synchronize()
    assert int(o["status"].item()) & cm._abi.BATCH_CANCELLED
    assert np.all(o["done"].cpu().numpy() == 0)
    # cancelled by a host thread part-way through
    flag[0] = 0
    timer = threading.Timer(max(ms_ref, 20.0) * 0.4e-3, lambda: flag.__setitem__(0, 1))
    print(f"[cancel] flag set after {max(ms_ref, 20.0) * 0.4:.0f} ms of a {ms_ref:.0f} ms search", flush=True)
    timer.start()
    o = cm.batch_search(plan, td, fd, sd, model, pd, work=work)
    torch.cuda.synchronize()
    timer.join()
    st, done = int(o["status"].item()), o["done"].cpu().numpy()
    print(f"[cancel] status={st} done={int((done == 1).sum())}/{len(done)}", flush=True)
    assert st in (0, cm._abi.BATCH_CANCELLED)
    assert set(np.unique(done)) <= {0, 1}
    # resume: the curves not done are searched, the done ones keep their records
    flag[0] = 0
    print("[cancel] resume", flush=True)
    cm.batch_search(plan, td, fd, sd, model, pd, work=work, out=o, resume=True)
    torch.cuda.synchronize()
    assert int(o["status"].item()) == 0 and np.all(o["done"].cpu().numpy() == 1)
    got = records(o)
    for k in want:
        assert np.array_equal(got[k], want[k], equal_nan=True), k
    assert np.array_equal(o["best"].cpu().numpy(), want_best)


def test_batch_workspace_without_tables_sets_status(cm, setup):
    """A workspace that does not hold the plan's tables: the persistent
    kernel checks the tables' tag and plan id first and returns at once."""
    import torch
    curves, model, packed, _ = setup
    grids, obs_off, per_off, t, f, s, p = packed
    plan = cm.batch_plan(grids, obs_off, per_off)
    other = cm.batch_plan(grids, obs_off, per_off)
    work = cm.batch_workspace(other)  # tables of another plan
    print("[tables] foreign tables", flush=True)
    o = cm.batch_search(plan, t, f, s, model, p, work=work)
    torch.cuda.synchronize()
    assert int(o["status"].item()) == cm._abi.BATCH_BAD_TABLES
    assert np.all(o["done"].cpu().numpy() == 0)


def test_batch_flags_unsorted_curve(cm, setup):
    """A curve whose times are out of order is reported (done = -1 and the
    status bit); the other curves are unaffected."""
    import torch
    curves, model, packed, single = setup
    grids, obs_off, per_off, t, f, s, p = packed
    t = t.copy()
    a, b = int(obs_off[5]), int(obs_off[6])
    t[a + 10], t[a + 11] = t[a + 11], t[a + 10]
    plan = cm.batch_plan(grids, obs_off, per_off)
    print("[unsorted] curve 5", flush=True)
    o = cm.batch_search(plan, t, f, s, model, p)
    torch.cuda.synchronize()
    assert int(o["status"].item()) == cm._abi.BATCH_UNSORTED
    done = o["done"].cpu().numpy()
    assert done[5] == -1 and np.all(np.delete(done, 5) == 1)
    h = records(o)
    for ci, r in enumerate(single):
        if ci == 5 or not r:
            continue
        sl = slice(per_off[ci], per_off[ci + 1])
        for k in ("lr", "epoch", "dur", "depth", "depth_var"):
            assert np.array_equal(h[k][sl], r[k], equal_nan=True), (ci, k)


def test_batch_duration_ranges_match_single_calls(cm, setup):
    """Per-period duration ranges (the Keplerian filter's output form) in
    the batch give the records of single-curve searches with the same
    ranges."""
    import torch
    curves, model, packed, _ = setup
    grids, obs_off, per_off, t, f, s, p = packed
    J = grids[0].n_dur
    rng = np.random.default_rng(17)
    K = int(per_off[-1])
    lo = rng.integers(0, J // 2, K)
    jr = np.stack([lo, np.minimum(J - 1, lo + rng.integers(0, J, K))], axis=1).astype(np.int32)
    plan = cm.batch_plan(grids, obs_off, per_off)
    print("[jrange] batch", flush=True)
    o = cm.batch_search(plan, t, f, s, model, p, jrange=jr)
    torch.cuda.synchronize()
    assert int(o["status"].item()) == 0
    h = records(o)
    for ci, c in enumerate(curves):
        if not len(c.periods):
            continue
        sl = slice(per_off[ci], per_off[ci + 1])
        g = grids[ci]
        flux, ivar, _ = cm.resample(g, c.t, c.f, c.sigma)
        fold = cm.linear_search(g, flux, ivar, model)
        ref = cm.periodic_search(g, fold, c.periods, jrange=jr[sl])
        torch.cuda.synchronize()
        for k, v in ref.items():
            assert np.array_equal(h[k][sl], v.cpu().numpy(), equal_nan=True), (ci, k)
