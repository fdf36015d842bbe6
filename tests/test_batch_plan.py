"""Host-side checks of the batched search's plan (no GPU): the tables image
the persistent kernel reads is parsed here with its own layout description
and checked for what the kernel relies on --

* every work item belongs to exactly one (curve, stage) segment, in order;
* every dependency an item waits for (the previous stage of its curve, or
  the decode of the curve that used its arena slot before) consists of
  items queued strictly earlier, so workgroups that pop items in queue
  order always drain the queue (the earliest unfinished item never waits);
* every index the items derive stays inside its buffer: observations,
  periods, keys, arena slots, resampled points, fold rows and epoch chunks.
A simulation of workgroups popping items and waiting on counters confirms
that the queue drains with any number of workgroups."""

import ctypes
import heapq

import numpy as np
import pytest

HEADER = np.dtype([("magic", "<u8"), ("plan_id", "<u8"), ("n_curves", "<i8"), ("n_groups", "<i8"),
                   ("n_segments", "<i8"), ("n_items", "<i8"), ("off_curves", "<i8"), ("off_groups", "<i8"),
                   ("off_grids", "<i8"), ("off_segments", "<i8"), ("tables_bytes", "<i8"),
                   ("period_block", "<i4"), ("lds_bytes", "<i4"), ("lds_cap", "<i4"), ("linear_windows", "<i4"),
                   ("pop_items", "<i4"), ("reserved", "<i4")])
CURVE = np.dtype([("obs_off", "<i8"), ("n_obs", "<i8"), ("per_off", "<i8"), ("n_per", "<i8"), ("slot_off", "<i8"),
                  ("ivar_off", "<i8"), ("fold_off", "<i8"), ("ptab_off", "<i8"), ("n_items", "<i8", (4,)),
                  ("group", "<i4"), ("n_res", "<i4"), ("n_lin_per_dur", "<i4"), ("n_pblk", "<i4"),
                  ("n_chunks", "<i4"), ("n_tiles", "<i4")])
GROUP = np.dtype([("n_items", "<i8", (4,)), ("prev_group", "<i4"), ("n_curves", "<i4")])
SEGMENT = np.dtype([("first", "<i8"), ("curve", "<i4"), ("stage", "<i4")])
RES, LIN, FOLD, EPI = range(4)
RES_POINTS, LIN_TILES, THREADS, EPI_PERIODS = 2048, 4, 256, 256
PERIOD_INFO_BYTES = 24  # u64 step, i32 epochs, i32 jlo, i32 jhi, padded to 8
MAX_SETS, MAX_GROUP, GROUP_FOLD_ITEMS = 8, 16, 49152


def parse(plan):
    raw = plan.tables()
    h = np.frombuffer(raw, HEADER, count=1)[0]
    cur = np.frombuffer(raw, CURVE, count=int(h["n_curves"]), offset=int(h["off_curves"]))
    grp = np.frombuffer(raw, GROUP, count=int(h["n_groups"]), offset=int(h["off_groups"]))
    seg = np.frombuffer(raw, SEGMENT, count=int(h["n_segments"]), offset=int(h["off_segments"]))
    return h, cur, grp, seg


def make(cm, curves, **kw):
    grids = [cm.grid_plan(c.t[0], c.t[-1], c.cadence, c.durations) for c in curves]
    oo = np.concatenate([[0], np.cumsum([c.n_obs for c in curves])])
    po = np.concatenate([[0], np.cumsum([len(c.periods) for c in curves])])
    return grids, oo, po, cm.batch_plan(grids, oo, po, **kw)


def segments_of(h, seg):
    """(curve, stage) -> (first, end) item range."""
    out = {}
    firsts = list(seg["first"]) + [int(h["n_items"])]
    for s, (f, c, st) in enumerate(zip(seg["first"], seg["curve"], seg["stage"])):
        out[(int(c), int(st))] = (int(f), int(firsts[s + 1]))
    return out


def dependency(cur, grp, c, stage):
    """The (curve, stage) keys whose items must all be complete first: the
    previous stage of every curve of c's group, or for RES the decode of
    every curve of the group that used the slot set before."""
    g = int(cur[c]["group"])
    members = lambda gi: [k for k in range(len(cur)) if int(cur[k]["group"]) == gi]
    if stage == RES:
        pg = int(grp[g]["prev_group"])
        return [] if pg < 0 else [(k, EPI) for k in members(pg)]
    return [(k, stage - 1) for k in members(g)]


def slot_size(cur, c):
    return int(cur[c]["ptab_off"]) + PERIOD_INFO_BYTES * max(int(cur[c]["n_per"]), 1)


def check_plan(cm, curves, grids, oo, po, plan):
    h, cur, grp, seg = parse(plan)
    n = len(curves)
    assert h["n_curves"] == n and h["n_segments"] == len(seg) and h["n_groups"] == len(grp)
    B = int(h["period_block"])
    Wl = int(h["linear_windows"])
    assert Wl in (1, 2)
    # segments: increasing, contiguous, one per (curve, stage) with items
    assert seg["first"][0] == 0 and np.all(np.diff(seg["first"]) > 0)
    rng = segments_of(h, seg)
    assert len(rng) == len(seg)
    for c in range(n):
        for st in range(4):
            cnt = int(cur[c]["n_items"][st])
            if cnt == 0:
                assert (c, st) not in rng
            else:
                f, e = rng[(c, st)]
                assert e - f == cnt, (c, st)
    assert sum(int(x) for x in cur["n_items"].sum(axis=1)) == h["n_items"]
    # groups: consecutive in queue order, closed by size or fold items, with
    # per-stage sums and the previous user of their slot set
    order = plan.order()
    G = len(grp)
    S = min(MAX_SETS, G)
    gseq = [int(cur[c]["group"]) for c in order]
    assert gseq[0] == 0 and all(b - a in (0, 1) for a, b in zip(gseq, gseq[1:])) and gseq[-1] == G - 1
    for gi in range(G):
        mem = [c for c in order if int(cur[c]["group"]) == gi]
        assert int(grp[gi]["n_curves"]) == len(mem) <= MAX_GROUP
        assert np.array_equal(grp[gi]["n_items"], cur[mem]["n_items"].sum(axis=0))
        assert int(grp[gi]["prev_group"]) == (gi - S if gi >= S else -1)
        fold_before_last = int(cur[mem[:-1]]["n_items"][:, FOLD].sum()) if len(mem) > 1 else 0
        assert fold_before_last < GROUP_FOLD_ITEMS  # a group closes only once it has enough fold items
    # dependencies sit earlier in the queue
    for (c, st), (f, e) in rng.items():
        for dep in dependency(cur, grp, c, st):
            if dep in rng:
                assert rng[dep][1] <= f, ((c, st), dep, rng[dep], (f, e))
    # bounds of what items index
    for p, c in enumerate(order):
        g = grids[c]
        d = cur[c]
        assert d["obs_off"] == oo[c] and d["n_obs"] == oo[c + 1] - oo[c]
        assert d["per_off"] == po[c] and d["n_per"] == po[c + 1] - po[c]
        assert d["n_res"] * RES_POINTS >= g.n > (d["n_res"] - 1) * RES_POINTS
        assert d["n_tiles"] * THREADS * Wl >= g.n_t0 > (d["n_tiles"] - 1) * THREADS * Wl
        assert d["n_lin_per_dur"] * LIN_TILES >= d["n_tiles"]
        assert d["n_items"][LIN] == g.n_dur * d["n_lin_per_dur"]
        assert d["n_pblk"] * B >= d["n_per"] > (d["n_pblk"] - 1) * B
        assert d["n_items"][FOLD] == g.n_dur * d["n_pblk"] * d["n_chunks"]
        assert 1 <= d["n_chunks"] <= 64
        assert d["n_items"][EPI] == max(1, -(-int(d["n_per"]) // EPI_PERIODS))
        # the slot: flux, ivar, the fold-ready array and the period table fit
        assert d["slot_off"] % 256 == 0 and d["ivar_off"] >= 4 * g.n and d["fold_off"] - d["ivar_off"] >= 4 * g.n
        assert d["ptab_off"] - d["fold_off"] >= 8 * g.n_dur * g.n_t0
        assert slot_size(cur, c) + d["slot_off"] <= plan.info["workspace_bytes"]
        assert g.n_t0 < 1 << 28
    # slots of curves that can be live together do not overlap: curves of one
    # group, and of groups in different slot sets
    spans = [(int(cur[c]["slot_off"]), int(cur[c]["slot_off"]) + slot_size(cur, c), int(cur[c]["group"]))
             for c in range(n)]
    for i in range(n):
        for k in range(i + 1, n):
            a, b = spans[i], spans[k]
            if a[2] == b[2] or a[2] % S != b[2] % S:
                assert a[1] <= b[0] or b[1] <= a[0], (i, k, a, b)
    assert 0 < h["lds_bytes"] <= h["lds_cap"]
    return h, cur, grp, seg, rng


def simulate(cur, grp, rng, n_items, workers, seed):
    """Workgroups pop items in queue order; an item whose dependency is not
    complete waits (holding its workgroup) until it is.  Returns the finish
    time; raises if the queue stops with items outstanding (a deadlock)."""
    r = np.random.default_rng(seed)
    owner = []
    for (c, st), (f, e) in rng.items():
        owner += [(i, c, st) for i in range(f, e)]
    owner.sort()
    done = {k: 0 for k in rng}
    need = {k: e - f for k, (f, e) in rng.items()}
    deps = {k: [d for d in dependency(cur, grp, *k) if d in rng] for k in rng}
    head, t, running, waiting = 0, 0.0, [], []
    free = workers
    finished = 0
    while finished < n_items:
        while free and head < n_items:
            _, c, st = owner[head]
            head += 1
            free -= 1
            waiting.append((c, st))
        still = []
        for c, st in waiting:
            if all(done[d] == need[d] for d in deps[(c, st)]):
                heapq.heappush(running, (t + r.uniform(0.5, 2.0), c, st))
            else:
                still.append((c, st))
        waiting = still
        if not running:
            raise AssertionError(f"deadlock: {len(waiting)} workgroups waiting, {finished} of {n_items} done")
        t, c, st = heapq.heappop(running)
        done[(c, st)] += 1
        finished += 1
        free += 1
    return t


def simulate_runs(cur, grp, rng, n_items, workers, pop, seed):
    """The kernel's queue protocol with runs: a workgroup pops `pop`
    consecutive items, runs them in order, and adds its finished items of one
    (curve, stage) to that stage's counter only before it moves to another
    (curve, stage), waits, or pops again.  Dependency checks see counted items
    only.  Raises on a deadlock, or if a workgroup would wait while holding
    uncounted items; returns the finish time."""
    r = np.random.default_rng(seed)
    key_of = [None] * n_items
    for k, (f, e) in rng.items():
        for i in range(f, e):
            key_of[i] = k
    counted = {k: 0 for k in rng}
    need = {k: e - f for k, (f, e) in rng.items()}
    deps = {k: [d for d in dependency(cur, grp, *k) if d in rng] for k in rng}
    state = {"head": 0, "t": 0.0}
    wgs = [dict(next=0, end=0, pend=None, n=0, mode="idle") for _ in range(workers)]
    running = []

    def flush(w):
        if w["n"]:
            counted[w["pend"]] += w["n"]
            assert counted[w["pend"]] <= need[w["pend"]]
            w["n"] = 0

    def advance(i):
        w = wgs[i]
        if w["next"] >= w["end"]:
            flush(w)
            if state["head"] >= n_items:
                w["mode"] = "exit"
                return
            w["next"], w["end"] = state["head"], min(state["head"] + pop, n_items)
            state["head"] = w["end"]
        k = key_of[w["next"]]
        if w["n"] and k != w["pend"]:
            flush(w)
        if all(counted[d] == need[d] for d in deps[k]):
            heapq.heappush(running, (state["t"] + r.uniform(0.5, 2.0), i))
            w["mode"] = "run"
        else:
            assert w["n"] == 0, "waiting while holding uncounted items"
            w["mode"] = "wait"

    for i in range(workers):
        advance(i)
    finished = 0
    while running:
        state["t"], i = heapq.heappop(running)
        w = wgs[i]
        w["pend"], w["n"] = key_of[w["next"]], w["n"] + 1
        w["next"] += 1
        finished += 1
        advance(i)
        for j, v in enumerate(wgs):
            if v["mode"] == "wait":
                advance(j)
    if finished < n_items or any(w["mode"] != "exit" for w in wgs):
        raise AssertionError(f"deadlock: {finished} of {n_items} done")
    assert counted == need
    return state["t"]


@pytest.fixture(scope="module")
def cm():
    import paper_2503_20875_amd as cm
    from paper_2503_20875_amd import _abi
    import os
    if not os.path.exists(_abi.LIB_PATH):
        from paper_2503_20875_amd import build
        build.build()
    return cm


def _batch(n, seed, n_min=2000, n_max=15000, thin=25, edges=True):
    from synthlc import workloads as W
    curves = W.batched_survey(n, seed=seed, n_min=n_min, n_max=n_max)
    for c in curves:
        c.periods = c.periods[::thin].copy()
    if edges and n >= 4:
        tiny = curves[1]
        tiny.t, tiny.f, tiny.sigma = tiny.t[:2].copy(), tiny.f[:2].copy(), tiny.sigma[:2].copy()
        curves[3].periods = np.zeros(0)
    return curves


@pytest.mark.parametrize("n,seed,shuffle,block", [(1, 1, 0, 0), (2, 2, 0, 4), (3, 3, 0, 8), (5, 4, 0, 0),
                                                  (10, 7, 0, 0), (10, 7, 99, 0), (37, 5, 3, 4)])
def test_plan_tables_queue_and_bounds(cm, n, seed, shuffle, block):
    curves = _batch(n, seed)
    grids, oo, po, plan = make(cm, curves, period_block=block, shuffle_seed=shuffle)
    h, cur, grp, seg, rng = check_plan(cm, curves, grids, oo, po, plan)
    assert plan.info["n_launches"] == 2
    assert plan.info["n_items"] == h["n_items"]
    for workers in (1, 3, 64):
        simulate(cur, grp, rng, int(h["n_items"]), workers, seed)
    for workers, pop in ((1, 8), (3, 2), (7, 64), (64, 3)):
        simulate_runs(cur, grp, rng, int(h["n_items"]), workers, pop, seed)


def test_plan_groups_reuse_slot_sets(cm):
    """Many small curves: groups of up to 16 curves, more groups than slot
    sets, so every set is reused; the tables, slot spans and queue checks
    hold, and the queue drains under both protocols."""
    curves = _batch(160, 13, n_min=2000, n_max=6000, thin=2000, edges=False)
    grids, oo, po, plan = make(cm, curves)
    h, cur, grp, seg, rng = check_plan(cm, curves, grids, oo, po, plan)
    assert len(grp) > MAX_SETS and int(grp["n_curves"].max()) > 1
    assert np.any(grp["prev_group"] >= 0)
    for workers in (1, 16):
        simulate(cur, grp, rng, int(h["n_items"]), workers, 3)
    simulate_runs(cur, grp, rng, int(h["n_items"]), 16, 8, 3)


def test_plan_order_is_by_fold_cost_or_seeded(cm):
    curves = _batch(12, 11, edges=False)
    grids, oo, po, plan = make(cm, curves)
    J = grids[0].n_dur
    cost = [(po[c + 1] - po[c]) * J * g.n_t0 for c, g in enumerate(grids)]
    order = plan.order()
    assert sorted(order.tolist()) == list(range(12))
    assert all(cost[a] >= cost[b] for a, b in zip(order, order[1:]))
    o1 = make(cm, curves, shuffle_seed=5)[3].order()
    o2 = make(cm, curves, shuffle_seed=5)[3].order()
    o3 = make(cm, curves, shuffle_seed=6)[3].order()
    assert np.array_equal(o1, o2) and sorted(o1.tolist()) == list(range(12)) and not np.array_equal(o1, o3)


def test_plan_ids_differ_and_validation(cm):
    curves = _batch(4, 9)
    grids, oo, po, p1 = make(cm, curves)
    p2 = make(cm, curves)[3]
    assert parse(p1)[0]["plan_id"] != parse(p2)[0]["plan_id"]
    other = cm.grid_plan(curves[0].t[0], curves[0].t[-1], curves[0].cadence, curves[0].durations * 1.01)
    with pytest.raises(cm.CetraError, match="durations"):
        cm.batch_plan([other] + grids[1:], oo, po)
    with pytest.raises(cm.CetraError, match="offsets"):
        cm.batch_plan(grids, oo[::-1].copy(), po)
    with pytest.raises(cm.CetraError, match="fold_period_block"):
        cm.batch_plan(grids, oo, po, period_block=16)
    with pytest.raises(cm.CetraError, match="pop_items"):
        cm.batch_plan(grids, oo, po, pop_items=65)
    assert parse(make(cm, curves, pop_items=5)[3])[0]["pop_items"] == 5
    with pytest.raises(ValueError):
        cm.batch_plan(grids, oo[:-1], po)


def test_search_rejects_bad_arguments_on_the_host(cm):
    from paper_2503_20875_amd import _abi
    lib = _abi.load()
    curves = _batch(3, 2)
    plan = make(cm, curves)[3]
    P = ctypes.c_void_p(8)  # never dereferenced: every call below fails validation first
    rc = lib.cetra_batch_search(plan.handle, None, P, P, P, P, P, None, None, 0, P, 1, P, P, P, P, P, P, P, P)
    assert rc == -3 and b"workspace" in lib.cetra_last_error()
    rc = lib.cetra_batch_search(plan.handle, None, P, P, P, P, P, None, None, 2, P, 1 << 40, P, P, P, P, P, P, P, P)
    assert rc == -1 and b"flags" in lib.cetra_last_error()
    rc = lib.cetra_batch_search(plan.handle, None, P, P, P, P, P, None, None, 0, P, 1 << 40, P, P, P, P, P, P, None,
                                P)
    assert rc == -1 and b"NULL" in lib.cetra_last_error()
    need, tb = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.cetra_batch_workspace(plan.handle, ctypes.byref(need), ctypes.byref(tb)) == 0
    assert need.value == plan.info["workspace_bytes"] and tb.value == plan.info["tables_bytes"]
    assert len(plan.tables()) == tb.value
