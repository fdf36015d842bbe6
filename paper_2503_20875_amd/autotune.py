"""Launch-tuning search for the periodic search.

Times the fold (``cetra_periodic_search``) on the caller's own grid,
fold-ready array and periods under each candidate tuning -- period block,
resident workgroups per compute unit, units per workgroup and the fold
variant (lane epochs 64 apart, or adjacent with 16-byte loads) -- and keeps
the fastest with ``cetra_set_tuning``.
Results do not depend on the tuning (the parity tests check that every
variant returns identical records); only the time does.
"""

from __future__ import annotations

import itertools

from . import get_tuning, periodic_search, periodic_workspace, set_tuning

DEFAULT_CANDIDATES = tuple(
    (b, w, u, v) for b, w, u, v in itertools.product((4, 8, 16), (8,), (4, 16), (0, 2)))


def tune_fold(grid, fold, periods, candidates=DEFAULT_CANDIDATES, repeats: int = 2, apply: bool = True):
    """Returns (best tuning dict, {candidate: mean ms}).  The first launch of
    each candidate is a warm-up and is not timed."""
    import torch
    periods = periods if isinstance(periods, torch.Tensor) else torch.as_tensor(periods, device="cuda")
    K = int(periods.numel())
    work = torch.empty(max(periodic_workspace(grid, K), 1), dtype=torch.uint8, device="cuda")
    before = get_tuning()
    out = None
    times = {}
    try:
        for cand in candidates:
            set_tuning(*cand)
            out = periodic_search(grid, fold, periods, work=work, out=out)
            ms = []
            for _ in range(repeats):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                periodic_search(grid, fold, periods, work=work, out=out)
                e1.record()
                e1.synchronize()
                ms.append(e0.elapsed_time(e1))
            times[tuple(cand)] = sum(ms) / len(ms)
    finally:
        set_tuning(**before)
    best = min(times, key=times.get)
    cfg = dict(fold_period_block=best[0], fold_wgs_per_cu=best[1], fold_units_per_wg=best[2], fold_variant=best[3])
    if apply:
        set_tuning(**cfg)
    return cfg, times
