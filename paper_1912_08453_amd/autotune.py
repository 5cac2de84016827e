"""Empirical tuning of the library's work-saving settings.

The settings (pm_set_param: the final search's work-saving switches and
grid, the LCC sweeps' degree-bin bounds) change only how the prune spends
its time, never which roles and edges survive, so they can be chosen by
timing alone.  `autotune` runs a coordinate search: for each setting in turn it
times the prune of the given templates with every candidate value, the
others held at their best so far, and keeps the fastest; one or more
passes over all settings.  The winning values are left set on the context.

    from paper_1912_08453_amd import autotune
    best, table = autotune.autotune(ctx, template_ids)
"""
from __future__ import annotations

import json
import os
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple


def default_space(ctx) -> Dict[str, List[int]]:
    """Candidate values per setting; the search grid is offered at half,
    one and two times its current value (by default 8 blocks per compute
    unit), the grid shared by concurrent searches off or at two and four
    times it."""
    g = ctx.get_param("search_grid")
    return {
        "edge_chunk": [4, 8, 16, 32, 64],
        "edge_stripes": [1, 16, 64, 256],
        "expand": [0, 1],
        "expand_edges": [0, 1],
        "expand_max": [1024, 4096, 16384, -1],
        "witness": [0, 1],
        "relist": [0, 1],
        "search_grid": sorted({max(1, g // 2), g, 2 * g}),
        "search_grid_solo": [0, 2 * g, 4 * g],
        "split_budget": [0, 2048, 8192, 32768],
        "edge_tail": [0, 16384, 65536],
        "read_first": [0, 1],
        "lcc_bin_small": [4, 8, 16],
        "lcc_bin_mid": [32, 64, 128, 256],
    }


def prune_timer(ctx, tids: Sequence[int], batch: bool = False, reps: int = 2, **prune_kw):
    """A timer for `autotune`: the best of `reps` wall-clock times of
    pruning every template (one call per template, or one batched call
    over a contiguous id range when `batch`), with the device drained
    before and after."""
    import torch

    def run():
        if batch:
            ctx.prune(tids[0], count=len(tids), **prune_kw)
        else:
            for t in tids:
                ctx.prune(t, **prune_kw)

    def timer() -> float:
        best = None
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run()
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0)
            best = ms if best is None else min(best, ms)
        return best

    return timer


def coordinate_search(set_value: Callable[[str, int], None], timer: Callable[[], float],
                      start: Dict[str, int], space: Dict[str, Sequence[int]],
                      passes: int = 1, log: Optional[Callable[[str], None]] = None
                      ) -> Tuple[Dict[str, int], List[Tuple[str, int, float]]]:
    """Coordinate search over `space` from `start`.  Each setting's
    candidates are timed with the other settings at their current best; a
    candidate replaces the current value only if strictly faster.  Returns
    the best assignment (also left applied through `set_value`) and the
    table of (setting, value, ms) measurements."""
    best = dict(start)
    for k, v in best.items():
        set_value(k, v)
    base = timer()
    table = [("start", 0, base)]
    for _ in range(passes):
        for k, cands in space.items():
            cur = best[k]
            best_ms = base
            for v in cands:
                if v == cur:
                    continue
                set_value(k, v)
                ms = timer()
                table.append((k, v, ms))
                if log:
                    log(f"{k}={v}: {ms:.2f} ms (best {best_ms:.2f} ms at {k}={best[k]})")
                if ms < best_ms:
                    best_ms = ms
                    best[k] = v
            set_value(k, best[k])
            base = best_ms
    return best, table


def autotune(ctx, tids: Sequence[int], space: Optional[Dict[str, Sequence[int]]] = None,
             passes: int = 1, batch: bool = False, reps: int = 2,
             log: Optional[Callable[[str], None]] = None, **prune_kw):
    """Tune the context's settings on the prune of templates `tids`; returns
    (best settings, measurement table)."""
    space = default_space(ctx) if space is None else space
    start = {k: ctx.get_param(k) for k in space}
    timer = prune_timer(ctx, tids, batch=batch, reps=reps, **prune_kw)
    timer()   # warm-up: workspaces sized, kernels loaded
    return coordinate_search(ctx.set_param, timer, start, space, passes=passes, log=log)


TUNED_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_settings.json")


def load_tuned(workload: str, path: str = TUNED_PATH) -> Dict[str, int]:
    """Settings the autotuner chose for a named workload (empty if none)."""
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return dict(json.load(f).get(workload, {}).get("settings", {}))


def apply_tuned(ctx, workload: str) -> Dict[str, int]:
    """Set the stored settings of `workload` on the context; returns them."""
    s = load_tuned(workload)
    # the bin bounds must stay ordered while they are set one at a time:
    # raise the upper one first when the lower one grows past it
    first = "lcc_bin_mid" if s.get("lcc_bin_small", 0) > ctx.get_param("lcc_bin_mid") \
        else "lcc_bin_small"
    for k in sorted(s, key=lambda k: (k != first, k)):
        ctx.set_param(k, int(s[k]))
    return s
