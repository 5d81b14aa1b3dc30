"""Autotuner for the launch tuning of a context (sbr_context_set_tuning).

The tuning never changes results (packet size, workgroup counts, LDS staging
and the refinement's lookahead only change how work is scheduled), so the
tuner only measures time: for each candidate it applies the tuning, runs the
given workload `warmup` times, times `steps` runs, and keeps the fastest.
"""
from __future__ import annotations

import itertools
import time

DEFAULT_SPACE = {
    "trace_chunk": [1, 2, 4],
    # four workgroups per CU fill the machine; a small scene's trace runs
    # faster with fewer (its BVH then shares each CU's L1 among fewer waves)
    "persist_blocks": [1024, 2048, 640, 768],
    "lds_budget": [0, 65536],
    "stack_depth": [16],
    "trace_block": [256],
    "lookahead_max_paths": [0, 4096],
}


def _time(run, warmup, steps, sync):
    for _ in range(warmup):
        run()
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    sync()
    return (time.perf_counter() - t0) / steps


def autotune(ctx, run, space=None, warmup=1, steps=2):
    """Try every combination in `space` (dict of field -> candidate values)
    on the workload `run()` (a callable that makes one library call through
    ctx).  Leaves ctx tuned to the first combination within 2% of the fastest
    and returns
    (best_tuning, [(tuning, seconds), ...])."""
    import torch
    space = dict(DEFAULT_SPACE if space is None else space)
    keys = list(space)
    results = []
    base = ctx.tuning()
    for combo in itertools.product(*(space[k] for k in keys)):
        t = dict(zip(keys, combo))
        ctx.set_tuning(**dict(base, **t))
        sec = _time(run, warmup, steps, torch.cuda.synchronize)
        results.append((t, sec))
    # the first combination (in the space's order) within 2% of the fastest,
    # so that near-ties do not flip between runs
    fastest = min(sec for _, sec in results)
    best = next(t for t, sec in results if sec <= fastest * 1.02)
    ctx.set_tuning(**dict(base, **best))
    return best, results
