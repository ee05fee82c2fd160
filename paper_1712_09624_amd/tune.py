"""Launch-shape autotuner of the lookup kernels and of plans.

Times every lookup launch shape (lanes per lookup: 8, lines landing in LDS,
4, lines spread over a quad's registers, or 1, bucket heads in registers;
lookups in flight per lane, block size, grid cap) on a caller's table and key batches, and returns
the shapes ranked by lookups per second.  Timing uses device events on the
current stream; the answers do not depend on the shape (the parity tests
check every shape), only the speed does.
"""

from __future__ import annotations

import itertools

SHAPES = [
    {"lanes_per_lookup": lanes, "lookups_per_lane": per, "block": block, "blocks_per_cu": bpc}
    for lanes, per, block, bpc in itertools.product((8,), (1, 2), (64, 128, 256), (0, 5, 10))
] + [
    {"lanes_per_lookup": 4, "lookups_per_lane": per, "block": block, "blocks_per_cu": bpc}
    for per, block, bpc in itertools.product((1, 2), (64, 128, 256), (0, 8, 16))
] + [
    {"lanes_per_lookup": 1, "lookups_per_lane": per, "block": block, "blocks_per_cu": bpc}
    for per, block, bpc in itertools.product((1, 2, 4), (64, 128, 256), (0, 8, 16))
]


def time_lookup(table, keys, mode, found, values, reps=3):
    import torch
    s = torch.cuda.current_stream()
    table.lookup(keys, mode, found=found, values=values)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        table.lookup(keys, mode, found=found, values=values)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(table, batches, mode="cuckoopp", shapes=None, reps=3, apply=True):
    """batches: list of device key tensors (e.g. a positive and a negative
    batch).  The score of a shape is the total time over the batches.
    Returns [(total_ms, shape, [ms per batch])] sorted fastest first, and
    sets the fastest shape on the table when apply is true."""
    import torch
    shapes = shapes or SHAPES
    n = max(int(b.shape[0]) for b in batches)
    found = torch.empty(n, dtype=torch.uint8, device=batches[0].device)
    values = torch.empty(n, dtype=torch.int64, device=batches[0].device)
    before = table.get_lookup_launch()
    results = []
    for sh in shapes:
        table.set_lookup_launch(sh["lanes_per_lookup"], sh["lookups_per_lane"], sh["block"],
                                sh["blocks_per_cu"])
        per = [time_lookup(table, b, mode, found[: b.shape[0]], values[: b.shape[0]], reps)
               for b in batches]
        results.append((sum(per), dict(sh), per))
    results.sort(key=lambda r: r[0])
    best = results[0][1] if apply else before
    table.set_lookup_launch(best["lanes_per_lookup"], best["lookups_per_lane"], best["block"],
                            best["blocks_per_cu"])
    return results


# Launch shapes of a plan's persistent kernel: lanes per lookup (8: lines in
# LDS, 4: lines in a quad's registers, 1: bucket heads in registers) with
# lookups per lane, block size,
# blocks per compute unit (persistent grid), lookup passes per work item and
# schedule (0 static, 1 dynamic).
PLAN_SHAPES = [
    {"lookups_per_lane": per, "block": block, "blocks_per_cu": bpc, "passes_per_item": passes,
     "schedule": sched, "lanes_per_lookup": lanes}
    for (lanes, per), block, bpc, passes, sched in itertools.product(
        ((8, 1), (8, 2), (4, 1), (4, 2), (1, 1), (1, 2), (1, 4)), (64, 128, 256), (2, 4, 8, 16), (1, 2, 4), (0, 1))
]


def time_plan(plan, keys, found, values, reps=5, **lookup_args):
    import torch
    s = torch.cuda.current_stream()
    plan.lookup(keys, found, values, **lookup_args)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        plan.lookup(keys, found, values, **lookup_args)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_plan(plan, keys, found, values, shapes=None, reps=5, apply=True, **lookup_args):
    """Times every plan launch shape on the plan's own batches (lookup_args,
    e.g. now= for a plan with tables with timers, go to each lookup).
    Returns [(ms, shape)] sorted fastest first, and keeps the fastest shape
    on the plan when apply is true (else restores the shape it had)."""
    shapes = shapes or PLAN_SHAPES
    before = plan.get_launch()
    results = []
    for sh in shapes:
        plan.set_launch(sh["lookups_per_lane"], sh["block"], sh["blocks_per_cu"],
                        sh["passes_per_item"], sh["schedule"], sh["lanes_per_lookup"])
        results.append((time_plan(plan, keys, found, values, reps, **lookup_args), dict(sh)))
    results.sort(key=lambda r: r[0])
    best = results[0][1] if apply else before
    plan.set_launch(best["lookups_per_lane"], best["block"], best["blocks_per_cu"],
                    best["passes_per_item"], best["schedule"], best["lanes_per_lookup"])
    return results
