"""A plan at the batching workload's scale, bit-exact against the oracle.

128 tables drawn from the many-table workload's distribution (bucket counts
log-uniform over 2^10..2^18, loads uniform in [0.6, 0.95], lookup batches
uniform in [32, 4096], each table with its own negative rate uniform in
[0, 1]; about 260 000 lookups), every table image built by the oracle and
imported.  The plan runs at the shape the autotuner picks on these batches,
eagerly and replayed from a HIP graph, and at shapes whose persistent grid
is small enough that every wavefront runs many work items (so the item
pipeline, which prefetches the next item's descriptor and keys during the
current one, runs deep).  Every position of every range must equal the
oracle's answer; positions outside the ranges stay untouched."""

import numpy as np
import pytest

from gpu_util import say, to_dev, u64, u8
from test_gpu_plan import SENTINEL_F, SENTINEL_V, Fleet, run_plan

pytestmark = pytest.mark.gpu

NTABLES = 128


@pytest.fixture(scope="module")
def big_fleet():
    say(f"building {NTABLES} oracle tables of 2^10..2^18 buckets")
    f = Fleet(NTABLES, 4, 10, 18, 32, 4096)
    yield f
    f.close()


@pytest.fixture(scope="module")
def expected(big_fleet):
    return big_fleet.expected()


def test_fleet_matches_the_workload_distribution(big_fleet):
    b = np.array([t.log2_buckets for t in big_fleet.tables])
    assert b.min() >= 10 and b.max() <= 18 and len(set(b.tolist())) >= 7
    c = big_fleet.counts.astype(np.int64)
    assert c.min() >= 32 and c.max() <= 4096 and c.sum() > 100_000


def test_tuned_plan_eager_and_graph(big_fleet, expected):
    """The autotuner's shape (timed over every plan shape on these batches),
    then two eager launches and three replays of a captured launch, with
    eager lookups on the stream between the replays."""
    import torch
    from paper_1712_09624_amd import tune
    from paper_1712_09624_amd.ckpp import Plan
    want_f, want_v = expected
    plan = Plan(big_fleet.tables, big_fleet.offsets, big_fleet.counts)
    keys = to_dev(big_fleet.all_keys)
    found = torch.full((big_fleet.span,), SENTINEL_F, dtype=torch.uint8, device="cuda:0")
    vals = torch.full((big_fleet.span,), SENTINEL_V, dtype=torch.int64, device="cuda:0")
    say(f"tuning the plan over {len(tune.PLAN_SHAPES)} shapes, span {big_fleet.span}")
    res = tune.tune_plan(plan, keys, found, vals, reps=2)
    best = plan.get_launch()
    assert best == res[0][1]
    say(f"tuned shape {best}: eager launches")
    for rep in range(2):
        f, v = run_plan(plan, big_fleet)
        assert np.array_equal(f, want_f), f"found differs at the tuned shape (launch {rep})"
        assert np.array_equal(v, want_v), f"values differ at the tuned shape (launch {rep})"
    g_found = torch.full((big_fleet.span,), SENTINEL_F, dtype=torch.uint8, device="cuda:0")
    g_vals = torch.full((big_fleet.span,), SENTINEL_V, dtype=torch.int64, device="cuda:0")
    plan.lookup(keys, g_found, g_vals)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    say("capturing the tuned plan launch")
    with torch.cuda.graph(graph):
        plan.lookup(keys, g_found, g_vals)
    torch.cuda.synchronize()
    probe = big_fleet.tables[0]
    pk = to_dev(big_fleet.keys[0])
    for rep in range(3):
        g_found.fill_(SENTINEL_F)
        g_vals.fill_(SENTINEL_V)
        torch.cuda.synchronize()
        say(f"graph replay {rep}")
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(u8(g_found), want_f), f"found differs (replay {rep})"
        assert np.array_equal(u64(g_vals), want_v), f"values differ (replay {rep})"
        probe.lookup(pk)  # eager work between replays
        torch.cuda.synchronize()
    del graph
    plan.close()


# (lookups per lane, block, blocks per CU, passes per item, schedule, lanes
# per lookup): one 64-thread block per compute unit is 256 wavefronts for
# some 4 000 work items, so each wavefront runs about sixteen
FEW_WAVE_SHAPES = [(1, 64, 1, 1, 0, 8), (1, 64, 1, 1, 1, 8), (2, 64, 1, 1, 1, 8),
                   (1, 64, 1, 1, 0, 4), (2, 64, 1, 2, 1, 4), (1, 64, 1, 1, 0, 1),
                   (4, 64, 1, 1, 1, 1), (2, 128, 2, 3, 0, 1)]


@pytest.mark.parametrize("shape", FEW_WAVE_SHAPES, ids=[f"per{a}_b{b}_bpc{c}_p{d}_s{e}_l{g}"
                                                        for a, b, c, d, e, g in FEW_WAVE_SHAPES])
def test_many_items_per_wave(big_fleet, expected, shape):
    from paper_1712_09624_amd.ckpp import Plan
    want_f, want_v = expected
    plan = Plan(big_fleet.tables, big_fleet.offsets, big_fleet.counts)
    plan.set_launch(*shape)
    items = plan.info()["nitems"]
    say(f"fleet plan shape={shape} items={items}")
    for rep in range(2):
        f, v = run_plan(plan, big_fleet)
        assert np.array_equal(f, want_f), f"found differs (launch {rep})"
        assert np.array_equal(v, want_v), f"values differ (launch {rep})"
    plan.close()
