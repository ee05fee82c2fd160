"""Plans (many tables' lookup batches in one persistent launch) against the
oracle, bit-exact, and against one lookup call per table.

Every table image is built by the oracle and imported, so each table's
answers are unique; the plan must give them at every position of its
ranges and leave every other position untouched."""

import numpy as np
import pytest

from gpu_util import say, to_dev, u64, u8, vals_dev
from oracle import oracle as O
from paper_1712_09624_amd import workload as W

pytestmark = pytest.mark.gpu

OMODE = {"cuckoopp": O.MODE_CUCKOOPP, "both": O.MODE_BOTH, "optimistic": O.MODE_OPTIMISTIC}
PLAN_SHAPES = [(per, block, bpc, passes, sched, 8) for per in (1, 2) for block in (64, 128, 256)
               for bpc, passes in ((1, 1), (8, 1), (2, 3)) for sched in (0, 1)]
PLAN_SHAPES += [(per, block, bpc, passes, sched, 4) for per in (1, 2) for block in (64, 256)
                for bpc, passes in ((8, 1), (2, 3)) for sched in (0, 1)]
PLAN_SHAPES += [(per, block, bpc, passes, sched, 1) for per in (1, 2, 4) for block in (64, 256)
                for bpc, passes in ((8, 1), (2, 3)) for sched in (0, 1)]
SENTINEL_F, SENTINEL_V = 0xAB, 0x5A5A5A5A5A5A5A5A


class Fleet:
    """Tables of uneven size, load, batch and negative rate, built by the
    oracle; batches concatenated with gaps between the ranges."""

    def __init__(self, ntables, seed, log2_lo, log2_hi, batch_lo, batch_hi, plain_every=0,
                 modes=None, zero_every=0, timed_every=0, now0=0):
        """timed_every: every timed_every-th table (from the second) has
        timers, its entries' expiration times uniform over the 1024 units
        after now0."""
        from paper_1712_09624_amd.ckpp import Table
        cfg = W.many_tables(ntables, seed, log2_lo, log2_hi, 0.6, 0.95, batch_lo, batch_hi)
        self.refs, self.tables, self.keys, self.live = [], [], [], []
        self.modes = []
        offsets, counts, chunks = [], [], []
        pos = 0
        for i in range(ntables):
            B = int(cfg["log2_buckets"][i])
            plain = bool(plain_every) and i % plain_every == plain_every - 1
            timed = bool(timed_every) and i % timed_every == 1
            n = W.keys_at_load(B, float(cfg["load"][i]))
            keys = W.distinct_five_tuples(n, seed * 1000 + i)
            ref = O.OracleTable(B, W.HASH_SEED, W.MAX_KICKS, plain, timed=timed)
            if timed:
                exp = W.times_after(n, now0, 1024, seed * 1000 + i)
                ref.insert_at(keys, W.insertion_values(n, 1000 * i), exp, now0)
            else:
                ref.insert(keys, W.insertion_values(n, 1000 * i))
            t = Table(B, W.HASH_SEED, W.MAX_KICKS, plain=plain, device=0, timers=timed)
            b, k = ref.image()
            t.import_image(b, k)
            cnt = int(cfg["batch"][i])
            if zero_every and i % zero_every == 0:
                cnt = 0
            look, _, _ = W.lookup_mix(keys, cnt, float(cfg["neg_rate"][i]), seed * 1000 + i)
            gap = i % 3  # unused positions between ranges
            pos += gap
            chunks.append(np.zeros((gap, 16), np.uint8))
            offsets.append(pos)
            counts.append(cnt)
            chunks.append(look)
            pos += cnt
            mode = modes[i % len(modes)] if modes else "cuckoopp"
            self.modes.append(mode)
            self.refs.append(ref)
            self.tables.append(t)
            self.keys.append(look)
        self.offsets = np.array(offsets, np.uint64)
        self.counts = np.array(counts, np.uint64)
        self.all_keys = np.concatenate(chunks) if chunks else np.zeros((0, 16), np.uint8)
        self.span = pos

    def expected(self, now=None, refresh=None):
        """Oracle answers at every position; sentinels outside the ranges.
        Tables with timers answer at `now`, refreshing found entries to
        `refresh` when it is given."""
        f = np.full(self.span, SENTINEL_F, np.uint8)
        v = np.full(self.span, SENTINEL_V, np.uint64)
        for i, ref in enumerate(self.refs):
            o, c = int(self.offsets[i]), int(self.counts[i])
            if c == 0:
                continue
            mode = self.modes[i]
            if mode == "cuckoopp" and ref.plain:
                mode = "both"
            if ref.timed:
                wf, wv = ref.lookup_at(self.keys[i], now, OMODE[mode], refresh=refresh)
            else:
                wf, wv, _, _ = ref.lookup(self.keys[i], OMODE[mode])
            f[o:o + c] = wf
            v[o:o + c] = wv
        return f, v

    def close(self):
        for t in self.tables:
            t.close()


def ckpp_default_plan_launch():
    from paper_1712_09624_amd import ckpp
    return ckpp.DEFAULT_PLAN_LAUNCH


def run_plan(plan, fleet, **lookup_args):
    import torch
    keys = to_dev(fleet.all_keys)
    found = torch.full((fleet.span,), SENTINEL_F, dtype=torch.uint8, device="cuda:0")
    vals = torch.full((fleet.span,), SENTINEL_V, dtype=torch.int64, device="cuda:0")
    plan.lookup(keys, found, vals, **lookup_args)
    return u8(found), u64(vals)


@pytest.fixture(scope="module")
def fleet():
    # 48 tables of 2^1..2^12 buckets, batches 0..700 (every 7th empty),
    # every 5th table plain, modes cycling through the three
    f = Fleet(48, 3, 1, 12, 1, 700, plain_every=5, modes=["cuckoopp", "optimistic", "both"],
              zero_every=7)
    yield f
    f.close()


@pytest.mark.parametrize("shape", PLAN_SHAPES, ids=[f"per{a}_b{b}_bpc{c}_p{d}_s{e}_l{g}"
                                                    for a, b, c, d, e, g in PLAN_SHAPES])
def test_plan_matches_oracle(fleet, shape):
    from paper_1712_09624_amd.ckpp import Plan
    want_f, want_v = fleet.expected()
    plan = Plan(fleet.tables, fleet.offsets, fleet.counts, fleet.modes)
    plan.set_launch(*shape)
    assert plan.get_launch() == dict(zip(("lookups_per_lane", "block", "blocks_per_cu",
                                          "passes_per_item", "schedule", "lanes_per_lookup"),
                                         shape))
    say(f"plan lookup shape={shape} tables={len(fleet.tables)} span={fleet.span}")
    for rep in range(2):  # a second launch starts from the rewound counters
        f, v = run_plan(plan, fleet)
        assert np.array_equal(f, want_f), f"found differs (launch {rep})"
        assert np.array_equal(v, want_v), f"values differ (launch {rep})"
    plan.close()


NO_PESSIMISTIC_SHAPES = [(1, 128, 8, 1, 0, 8), (2, 256, 4, 1, 1, 8), (1, 128, 8, 1, 0, 4),
                         (1, 64, 4, 2, 1, 4), (2, 256, 16, 3, 0, 4), (2, 64, 8, 1, 1, 4),
                         (2, 128, 8, 1, 0, 1)]


@pytest.mark.parametrize("shape", NO_PESSIMISTIC_SHAPES,
                         ids=[f"per{a}_b{b}_bpc{c}_p{d}_s{e}_l{g}"
                              for a, b, c, d, e, g in NO_PESSIMISTIC_SHAPES])
def test_plan_without_pessimistic_tables(shape):
    """A plan with no pessimistic table runs the kernel built without that
    mode (one line buffer with 8 lanes, fewer registers with 4)."""
    from paper_1712_09624_amd.ckpp import Plan
    f = Fleet(40, 13, 1, 12, 1, 900, modes=["cuckoopp", "optimistic"], zero_every=9)
    want_f, want_v = f.expected()
    plan = Plan(f.tables, f.offsets, f.counts, f.modes)
    plan.set_launch(*shape)
    say(f"plan without pessimistic tables, shape={shape} span={f.span}")
    got_f, got_v = run_plan(plan, f)
    assert np.array_equal(got_f, want_f) and np.array_equal(got_v, want_v)
    plan.close()
    f.close()


TIMED_SHAPES = [(1, 128, 8, 1, 0, 8), (2, 64, 4, 2, 1, 8), (1, 128, 8, 1, 0, 4),
                (2, 256, 2, 3, 1, 4), (1, 64, 8, 1, 0, 1), (4, 128, 4, 2, 1, 1)]


@pytest.mark.parametrize("shape", TIMED_SHAPES, ids=[f"per{a}_b{b}_bpc{c}_p{d}_s{e}_l{g}"
                                                     for a, b, c, d, e, g in TIMED_SHAPES])
def test_plan_with_tables_with_timers(shape):
    """Tables with and without timers in one plan: a table with timers
    answers as the oracle's lookups at the launch's time (the clock wraps),
    the others as without timers."""
    from paper_1712_09624_amd.ckpp import CkppError, Plan
    now0 = 65000
    f = Fleet(30, 17, 1, 11, 1, 900, plain_every=4, modes=["cuckoopp", "optimistic", "both"],
              zero_every=8, timed_every=2, now0=now0)
    plan = Plan(f.tables, f.offsets, f.counts, f.modes)
    plan.set_launch(*shape)
    for dt in (0, 500, 1023, 1024):
        now = (now0 + dt) & 0xFFFF
        want_f, want_v = f.expected(now=now)
        say(f"timed plan shape={shape} now={now}")
        got_f, got_v = run_plan(plan, f, now=now)
        assert np.array_equal(got_f, want_f), f"found differs at now={now}"
        assert np.array_equal(got_v, want_v), f"values differ at now={now}"
    with pytest.raises(CkppError):  # a plan with timed tables runs with a time
        run_plan(plan, f)
    plan.close()
    f.close()


def test_plan_refreshing_lookup_with_tables_with_timers():
    """A refreshing plan lookup leaves every table's image as the oracle's
    refreshing lookups do (the tables without timers untouched)."""
    from paper_1712_09624_amd.ckpp import CkppError, Plan
    now0 = 200
    f = Fleet(20, 19, 2, 10, 1, 900, modes=["cuckoopp", "optimistic"], timed_every=2, now0=now0)
    plan = Plan(f.tables, f.offsets, f.counts, f.modes)
    now, new_exp = now0 + 300, now0 + 1000
    with pytest.raises(CkppError):  # a refresh time outside [now, now + 1023]
        run_plan(plan, f, now=now, refresh=now + 1024)
    want_f, want_v = f.expected(now=now, refresh=new_exp)
    say("refreshing timed plan lookup")
    got_f, got_v = run_plan(plan, f, now=now, refresh=new_exp)
    assert np.array_equal(got_f, want_f) and np.array_equal(got_v, want_v)
    for ref, t in zip(f.refs, f.tables):
        gb, gk = t.export()
        rb, rk = ref.image()
        assert np.array_equal(gb, rb) and np.array_equal(gk, rk), "images differ after refresh"
    plan.close()
    f.close()


def test_plan_equals_per_table_calls(fleet):
    """The plan's answers are those of one ckpp_lookup_batch per table."""
    from paper_1712_09624_amd.ckpp import Plan
    plan = Plan(fleet.tables, fleet.offsets, fleet.counts, fleet.modes)
    say("plan vs per-table lookup calls")
    f, v = run_plan(plan, fleet)
    for i, t in enumerate(fleet.tables):
        o, c = int(fleet.offsets[i]), int(fleet.counts[i])
        if c == 0:
            continue
        tf, tv = t.lookup(to_dev(fleet.keys[i]), fleet.modes[i])
        assert np.array_equal(u8(tf), f[o:o + c]) and np.array_equal(u64(tv), v[o:o + c])
    plan.close()


def test_plan_info_and_items():
    from paper_1712_09624_amd.ckpp import Plan
    f = Fleet(5, 9, 4, 6, 1, 300)
    plan = Plan(f.tables, f.offsets, f.counts)
    inf = plan.info()
    assert inf["ntables"] == 5 and inf["lookups"] == int(f.counts.sum())
    assert inf["key_span"] == f.span
    assert plan.get_launch() == ckpp_default_plan_launch()
    for per, passes, lanes in ((1, 1, 8), (2, 1, 8), (2, 4, 8), (1, 3, 4), (2, 2, 4), (4, 2, 1)):
        plan.set_launch(per, 128, 4, passes, 0, lanes)
        tile = 64 * per * passes
        assert plan.info()["nitems"] == int(sum((int(c) + tile - 1) // tile for c in f.counts))
    plan.close()
    f.close()


def test_plan_rejects_bad_arguments():
    import torch
    from paper_1712_09624_amd.ckpp import CkppError, Plan
    f = Fleet(3, 11, 4, 5, 10, 20)
    with pytest.raises(CkppError):  # overlapping ranges
        Plan(f.tables, [0, 5, 100], [10, 10, 10])
    with pytest.raises(CkppError):  # unknown mode
        Plan(f.tables, [0, 20, 40], [10, 10, 10], modes=[0, 7, 0])
    plan = Plan(f.tables, [0, 20, 40], [10, 10, 10])
    with pytest.raises(CkppError):
        plan.set_launch(3, 128, 8, 1)
    with pytest.raises(CkppError):
        plan.set_launch(2, 96, 8, 1)
    with pytest.raises(CkppError):
        plan.set_launch(2, 128, 0, 1)
    with pytest.raises(CkppError):
        plan.set_launch(2, 128, 4, 1, 2)
    with pytest.raises(CkppError):  # four lookups per lane need one lane per lookup
        plan.set_launch(4, 128, 4, 1, 0, 8)
    with pytest.raises(CkppError):  # two lanes per lookup: no such form
        plan.set_launch(1, 128, 4, 1, 0, 2)
    with pytest.raises(CkppError):  # four lookups per lane need one lane per lookup
        plan.set_launch(4, 128, 4, 1, 0, 4)
    with pytest.raises(CkppError):  # fewer keys than the plan's span
        plan.lookup(torch.zeros((30, 16), dtype=torch.uint8, device="cuda:0"))
    plan.close()
    # a plan whose batches are all empty launches nothing
    empty = Plan(f.tables, [0, 0, 0], [0, 0, 0])
    say("empty plan")
    fo, vo = empty.lookup(torch.zeros((1, 16), dtype=torch.uint8, device="cuda:0"))
    torch.cuda.synchronize()
    empty.close()
    f.close()


def test_plan_graph_replays_follow_table_updates():
    """One plan launch captured in a HIP graph and replayed three times, with
    eager inserts and deletes on the tables between the replays: every
    replay equals the eager plan lookup and the per-table oracle answers."""
    import torch
    from paper_1712_09624_amd.ckpp import Plan
    f = Fleet(12, 21, 6, 11, 100, 900)
    plan = Plan(f.tables, f.offsets, f.counts)
    keys = to_dev(f.all_keys)
    g_found = torch.zeros(f.span, dtype=torch.uint8, device="cuda:0")
    g_vals = torch.zeros(f.span, dtype=torch.int64, device="cuda:0")
    plan.lookup(keys, g_found, g_vals)  # warm-up outside the capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    say("capturing plan lookup")
    with torch.cuda.graph(graph):
        plan.lookup(keys, g_found, g_vals)
    torch.cuda.synchronize()
    for rep in range(3):
        if rep:
            # eager work on the default stream between replays: delete a
            # slice of each batch's keys and insert the batch's first keys
            # with new values
            for i, (t, ref) in enumerate(zip(f.tables, f.refs)):
                look = f.keys[i]
                dk = look[rep::7]
                t.delete(to_dev(dk))
                ref.delete(dk)
                ik = np.unique(look[:5], axis=0)
                iv = np.arange(ik.shape[0], dtype=np.uint64) + np.uint64(10**9 * rep + 1000 * i)
                st, _ = t.insert(to_dev(ik), vals_dev(iv))
                assert (u8(st) != O.FAILED).all()
                assert (ref.insert(ik, iv) != O.FAILED).all()
            torch.cuda.synchronize()
        want_f, want_v = f.expected()
        say(f"graph replay {rep}")
        g_found.fill_(SENTINEL_F)
        g_vals.fill_(SENTINEL_V)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        e_found, e_vals = run_plan(plan, f)
        assert np.array_equal(u8(g_found), want_f) and np.array_equal(u64(g_vals), want_v)
        assert np.array_equal(e_found, want_f) and np.array_equal(e_vals, want_v)
    del graph
    plan.close()
    f.close()
