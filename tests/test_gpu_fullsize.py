"""Full-size GPU checks, at the shapes the benchmark runs (2^24 buckets x 8
slots) and in its launch configuration.

The oracle cannot build tables of 120M+ keys within a test, so these check
every output against properties that hold at any size: the dictionary
definition of the result (an inserted key is found with the value it was
given -- its insertion index -- and a key never inserted or deleted misses
with value 0), agreement of the three lookup modes, and the oracle's image
invariants on the exported table."""

import numpy as np
import pytest

from gpu_util import say, to_dev, u64, u8, vals_dev
from oracle import oracle as O
from paper_1712_09624_amd import workload as W

pytestmark = pytest.mark.gpu

B = 24


def build(keys, vals, batch):
    import torch
    from paper_1712_09624_amd.ckpp import Table
    t = Table(B, W.HASH_SEED, W.MAX_KICKS, device=0)
    dk, dv = to_dev(keys), vals_dev(vals)
    st = torch.empty(len(keys), dtype=torch.uint8, device="cuda:0")
    nf = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    for s in range(0, len(keys), batch):
        t.insert(dk[s:s + batch], dv[s:s + batch], status=st[s:s + batch], nfailed=nf)
    torch.cuda.synchronize()
    del dk, dv
    return t, u8(st), int(nf.item())


def check_lookups(t, keys, want_found, want_vals, chunk=1 << 26):
    for s in range(0, len(keys), chunk):
        q = to_dev(keys[s:s + chunk])
        ref_f, ref_v = None, None
        for mode in ("cuckoopp", "both", "optimistic"):
            f, v = t.lookup(q, mode)
            f, v = u8(f), u64(v)
            if ref_f is None:
                ref_f, ref_v = f, v
                assert np.array_equal(f, want_found[s:s + chunk]), "found flags"
                assert np.array_equal(v, want_vals[s:s + chunk]), "values"
            else:
                assert np.array_equal(f, ref_f) and np.array_equal(v, ref_v), f"mode {mode} differs"


def check_image(t, plain=False):
    b, k = t.export()
    rc, msg = O.check_image(b, k, B, W.HASH_SEED, plain)
    assert rc == 0, msg


def test_benchmark_table_lookups():
    """The benchmark's table (load 0.9, built in 4M-key batches) and its
    lookup batches: 2^26 positive and 2^26 negative keys."""
    n = W.keys_at_load(B, 0.9)
    say(f"full size: generating {n} keys")
    keys = W.distinct_five_tuples(n, 1)
    vals = W.insertion_values(n)
    say("full size: build 2^24 buckets at load 0.9")
    t, st, nf = build(keys, vals, 1 << 22)
    assert nf == 0 and (st == O.INSERTED).all()
    s = t.stats()
    assert s["live"] == n and s["locked"] == 0 and s["retry_exhausted"] == 0
    pos, _, idx = W.lookup_mix(keys, 1 << 26, 0.0, 2)
    neg = W.five_tuples(1 << 26, 3, stream=W.STREAM_NEGATIVE)
    say("full size: 2^26 positive lookups, three modes")
    check_lookups(t, pos, np.ones(len(pos), np.uint8), vals[idx])
    say("full size: 2^26 negative lookups, three modes")
    check_lookups(t, neg, np.zeros(len(neg), np.uint8), np.zeros(len(neg), np.uint64))
    # the other lookup forms the tuners choose from: 4 lanes and 1 lane per lookup
    for shape in ((4, 1, 256, 0), (1, 2, 128, 0)):
        t.set_lookup_launch(*shape)
        say(f"full size: positive and negative lookups, three modes, shape {shape}")
        check_lookups(t, pos, np.ones(len(pos), np.uint8), vals[idx])
        check_lookups(t, neg, np.zeros(len(neg), np.uint8), np.zeros(len(neg), np.uint64))
    say("full size: image invariants")
    check_image(t)
    t.close()


def test_batched_build_delete_reinsert():
    """Insert workload: an empty 2^24-bucket table filled to load 0.95 in
    batches of 65536 keys, a random 20% deleted, as many fresh keys
    re-inserted; every live, deleted and fresh key is then looked up."""
    n = W.keys_at_load(B, 0.95)
    say(f"insert workload: generating {n} keys")
    keys = W.distinct_five_tuples(n, 11)
    vals = W.insertion_values(n)
    say("insert workload: build in batches of 65536")
    t, st, nf = build(keys, vals, 65536)
    assert set(np.unique(st)) <= {O.INSERTED, O.FAILED}
    ins = st == O.INSERTED
    assert nf == int((~ins).sum())
    assert nf <= n // 100000, f"{nf} failures at load 0.95"
    nd = n // 5
    rows = W.choose_rows(n, nd, 12)
    say(f"insert workload: delete {nd}")
    d = u8(t.delete(to_dev(keys[rows])))
    assert np.array_equal(d, ins[rows].astype(np.uint8))
    fresh = W.distinct_five_tuples(nd, 13, stream=W.STREAM_FRESH)
    fvals = W.insertion_values(nd, n)
    import torch
    say(f"insert workload: re-insert {nd}")
    st2 = torch.empty(nd, dtype=torch.uint8, device="cuda:0")
    dk, dv = to_dev(fresh), vals_dev(fvals)
    for s in range(0, nd, 65536):
        t.insert(dk[s:s + 65536], dv[s:s + 65536], status=st2[s:s + 65536])
    st2 = u8(st2)
    assert set(np.unique(st2)) <= {O.INSERTED, O.FAILED}
    live = ins.copy()
    live[rows] = False
    want_f = live.astype(np.uint8)
    want_v = np.where(live, vals, 0).astype(np.uint64)
    ins2 = st2 == O.INSERTED
    s = t.stats()
    assert s["live"] == int(live.sum()) + int(ins2.sum()) and s["retry_exhausted"] == 0
    say("insert workload: lookups of all original keys")
    check_lookups(t, keys, want_f, want_v)
    say("insert workload: lookups of the fresh keys")
    check_lookups(t, fresh, ins2.astype(np.uint8), np.where(ins2, fvals, 0).astype(np.uint64))
    say("insert workload: image invariants")
    check_image(t)
    t.close()


def test_benchmark_table_with_timers():
    """The benchmark's table with timers (expiration times uniform over the
    1024 units after 65000, so the window wraps) in the default launch
    configuration: at 65000 every key is found with its value; at 65512
    exactly the keys whose time has not passed; a refreshing lookup keeps
    every key it finds alive until its new time; the scan then removes the
    rest, and the invariants hold throughout."""
    import torch
    from paper_1712_09624_amd.ckpp import Table
    n = W.keys_at_load(B, 0.9)
    keys = W.distinct_five_tuples(n, 1)
    vals = W.insertion_values(n)
    now0 = 65000
    exp = W.times_after(n, now0, 1024, 1)
    say("full size timers: build 2^24 buckets at load 0.9")
    t = Table(B, W.HASH_SEED, W.MAX_KICKS, device=0, timers=True)
    nf = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    for s in range(0, n, 1 << 22):
        t.insert_at(to_dev(keys[s:s + (1 << 22)]), vals_dev(vals[s:s + (1 << 22)]),
                    to_dev(exp[s:s + (1 << 22)].view(np.int16)), now0, nfailed=nf)
    torch.cuda.synchronize()
    assert int(nf.item()) == 0
    pos, _, idx = W.lookup_mix(keys, 1 << 26, 0.0, 2)
    dpos = to_dev(pos)
    say("full size timers: lookups at the build time")
    f, v = t.lookup_at(dpos, now0)
    assert u8(f).all() and np.array_equal(u64(v), vals[idx])
    half = (now0 + 512) & 0xFFFF
    alive = (((exp.astype(np.int64) - half) & 0xFFFF) < 1024)
    say("full size timers: lookups half way, with refresh")
    new_exp = (half + 1000) & 0xFFFF
    f, v = t.lookup_at(dpos, half, refresh=new_exp)
    f, v = u8(f), u64(v)
    assert np.array_equal(f, alive[idx].astype(np.uint8))
    assert np.array_equal(v, np.where(alive[idx], vals[idx], 0).astype(np.uint64))
    refreshed = np.zeros(n, bool)
    refreshed[idx[f == 1]] = True
    later = (half + 700) & 0xFFFF
    say("full size timers: scan")
    removed = t.expire_scan(later)
    want_alive = refreshed  # every other entry has expired by then
    assert int(removed.item()) == n - int(want_alive.sum())
    assert t.stats()["live"] == int(want_alive.sum())
    f, v = t.lookup_at(to_dev(keys), later)
    assert np.array_equal(u8(f), want_alive.astype(np.uint8))
    b, k = t.export()
    rc, msg = O.check_image(b, k, B, W.HASH_SEED, timed=True)
    assert rc == 0, msg
    t.close()
