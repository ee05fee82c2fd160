"""Serving rounds of every size class of the lookup phase, against the
oracle, bit-exact: the phase runs 4, 2 or 1 lookups per lane per pass in
registers, the most that every lane of the loop's grid has (on a 256-block
grid of 512-thread blocks, 131 072 lanes: 4 from 524 288 lookups in a round,
2 from 262 144).  Bursts of 600 013, 300 007, 150 001 and 70 001 lookups
(each size class, with a ragged last pass), half of them of
stored keys, half fresh, the first with inserts and deletes in the same
round, on a table without timers in the Cuckoo++, optimistic and
pessimistic modes; and a 300 007-lookup burst on a table with timers whose
lookups renew the entries they find."""

import numpy as np
import pytest

from gpu_util import say, to_dev, u64, u8, vals_dev
from oracle import oracle as O
from paper_1712_09624_amd import workload as W

pytestmark = pytest.mark.gpu

OMODES = {"cuckoopp": O.MODE_CUCKOOPP, "optimistic": O.MODE_OPTIMISTIC, "both": O.MODE_BOTH}


def mixed_lookups(keys, n, rng, fresh):
    pos = keys[rng.integers(0, len(keys), n)]
    return np.ascontiguousarray(np.where((rng.random(n) < 0.5)[:, None], fresh[:n], pos))


@pytest.mark.parametrize("mode", ["cuckoopp", "optimistic", "both"])
def test_large_rounds_match_oracle(mode):
    import torch
    from paper_1712_09624_amd.ckpp import Server, Table
    B = 17
    n = W.keys_at_load(B, 0.85)
    keys = W.distinct_five_tuples(n, 61)
    ref = O.OracleTable(B, W.HASH_SEED, W.MAX_KICKS, False)
    assert (ref.insert(keys, W.insertion_values(n)) == O.INSERTED).all()
    t = Table(B, W.HASH_SEED, W.MAX_KICKS, device=0)
    t.import_image(*ref.image())
    rng = np.random.default_rng(62)
    fresh = W.five_tuples(1 << 20, 63, W.STREAM_FRESH)
    # deletes take stored keys that no lookup of the test reads; inserts are
    # fresh keys beyond the lookups' share
    perm = rng.permutation(n)
    dels, pool = keys[perm[:500]], keys[perm[500:]]
    bursts = []
    for nl, ni, nd, off in ((600_013, 1000, 500, 0), (300_007, 0, 0, 600_013),
                            (150_001, 0, 0, 300_000), (70_001, 0, 0, 700_000)):
        look = mixed_lookups(pool, nl, rng, fresh[off:])
        ins = np.ascontiguousarray(fresh[950_000:950_000 + ni])
        iv = np.arange(ni, dtype=np.uint64) + np.uint64(7 << 40)
        bursts.append((look, ins, iv, np.ascontiguousarray(dels[:nd])))
    want = []
    for look, ins, iv, dl in bursts:
        f, v, _, _ = ref.lookup(look, OMODES[mode])
        st = ref.insert(ins, iv) if len(ins) else np.zeros(0, np.uint8)
        df = ref.delete(dl) if len(dl) else np.zeros(0, np.uint8)
        want.append((f.astype(np.uint8), v.astype(np.uint64), st.astype(np.uint8),
                     df.astype(np.uint8)))
    with Server(t, capacity=1 << 20, mode=mode, idle_ms=500) as srv:
        for b, (look, ins, iv, dl) in enumerate(bursts):
            say(f"large round mode={mode} burst {b}: {len(look)} lookups, {len(ins)} inserts, "
                f"{len(dl)} deletes")
            counts, first = srv.put_burst(
                lookup_keys=to_dev(look),
                insert_keys=to_dev(ins) if len(ins) else None,
                insert_values=vals_dev(iv) if len(ins) else None,
                delete_keys=to_dev(dl) if len(dl) else None)
            bid = srv.submit(*counts)
            assert bid is not None
            srv.wait(bid, 20000)
            f, v = srv.get("lookup", first[0], counts[0])
            st = srv.get("insert", first[1], counts[1])
            df = srv.get("delete", first[2], counts[2])
            torch.cuda.current_stream().synchronize()
            for g, x, name in zip((u8(f), u64(v), u8(st), u8(df)), want[b],
                                  ("lookup found", "lookup values", "insert status",
                                   "delete found")):
                assert np.array_equal(g, x), f"burst {b}: {name} differs"
            assert int(u8(f).sum()) > len(look) // 3
    t.close()


def test_large_timed_round_renews_what_it_finds():
    import torch
    from paper_1712_09624_amd.ckpp import Server, Table
    B, now, ttl = 16, 1000, 500
    n = W.keys_at_load(B, 0.85)
    keys = W.distinct_five_tuples(n, 71)
    exp = W.times_after(n, now, 1024, 71)
    ref = O.OracleTable(B, W.HASH_SEED, W.MAX_KICKS, False, timed=True)
    assert (ref.insert_at(keys, W.insertion_values(n), exp, now) == O.INSERTED).all()
    t = Table(B, W.HASH_SEED, W.MAX_KICKS, device=0, timers=True)
    t.import_image(*ref.image())
    rng = np.random.default_rng(72)
    fresh = W.five_tuples(1 << 19, 73, W.STREAM_FRESH)
    look = mixed_lookups(keys, 300_007, rng, fresh)
    e = (now + ttl) & 0xFFFF
    wf, wv = ref.lookup_at(look, now, O.MODE_CUCKOOPP, refresh=e)
    with Server(t, capacity=1 << 19, idle_ms=500, ttl=ttl, refresh=True) as srv:
        assert srv.set_time(now)
        say(f"large timed round: {len(look)} lookups at time {now}, renewing to {e}")
        counts, first = srv.put_burst(lookup_keys=to_dev(look))
        bid = srv.submit(*counts)
        assert bid is not None
        srv.wait(bid, 20000)
        f, v = srv.get("lookup", first[0], counts[0])
        torch.cuda.current_stream().synchronize()
        assert np.array_equal(u8(f), wf), "found differs"
        assert np.array_equal(u64(v), wv), "values differ"
    # after the renewals, every key's state at a later time before e agrees
    # with the oracle's (renewed entries live to e, the others to their own
    # expiration time, some of them earlier)
    later = now + 400
    pf, pv = ref.lookup_at(keys, later, O.MODE_CUCKOOPP)
    gf, gv = t.lookup_at(to_dev(keys), later, "cuckoopp")
    assert np.array_equal(u8(gf), pf) and np.array_equal(u64(gv), pv)
    assert 0 < int(pf.sum()) < n
    t.close()
