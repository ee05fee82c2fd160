"""The serving loop on tables with timers (Sec. 4.2) against the oracle,
bit-exact: every burst runs at the server's time when it was submitted
(lookups find alive entries and renew them, inserts give their entries
expiration time now + ttl, deletes report alive keys), and the server runs
the anti-revival scan itself whenever its time has advanced 16384 units
since the last one.  The clock wraps and advances by more than 64512 units
in all, so an entry that expired early would look alive again without the
scans; the oracle takes the scans at the same times.

Bursts of one time are submitted back to back; their writes concern keys
that no other burst of that time reads (inserts are fresh keys, deletes take
keys no burst of that time looks up), so the oracle applies them one by
one."""

import numpy as np
import pytest

from gpu_util import say, to_dev, u64, u8, vals_dev
from oracle import oracle as O
from paper_1712_09624_amd import workload as W

pytestmark = pytest.mark.gpu

SCAN_STEP = 16384  # the server's scan is due once its time is this far past the last


def timed_oracle_and_table(B, load, now0, seed, plain):
    from paper_1712_09624_amd.ckpp import Table
    n = W.keys_at_load(B, load)
    keys = W.distinct_five_tuples(n, seed)
    exp = W.times_after(n, now0, 1024, seed)
    ref = O.OracleTable(B, W.HASH_SEED, W.MAX_KICKS, plain, timed=True)
    assert (ref.insert_at(keys, W.insertion_values(n), exp, now0) == O.INSERTED).all()
    t = Table(B, W.HASH_SEED, W.MAX_KICKS, plain=plain, device=0, timers=True)
    b, k = ref.image()
    t.import_image(b, k)
    return ref, t, keys


OMODES = {"cuckoopp": O.MODE_CUCKOOPP, "both": O.MODE_BOTH, "optimistic": O.MODE_OPTIMISTIC}


@pytest.mark.parametrize("plain,refresh,mode", [(False, True, "cuckoopp"), (True, True, "both"),
                                                (False, False, "cuckoopp"),
                                                (False, True, "optimistic"),
                                                (False, True, "both")])
def test_timed_server_matches_oracle(plain, refresh, mode):
    import torch
    from paper_1712_09624_amd.ckpp import Server
    B, ttl, now = 11, 300, 65000
    ref, t, keys = timed_oracle_and_table(B, 0.6, now, 40 + plain, plain)
    omode = OMODES[mode]
    rng = np.random.default_rng(7 + plain + 2 * refresh + 4 * len(mode))
    fresh = W.five_tuples(200000, 41, W.STREAM_FRESH)
    fi = 0
    pool = [k for k in keys]  # keys a burst may look up or delete
    inserted = []
    # steps: small ones (renewed entries stay alive), and large ones that
    # together pass 64512 units, wrapping the clock twice
    steps = [0, 40, 120, 250, 14000, 90, 14000, 14000, 14000, 200, 14000, 60, 9000]
    last_scan = None
    with Server(t, capacity=1 << 13, mode=mode, idle_ms=500, ttl=ttl, refresh=refresh) as srv:
        for si, step in enumerate(steps):
            now = (now + step) & 0xFFFF
            assert srv.set_time(now)
            if last_scan is None or ((now - last_scan) & 0xFFFF) >= SCAN_STEP:
                ref.expire_scan(now)
                last_scan = now
            # the bursts of this time: disjoint delete picks, lookups of the
            # rest of the pool and of fresh keys, inserts of fresh keys
            perm = rng.permutation(len(pool))
            nb = 3
            dpick = [perm[20 * b: 20 * b + int(rng.integers(0, 21))] for b in range(nb)]
            rest = perm[20 * nb:]
            bursts = []
            for b in range(nb):
                nl, ni = int(rng.integers(1, 300)), int(rng.integers(0, 50))
                pos = np.stack([pool[i] for i in rest[rng.integers(0, len(rest), nl)]])
                neg = fresh[fi:fi + nl]
                fi += nl
                look = np.where((rng.random(nl) < 0.3)[:, None], neg, pos)
                ins = fresh[fi:fi + ni]
                fi += ni
                ivals = rng.integers(0, 1 << 48, size=ni, dtype=np.int64).astype(np.uint64)
                # values of 2^48 or more: refused by the device layout of
                # tables with timers (FAILED, nothing changes for the key)
                ivals[rng.random(ni) < 0.05] |= np.uint64(1 << 50)
                dels = np.stack([pool[i] for i in dpick[b]]) if len(dpick[b]) else fresh[:0]
                bursts.append((np.ascontiguousarray(look), np.ascontiguousarray(ins), ivals,
                               np.ascontiguousarray(dels)))
            # the oracle, burst by burst
            want = []
            e = (now + ttl) & 0xFFFF
            for look, ins, ivals, dels in bursts:
                f, v = ref.lookup_at(look, now, omode, refresh=e if refresh else None)
                st = np.full(len(ins), O.FAILED, np.uint8)
                fits = (ivals >> np.uint64(48)) == 0
                if fits.any():
                    st[fits] = ref.insert_at(ins[fits], ivals[fits],
                                             np.full(int(fits.sum()), e, np.uint16), now)
                df = ref.delete_at(dels, now) if len(dels) else np.zeros(0, np.uint8)
                want.append((f.astype(np.uint8), v.astype(np.uint64), st.astype(np.uint8),
                             df.astype(np.uint8)))
            say(f"timed server plain={plain} refresh={refresh} mode={mode} step {si}: now={now} "
                f"scan={last_scan == now} bursts={[(len(x[0]), len(x[1]), len(x[3])) for x in bursts]}")
            placed = []
            for look, ins, ivals, dels in bursts:
                placed.append(srv.put_burst(
                    lookup_keys=to_dev(look),
                    insert_keys=to_dev(ins) if len(ins) else None,
                    insert_values=vals_dev(ivals) if len(ins) else None,
                    delete_keys=to_dev(dels) if len(dels) else None))
            ids = [srv.submit(*c) for c, _ in placed]
            assert None not in ids
            srv.wait(ids[-1], 10000)
            for b, ((c, first), w) in enumerate(zip(placed, want)):
                f, v = srv.get("lookup", first[0], c[0])
                st = srv.get("insert", first[1], c[1])
                df = srv.get("delete", first[2], c[2])
                torch.cuda.current_stream().synchronize()
                for g, x, name in zip((u8(f), u64(v), u8(st), u8(df)), w,
                                      ("lookup found", "lookup values", "insert status",
                                       "delete found")):
                    assert np.array_equal(g, x), f"step {si} burst {b}: {name} differs"
            # the pool loses the deleted keys and gains the inserted ones
            gone = set(int(i) for d in dpick for i in d)
            pool = [k for i, k in enumerate(pool) if i not in gone]
            for (look, ins, ivals, dels), w in zip(bursts, want):
                ok = w[2] != O.FAILED
                pool.extend(ins[ok])
                inserted.extend(ins[ok])
        st = srv.status()
        assert st["completed"] == st["submitted"]
        # a round never spans two times: at least one round per time
        assert st["rounds"] >= len(steps)
    # the whole dictionary at the final time, and the image invariants
    probe = np.concatenate([keys, np.stack(inserted), fresh[:5000]])
    for mode, om in (("cuckoopp", O.MODE_CUCKOOPP), ("both", O.MODE_BOTH)):
        wf, wv = ref.lookup_at(probe, now, om)
        gf, gv = t.lookup_at(to_dev(probe), now, mode)
        assert np.array_equal(u8(gf), wf), f"final {mode}: found differs"
        assert np.array_equal(u64(gv), wv), f"final {mode}: values differ"
    assert int(wf.sum()) > 0
    bk, kv = t.export()
    rc, msg = O.check_image(bk, kv, B, W.HASH_SEED, plain, timed=True)
    assert rc == 0, msg
    # once both tables drop their expired entries, they hold the same number
    # (which expired entries an insert overwrote depends on the order of
    # concurrent inserts; the alive ones do not)
    ref.expire_scan(now)
    t.expire_scan(now)
    torch.cuda.synchronize()
    st_t, st_r = t.stats(), ref.stats()
    assert st_t["live"] == st_r["live"] and st_t["locked"] == 0
    t.close()


def test_timed_server_argument_checks():
    """ttl must fit the table's kind; set_time refuses servers without
    timers and steps of 16384 or more, and accepts the same time again."""
    from paper_1712_09624_amd import ckpp
    from paper_1712_09624_amd.ckpp import CkppError, Server, Table
    t = Table(8, W.HASH_SEED, W.MAX_KICKS, device=0, timers=True)
    u = Table(8, W.HASH_SEED, W.MAX_KICKS, device=0)
    for bad in (0, 1024, ckpp.SERVER_REFRESH):
        with pytest.raises(CkppError):
            Server(t, capacity=1 << 8, idle_ms=100, ttl=bad)
    with pytest.raises(CkppError):
        Server(u, capacity=1 << 8, idle_ms=100, ttl=10)
    with Server(u, capacity=1 << 8, idle_ms=100) as srv:
        with pytest.raises(CkppError):
            srv.set_time(5)
    with Server(t, capacity=1 << 8, idle_ms=100, ttl=1023, refresh=True) as srv:
        assert srv.set_time(60000)
        assert srv.set_time(60000)
        with pytest.raises(CkppError):
            srv.set_time((60000 + SCAN_STEP) & 0xFFFF)
        assert srv.set_time((60000 + SCAN_STEP - 1) & 0xFFFF)
        # one empty burst for the scan at the first time; the step of 16383
        # is not 16384 past that scan, so no second one
        assert srv.status()["submitted"] == 1
    t.close()
    u.close()


def test_timed_server_scan_relaunches_an_idle_loop():
    """The loop exits when idle; a time change that makes the scan due
    submits its burst, which relaunches the loop, and the scan runs before
    the next burst: entries that expired before the new time are gone
    (the oracle agrees on every answer and on the stored-entry count)."""
    import time
    import torch
    from paper_1712_09624_amd import ckpp
    from paper_1712_09624_amd.ckpp import Server
    B, now = 9, 1000
    ref, t, keys = timed_oracle_and_table(B, 0.5, now, 77, False)
    with Server(t, capacity=1 << 12, idle_ms=20, ttl=100) as srv:
        assert srv.set_time(now)  # first time: a scan
        ref.expire_scan(now)
        fresh = W.distinct_five_tuples(64, 78, stream=W.STREAM_FRESH)
        vals = np.arange(64, dtype=np.uint64) + np.uint64(5)
        counts, first = srv.put_burst(insert_keys=to_dev(fresh), insert_values=vals_dev(vals))
        srv.wait(srv.submit(*counts), 10000)
        want = ref.insert_at(fresh, vals, np.full(64, now + 100, np.uint16), now)
        got = srv.get("insert", first[1], counts[1])
        torch.cuda.current_stream().synchronize()
        assert np.array_equal(u8(got), want)
        # let the loop leave, then step the time twice: the second step is
        # 16384 past the last scan, so it submits the scan's burst
        deadline = time.time() + 10
        while srv.status()["state"] != ckpp.SERVER_STOPPED and time.time() < deadline:
            time.sleep(0.01)
        assert srv.status()["state"] == ckpp.SERVER_STOPPED
        launches = srv.status()["launches"]
        assert srv.set_time(now + 9000)
        assert srv.status()["launches"] == launches  # no scan due yet: nothing submitted
        assert srv.set_time(now + 17000)
        ref.expire_scan(now + 17000)
        say("timed server: lookups after the relaunching scan")
        probe = np.concatenate([keys, fresh])
        counts, first = srv.put_burst(lookup_keys=to_dev(probe))
        srv.wait(srv.submit(*counts), 10000)
        f, v = srv.get("lookup", first[0], counts[0])
        torch.cuda.current_stream().synchronize()
        wf, wv = ref.lookup_at(probe, now + 17000, O.MODE_CUCKOOPP)
        assert np.array_equal(u8(f), wf) and np.array_equal(u64(v), wv)
        assert not wf.any()  # every entry had expired
        assert srv.status()["launches"] > launches
    # the loop's scan left only what the oracle's scans left: nothing
    assert t.stats()["live"] == ref.stats()["live"] == 0
    t.close()


def test_timed_server_insert_and_delete_of_one_key_in_a_round():
    """On a table with timers, a burst that inserts keys and deletes some of
    them: the deletes wait for the round's inserts, report found (the fresh
    entries are alive at the burst's time), and the keys end absent; stored
    keys deleted alongside report whether they were alive.  Results and the
    final dictionary equal the oracle's after the same bursts one by one."""
    import torch
    from paper_1712_09624_amd.ckpp import Server
    B, ttl, now = 10, 200, 3000
    ref, t, keys = timed_oracle_and_table(B, 0.5, now - 500, 31, False)
    fresh = W.distinct_five_tuples(2000, 32, stream=W.STREAM_FRESH)
    bursts = []
    for b in range(8):
        ins = fresh[250 * b: 250 * b + 60]
        dels = np.concatenate([ins[:20], keys[40 * b: 40 * b + 10]])  # own inserts + stored keys
        look = np.concatenate([keys[1000 + 30 * b: 1000 + 30 * b + 30],
                               fresh[250 * b + 200: 250 * b + 230]])
        ivals = np.arange(60, dtype=np.uint64) + np.uint64(10**9 * (b + 1))
        bursts.append((np.ascontiguousarray(look), np.ascontiguousarray(ins), ivals,
                       np.ascontiguousarray(dels)))
    e = (now + ttl) & 0xFFFF
    ref.expire_scan(now)
    want = []
    for look, ins, ivals, dels in bursts:
        f, v = ref.lookup_at(look, now, O.MODE_CUCKOOPP, refresh=e)
        st = ref.insert_at(ins, ivals, np.full(len(ins), e, np.uint16), now)
        df = ref.delete_at(dels, now)
        want.append((f.astype(np.uint8), v.astype(np.uint64), st.astype(np.uint8),
                     df.astype(np.uint8)))
    assert any(w[3][20:].any() for w in want) and not all(w[3][20:].all() for w in want)
    with Server(t, capacity=1 << 12, idle_ms=500, ttl=ttl, refresh=True) as srv:
        assert srv.set_time(now)
        say("timed server: bursts inserting and deleting the same keys, back to back")
        placed = [srv.put_burst(lookup_keys=to_dev(look), insert_keys=to_dev(ins),
                                insert_values=vals_dev(ivals), delete_keys=to_dev(dels))
                  for look, ins, ivals, dels in bursts]
        ids = [srv.submit(*c) for c, _ in placed]
        srv.wait(ids[-1], 10000)
        for i, ((c, first), w) in enumerate(zip(placed, want)):
            f, v = srv.get("lookup", first[0], c[0])
            st = srv.get("insert", first[1], c[1])
            df = srv.get("delete", first[2], c[2])
            torch.cuda.current_stream().synchronize()
            for g, x, name in zip((u8(f), u64(v), u8(st), u8(df)), w,
                                  ("lookup found", "lookup values", "insert status",
                                   "delete found")):
                assert np.array_equal(g, x), f"burst {i}: {name} differs"
    probe = np.concatenate([keys, fresh])
    wf, wv = ref.lookup_at(probe, now, O.MODE_CUCKOOPP)
    gf, gv = t.lookup_at(to_dev(probe), now)
    assert np.array_equal(u8(gf), wf) and np.array_equal(u64(gv), wv)
    bk, kv = t.export()
    rc, msg = O.check_image(bk, kv, B, W.HASH_SEED, False, timed=True)
    assert rc == 0, msg
    t.close()
