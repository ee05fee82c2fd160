"""The serving loop against the oracle, bit-exact: each burst's lookups see
the table as left by the bursts of earlier rounds, then its inserts and
deletes apply; every result is the same whether a burst runs alone or in a
mix with others (their writes concern other keys).

Tables are built by the oracle and imported; the oracle applies the same
bursts one by one (lookups, then inserts, then deletes of each burst)."""

import time

import numpy as np
import pytest

from gpu_util import say, to_dev, u64, u8, vals_dev
from oracle import oracle as O
from paper_1712_09624_amd import workload as W

pytestmark = pytest.mark.gpu


def oracle_and_table(B, load, seed, plain=False):
    from paper_1712_09624_amd.ckpp import Table
    n = W.keys_at_load(B, load)
    keys = W.distinct_five_tuples(n, seed)
    ref = O.OracleTable(B, W.HASH_SEED, W.MAX_KICKS, plain)
    assert (ref.insert(keys, W.insertion_values(n)) == O.INSERTED).all()
    t = Table(B, W.HASH_SEED, W.MAX_KICKS, plain=plain, device=0)
    b, k = ref.image()
    t.import_image(b, k)
    return ref, t, keys


def make_bursts(keys, nbursts, seed, max_lookup=400, max_insert=40, max_delete=20):
    """Bursts whose writes concern disjoint keys: inserts are fresh keys of
    their own burst, deletes take distinct stored keys that no burst looks
    up; lookups draw from the remaining stored keys and fresh keys."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = len(keys)
    perm = rng.permutation(n)
    ndel_total = min(n // 4, nbursts * max_delete)
    del_pool, look_pool = perm[:ndel_total], perm[ndel_total:]
    fresh = W.five_tuples(nbursts * (max_insert + max_lookup), seed, W.STREAM_FRESH)
    bursts, fi, di = [], 0, 0
    for b in range(nbursts):
        nl = int(rng.integers(1, max_lookup + 1))
        ni = int(rng.integers(0, max_insert + 1))
        nd = int(min(rng.integers(0, max_delete + 1), ndel_total - di))
        pos = keys[look_pool[rng.integers(0, len(look_pool), nl)]]
        neg = fresh[fi:fi + nl]
        fi += nl
        is_neg = rng.random(nl) < 0.5
        look = np.where(is_neg[:, None], neg, pos)
        ins = fresh[fi:fi + ni]
        fi += ni
        ivals = np.arange(ni, dtype=np.uint64) + np.uint64(10**12 + 10**6 * b)
        dels = keys[del_pool[di:di + nd]]
        di += nd
        bursts.append((np.ascontiguousarray(look), np.ascontiguousarray(ins), ivals,
                       np.ascontiguousarray(dels)))
    return bursts


def oracle_run(ref, bursts):
    out = []
    for look, ins, ivals, dels in bursts:
        f, v, _, _ = ref.lookup(look, O.MODE_BOTH if ref.plain else O.MODE_CUCKOOPP)
        st = ref.insert(ins, ivals) if len(ins) else np.zeros(0, np.uint8)
        df = ref.delete(dels) if len(dels) else np.zeros(0, np.uint8)
        out.append((f.astype(np.uint8), v.astype(np.uint64), st.astype(np.uint8),
                    df.astype(np.uint8)))
    return out


def put(srv, burst):
    import torch
    look, ins, ivals, dels = burst
    return srv.put_burst(
        lookup_keys=to_dev(look) if len(look) else None,
        insert_keys=to_dev(ins) if len(ins) else None,
        insert_values=vals_dev(ivals) if len(ins) else None,
        delete_keys=to_dev(dels) if len(dels) else None)


def fetch(srv, counts, first):
    import torch
    f, v = srv.get("lookup", first[0], counts[0])
    st = srv.get("insert", first[1], counts[1])
    df = srv.get("delete", first[2], counts[2])
    # this stream only: a device-wide synchronize would wait for the loop
    torch.cuda.current_stream().synchronize()
    return u8(f), u64(v), u8(st), u8(df)


def check(got, want, what):
    for g, w, name in zip(got, want, ("lookup found", "lookup values", "insert status",
                                      "delete found")):
        assert np.array_equal(g, w), f"{what}: {name} differs"


def test_server_bursts_match_oracle_alone_and_in_mix():
    from paper_1712_09624_amd.ckpp import Server
    ref_a, t_a, keys = oracle_and_table(12, 0.8, 5)
    ref_b, t_b, _ = oracle_and_table(12, 0.8, 5)
    bursts = make_bursts(keys, 24, 6)
    want = oracle_run(ref_a, bursts)
    # alone: one burst in flight at a time
    say("server alone: 24 bursts one by one")
    with Server(t_a, capacity=1 << 14, idle_ms=500) as srv:
        for i, b in enumerate(bursts):
            counts, first = put(srv, b)
            bid = srv.submit(*counts)
            srv.wait(bid, 10000)
            check(fetch(srv, counts, first), want[i], f"alone burst {i}")
        rounds_alone = srv.status()["rounds"]
    # mix: every burst put, then submitted back to back
    say("server mix: 24 bursts back to back")
    with Server(t_b, capacity=1 << 14, idle_ms=500) as srv:
        placed = [put(srv, b) for b in bursts]
        ids = [srv.submit(*c) for c, _ in placed]
        assert None not in ids
        srv.wait(ids[-1], 10000)
        for i, (c, f) in enumerate(placed):
            check(fetch(srv, c, f), want[i], f"mixed burst {i}")
        st = srv.status()
    assert st["completed"] == len(bursts) and st["submitted"] == len(bursts)
    assert st["rounds"] <= rounds_alone
    # both tables hold the dictionary the oracle holds after the bursts
    del ref_b
    for t, ref in ((t_a, ref_a), (t_b, ref_a)):
        bk, kv = t.export()
        rc, msg = O.check_image(bk, kv, 12, W.HASH_SEED, False)
        assert rc == 0, msg
        probe = np.concatenate([keys] + [b[1] for b in bursts])
        wf, wv, _, _ = ref.lookup(probe, O.MODE_CUCKOOPP)
        gf, gv = t.lookup(to_dev(probe))
        assert np.array_equal(u8(gf), wf) and np.array_equal(u64(gv), wv)
    t_a.close()
    t_b.close()


def test_server_ring_wrap_and_budget():
    from paper_1712_09624_amd.ckpp import Server
    ref, t, keys = oracle_and_table(10, 0.7, 8)
    bursts = make_bursts(keys, 40, 9, max_lookup=100, max_insert=10, max_delete=5)
    want = oracle_run(ref, bursts)
    say("server ring of 128 slots, budget 128")
    with Server(t, capacity=128, budget=128, idle_ms=500) as srv:
        # a burst larger than the budget is never admitted
        assert srv.submit(129, 0, 0) is None
        for i, b in enumerate(bursts):
            # the slots of a burst are reused by the next ones once the ring
            # wraps: its results are read before the next burst is put
            counts, first = put(srv, b)
            bid = srv.submit(*counts)
            assert bid is not None
            srv.wait(bid, 10000)
            check(fetch(srv, counts, first), want[i], f"burst {i}")
        assert srv.status()["lookup_tail"] > 4 * 128  # the ring wrapped
    t.close()


def test_server_idle_exit_and_relaunch():
    from paper_1712_09624_amd import ckpp
    ref, t, keys = oracle_and_table(9, 0.8, 11)
    bursts = make_bursts(keys, 2, 12)
    want = oracle_run(ref, bursts)
    say("server idle exit after 50 ms, relaunch on submit")
    with ckpp.Server(t, capacity=1 << 12, idle_ms=50) as srv:
        counts, first = put(srv, bursts[0])
        srv.wait(srv.submit(*counts), 10000)
        check(fetch(srv, counts, first), want[0], "before idle exit")
        deadline = time.time() + 10
        while srv.status()["state"] != ckpp.SERVER_STOPPED and time.time() < deadline:
            time.sleep(0.01)
        assert srv.status()["state"] == ckpp.SERVER_STOPPED
        counts, first = put(srv, bursts[1])
        srv.wait(srv.submit(*counts), 10000)
        check(fetch(srv, counts, first), want[1], "after relaunch")
        assert srv.status()["launches"] >= 2
    t.close()


@pytest.mark.parametrize("plain,mode", [(True, "cuckoopp"), (False, "optimistic"),
                                        (False, "both")])
def test_server_modes(plain, mode):
    from paper_1712_09624_amd.ckpp import Server
    ref, t, keys = oracle_and_table(11, 0.9, 13, plain=plain)
    bursts = make_bursts(keys, 6, 14)
    want = oracle_run(ref, bursts)  # every mode gives the dictionary's answers
    say(f"server plain={plain} mode={mode}")
    with Server(t, capacity=1 << 13, mode=mode, idle_ms=500) as srv:
        placed = [put(srv, b) for b in bursts]
        ids = [srv.submit(*c) for c, _ in placed]
        srv.wait(ids[-1], 10000)
        for i, (c, f) in enumerate(placed):
            check(fetch(srv, c, f), want[i], f"burst {i}")
    t.close()


def test_server_replay_open_loop():
    from paper_1712_09624_amd.ckpp import Server
    ref, t, keys = oracle_and_table(12, 0.85, 15)
    bursts = make_bursts(keys, 64, 16, max_lookup=300)
    want = oracle_run(ref, bursts)
    say("server replay of 64 bursts, 100 us apart")
    with Server(t, capacity=1 << 15, idle_ms=500) as srv:
        placed = [put(srv, b) for b in bursts]  # pre-staged in the rings
        arrival = np.arange(len(bursts)) * 1e-4
        counts = np.array([c for c, _ in placed], dtype=np.uint32)
        # replay submits the staged bursts itself
        adm, done = srv.replay(counts[:, 0], counts[:, 1], counts[:, 2], arrival, 30.0)
        assert (adm >= arrival - 1e-9).all() and (done >= adm).all()
        for i, (c, f) in enumerate(placed):
            check(fetch(srv, c, f), want[i], f"replayed burst {i}")
    t.close()


def test_server_many_small_bursts_past_the_tag_wrap():
    """40,000 small bursts, more than the 2^15 burst numbers the tags of the
    loop's latest-tails words tell apart, replayed 5 us apart so that rounds
    take one or a few bursts each: every lookup, insert status and delete
    result equals the oracle's, applied burst by burst."""
    import torch
    from paper_1712_09624_amd.ckpp import Server
    ref, t, keys = oracle_and_table(16, 0.5, 9)
    nb = 40000
    bursts = make_bursts(keys, nb, 10, max_lookup=3, max_insert=2, max_delete=1)
    want = oracle_run(ref, bursts)
    cat = [np.concatenate([b[k] for b in bursts]) for k in range(4)]
    counts = np.array([[len(b[0]), len(b[1]), len(b[3])] for b in bursts], dtype=np.uint32)
    say(f"server replay of {nb} small bursts, 5 us apart")
    with Server(t, capacity=1 << 17, idle_ms=2000) as srv:
        st0 = srv.status()
        pos = (st0["lookup_tail"], st0["insert_tail"], st0["delete_tail"])
        srv.put("lookup", pos[0], to_dev(cat[0]))
        srv.put("insert", pos[1], to_dev(cat[1]), vals_dev(cat[2]))
        srv.put("delete", pos[2], to_dev(cat[3]))
        arrival = np.arange(nb) * 5e-6
        srv.replay(counts[:, 0], counts[:, 1], counts[:, 2], arrival, 60.0)
        f, v = srv.get("lookup", pos[0], len(cat[0]))
        st = srv.get("insert", pos[1], len(cat[1]))
        df = srv.get("delete", pos[2], len(cat[3]))
        torch.cuda.current_stream().synchronize()
        status = srv.status()
    assert status["completed"] == nb and status["submitted"] == nb
    assert status["rounds"] < nb
    got = (u8(f), u64(v), u8(st), u8(df))
    for g, k, name in zip(got, range(4), ("lookup found", "lookup values", "insert status",
                                          "delete found")):
        w = np.concatenate([x[k] for x in want])
        assert np.array_equal(g, w), f"{name} differs"
    t.close()


def test_server_budget_of_2_24_reads_the_tail_records():
    """A server whose budget is 2^24 ops of a kind does not use the tagged
    tails block (its low bits could not tell such a round's tails): the
    leader reads each round's tails from the tail records.  Bursts alone and
    back to back equal the oracle."""
    from paper_1712_09624_amd.ckpp import Server
    ref_a, t_a, keys = oracle_and_table(12, 0.8, 41)
    ref_b, t_b, _ = oracle_and_table(12, 0.8, 41)
    bursts = make_bursts(keys, 16, 42)
    want = oracle_run(ref_a, bursts)
    del ref_b
    say("server with a 2^24 budget: 16 bursts one by one, then back to back")
    with Server(t_a, capacity=1 << 24, budget=1 << 24, idle_ms=500) as srv:
        for i, b in enumerate(bursts):
            counts, first = put(srv, b)
            bid = srv.submit(*counts)
            srv.wait(bid, 10000)
            check(fetch(srv, counts, first), want[i], f"alone burst {i}")
    with Server(t_b, capacity=1 << 24, budget=1 << 24, idle_ms=500) as srv:
        placed = [put(srv, b) for b in bursts]
        ids = [srv.submit(*c) for c, _ in placed]
        assert None not in ids
        srv.wait(ids[-1], 10000)
        for i, (c, f) in enumerate(placed):
            check(fetch(srv, c, f), want[i], f"mixed burst {i}")
    t_a.close()
    t_b.close()


def test_server_insert_and_delete_of_one_key_in_a_round():
    """A burst that inserts keys and deletes some of them: the deletes wait
    for the round's inserts (they are deferred past them), report found, and
    the keys end absent; bursts that write other keys run alongside.  The
    final table equals the oracle's after the same bursts one by one."""
    from paper_1712_09624_amd.ckpp import Server
    ref, t, keys = oracle_and_table(10, 0.5, 31)
    fresh = W.distinct_five_tuples(2000, 32, stream=W.STREAM_FRESH)
    bursts = []
    for b in range(8):
        ins = fresh[250 * b: 250 * b + 60]
        dels = np.concatenate([ins[:20], keys[40 * b: 40 * b + 10]])  # own inserts + stored keys
        look = np.concatenate([keys[1000 + 30 * b: 1000 + 30 * b + 30], fresh[250 * b + 200:
                                                                             250 * b + 230]])
        ivals = np.arange(60, dtype=np.uint64) + np.uint64(10**9 * (b + 1))
        bursts.append((np.ascontiguousarray(look), np.ascontiguousarray(ins), ivals,
                       np.ascontiguousarray(dels)))
    want = oracle_run(ref, bursts)
    with Server(t, capacity=1 << 12, idle_ms=500) as srv:
        say("server: one burst inserting and deleting the same keys")
        counts, first = put(srv, bursts[0])
        srv.wait(srv.submit(*counts), 10000)
        check(fetch(srv, counts, first), want[0], "burst 0")
        assert srv.status()["delete_ns"] > 0, "the deletes of the burst's own keys were deferred"
        say("server: seven such bursts back to back")
        placed = [put(srv, b) for b in bursts[1:]]
        ids = [srv.submit(*c) for c, _ in placed]
        srv.wait(ids[-1], 10000)
        for i, (c, f) in enumerate(placed):
            check(fetch(srv, c, f), want[i + 1], f"burst {i + 1}")
    bk, kv = t.export()
    rc, msg = O.check_image(bk, kv, 10, W.HASH_SEED, False)
    assert rc == 0, msg
    probe = np.concatenate([keys, fresh])
    wf, wv, _, _ = ref.lookup(probe, O.MODE_CUCKOOPP)
    gf, gv = t.lookup(to_dev(probe))
    assert np.array_equal(u8(gf), wf) and np.array_equal(u64(gv), wv)
    t.close()


def test_server_on_a_table_above_2_24_buckets():
    """A server on a 2^25-bucket table (8 GiB; the alternate bucket and the
    filter bits come from a second hash word), checked against the ground
    truth, which holds at any size: stored keys are found with their values,
    fresh keys are not, inserts of fresh keys report INSERTED and are found
    by later bursts, deletes of stored keys report found and the keys are
    gone afterwards."""
    import torch
    from paper_1712_09624_amd.ckpp import Server, Table
    B = 25
    n = W.keys_at_load(B, 0.05)
    keys = W.distinct_five_tuples(n, 61, check=False)
    vals = W.insertion_values(n)
    t = Table(B, W.HASH_SEED, W.MAX_KICKS, device=0)
    say(f"server on 2^{B} buckets: building {n} keys")
    for s in range(0, n, 1 << 22):
        st, nf = t.insert(to_dev(keys[s:s + (1 << 22)]), vals_dev(vals[s:s + (1 << 22)]))
        torch.cuda.synchronize()
        assert int(nf.item()) == 0
    rng = np.random.default_rng(62)
    fresh = W.distinct_five_tuples(4096, 63, stream=W.STREAM_FRESH)
    with Server(t, capacity=1 << 14, idle_ms=500) as srv:
        # burst 1: lookups of stored and fresh keys, inserts of fresh keys,
        # deletes of stored keys that no lookup of the burst reads
        rows = rng.choice(n, size=3000, replace=False)
        look = np.concatenate([keys[rows[:2000]], fresh[2048:3048]])
        dels = keys[rows[2000:2500]]
        ins = fresh[:2048]
        ivals = np.arange(2048, dtype=np.uint64) + np.uint64(7 << 40)
        counts, first = srv.put_burst(lookup_keys=to_dev(look), insert_keys=to_dev(ins),
                                      insert_values=vals_dev(ivals), delete_keys=to_dev(dels))
        srv.wait(srv.submit(*counts), 10000)
        f, v = srv.get("lookup", first[0], counts[0])
        st = srv.get("insert", first[1], counts[1])
        df = srv.get("delete", first[2], counts[2])
        torch.cuda.current_stream().synchronize()
        f, v, st, df = u8(f), u64(v), u8(st), u8(df)
        assert f[:2000].all() and np.array_equal(v[:2000], vals[rows[:2000]])
        assert not f[2000:].any()
        assert (st == O.INSERTED).all() and df.all()
        # burst 2: the inserted keys are found, the deleted ones are gone
        look2 = np.concatenate([ins, dels])
        counts, first = srv.put_burst(lookup_keys=to_dev(look2))
        srv.wait(srv.submit(*counts), 10000)
        f, v = srv.get("lookup", first[0], counts[0])
        torch.cuda.current_stream().synchronize()
        f, v = u8(f), u64(v)
        assert f[:2048].all() and np.array_equal(v[:2048], ivals)
        assert not f[2048:].any()
    s = t.stats()
    assert s["live"] == n + 2048 - 500 and s["locked"] == 0
    t.close()
