"""GPU inserts and deletes against the oracle.

Insert layouts are not unique (which slot, which keys are displaced), so a
GPU-built table is compared by what is unique: the dictionary it holds (the
found flag and value of every key, live, deleted or never inserted, compared
with the oracle that ran the same batches) and the image invariants (every
entry in one of its two buckets with its tag and other bucket, exact moved
counters, no filter false negative, reset filters, free locks)."""

import numpy as np
import pytest

from gpu_util import check_gpu_image, say, to_dev, u64, u8, vals_dev
from oracle import oracle as O
from paper_1712_09624_amd import workload as W

pytestmark = pytest.mark.gpu


def new_table(B, plain=False, max_kicks=W.MAX_KICKS):
    from paper_1712_09624_amd.ckpp import Table
    return Table(B, W.HASH_SEED, max_kicks, plain=plain, device=0)


def insert_batches(t, keys, vals, batch):
    import torch
    st_all = []
    nfail = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    for s in range(0, len(keys), batch):
        st, _ = t.insert(to_dev(keys[s:s + batch]), vals_dev(vals[s:s + batch]), nfailed=nfail)
        st_all.append(st)
    torch.cuda.synchronize()
    st = np.concatenate([u8(x) for x in st_all]) if st_all else np.zeros(0, np.uint8)
    return st, int(nfail.item())


def compare_dictionary(t, ref, probe, modes=("cuckoopp", "both", "optimistic")):
    omodes = {"cuckoopp": O.MODE_CUCKOOPP, "both": O.MODE_BOTH, "optimistic": O.MODE_OPTIMISTIC}
    for m in modes:
        want_f, want_v, _, _ = ref.lookup(probe, omodes[m])
        f, v = t.lookup(to_dev(probe), m)
        assert np.array_equal(u8(f), want_f), f"found flags differ ({m})"
        assert np.array_equal(u64(v), want_v), f"values differ ({m})"


@pytest.mark.parametrize("plain", [False, True], ids=["cuckoopp", "plain"])
def test_cfg1_insert(plain):
    """2^14 buckets filled to load 0.8 in batches of 65536 (last one ragged)."""
    B = 14
    n = W.keys_at_load(B, 0.8)
    keys = W.distinct_five_tuples(n, 1)
    vals = W.insertion_values(n)
    ref = O.OracleTable(B, W.HASH_SEED, W.MAX_KICKS, plain)
    assert (ref.insert(keys, vals) == O.INSERTED).all()
    say(f"cfg1 insert plain={plain} n={n}")
    t = new_table(B, plain)
    st, nfail = insert_batches(t, keys, vals, 65536)
    assert (st == O.INSERTED).all() and nfail == 0
    check_gpu_image(t, B, plain)
    s = t.stats()
    assert s["live"] == n and s["locked"] == 0 and s["retry_exhausted"] == 0
    probe = np.concatenate([keys, W.five_tuples(n, 2, stream=W.STREAM_NEGATIVE)])
    compare_dictionary(t, ref, probe)
    t.close()


def test_update_existing_keys():
    B = 12
    n = W.keys_at_load(B, 0.9)
    keys = W.distinct_five_tuples(n, 3)
    vals = W.insertion_values(n)
    ref = O.OracleTable(B, W.HASH_SEED, W.MAX_KICKS)
    ref.insert(keys, vals)
    t = new_table(B)
    say("update: first insert")
    insert_batches(t, keys, vals, 1 << 20)
    # half of the keys again (new values) plus fresh keys up to load 0.95
    rows = W.choose_rows(n, n // 2, 4)
    fresh = W.distinct_five_tuples(W.keys_at_load(B, 0.95) - n, 5, stream=W.STREAM_FRESH)
    k2 = np.concatenate([keys[rows], fresh])
    v2 = W.insertion_values(len(k2), 10**9)
    want = ref.insert(k2, v2)
    assert (want[: len(rows)] == O.UPDATED).all()
    say("update: second insert")
    st, nfail = insert_batches(t, k2, v2, 1 << 20)
    assert np.array_equal(st, want) and nfail == int((want == O.FAILED).sum())
    check_gpu_image(t, B)
    compare_dictionary(t, ref, np.concatenate([keys, fresh]))
    t.close()


@pytest.mark.parametrize("B", [10, 14, 16])
def test_delete_and_reinsert(B):
    """The batched build of the insert workload at small size: fill to load
    0.95 in batches, delete a random 20%, re-insert as many fresh keys; every
    live, deleted and fresh key answers as in the oracle."""
    n = W.keys_at_load(B, 0.95)
    keys = W.distinct_five_tuples(n, 6)
    vals = W.insertion_values(n)
    ref = O.OracleTable(B, W.HASH_SEED, W.MAX_KICKS)
    assert (ref.insert(keys, vals) == O.INSERTED).all()
    t = new_table(B)
    say(f"delete/reinsert B={B}: build")
    st, nfail = insert_batches(t, keys, vals, 4096)
    assert (st == O.INSERTED).all() and nfail == 0
    check_gpu_image(t, B)
    nd = n // 5
    rows = W.choose_rows(n, nd, 7)
    want_d = ref.delete(keys[rows])
    assert want_d.all()
    say(f"delete/reinsert B={B}: delete {nd}")
    d = u8(t.delete(to_dev(keys[rows])))
    assert np.array_equal(d, want_d)
    check_gpu_image(t, B)
    say(f"delete/reinsert B={B}: delete again (all absent)")
    assert not u8(t.delete(to_dev(keys[rows]))).any()
    fresh = W.distinct_five_tuples(nd, 8, stream=W.STREAM_FRESH)
    fv = W.insertion_values(nd, n)
    want_s = ref.insert(fresh, fv)
    say(f"delete/reinsert B={B}: re-insert {nd}")
    st, nfail = insert_batches(t, fresh, fv, 4096)
    assert np.array_equal(st, want_s)
    img_b, _ = check_gpu_image(t, B)
    assert t.stats()["live"] == ref.live
    compare_dictionary(t, ref, np.concatenate([keys, fresh, W.five_tuples(n, 9)]))
    t.close()


def test_two_bucket_capacity():
    """2 buckets: 16 keys fit, the 17th fails and the table is unchanged."""
    keys = W.distinct_five_tuples(17, 5)
    t = new_table(1)
    say("B=1: 16 keys")
    st, nfail = insert_batches(t, keys[:16], W.insertion_values(16), 16)
    assert (st == O.INSERTED).all() and nfail == 0
    b0, k0 = t.export()
    say("B=1: 17th key")
    st, nfail = insert_batches(t, keys[16:], W.insertion_values(1, 16), 1)
    assert st[0] == O.FAILED and nfail == 1
    b1, k1 = t.export()
    assert np.array_equal(b0, b1) and np.array_equal(k0, k1)
    f, v = t.lookup(to_dev(keys))
    assert list(u8(f)) == [1] * 16 + [0]
    assert list(u64(v)) == list(range(16)) + [0]
    t.close()


@pytest.mark.parametrize("B", [1, 2, 3, 4, 6, 8])
@pytest.mark.parametrize("over", [0.9, 1.3])
def test_contention_overfill(B, over):
    """Many lanes insert into a tiny table at once (up to 130% of its slots):
    each key is INSERTED or FAILED, the table holds exactly the INSERTED keys
    with their values, the invariants hold, and no lane gave up on a lock."""
    cap = 8 << B
    n = max(2, int(over * cap))
    keys = W.distinct_five_tuples(n, 100 + B)
    vals = W.insertion_values(n, 7)
    t = new_table(B)
    say(f"contention B={B} n={n}")
    st, nfail = insert_batches(t, keys, vals, n)
    assert set(np.unique(st)) <= {O.INSERTED, O.FAILED}
    ins = st == O.INSERTED
    assert nfail == int((~ins).sum())
    if over < 1.0 and B >= 3:
        assert ins.all(), f"failures below capacity: {int((~ins).sum())}"
    check_gpu_image(t, B)
    s = t.stats()
    assert s["live"] == int(ins.sum()) and s["retry_exhausted"] == 0
    f, v = t.lookup(to_dev(keys))
    assert np.array_equal(u8(f), ins.astype(np.uint8))
    assert np.array_equal(u64(v), np.where(ins, vals, 0).astype(np.uint64))
    # delete everything in one batch: all filters reset
    say(f"contention B={B}: delete all")
    d = u8(t.delete(to_dev(keys)))
    assert np.array_equal(d, ins.astype(np.uint8))
    s = t.stats()
    assert s["live"] == 0 and s["bloom_pc_sum"] == 0 and s["moved_hist"][0] == 1 << B
    check_gpu_image(t, B)
    t.close()


def test_retry_limit_per_key_outcome():
    """The per-key outcome of giving up on contended locks.  Sixteen keys of
    a 2-bucket table all need the same two bucket locks; with a retry limit
    of one attempt, the lanes that find a lock held report CKPP_RETRY: those
    keys are absent afterwards (nothing stored, not counted as FAILED), the
    others are INSERTED with their values, and the table keeps its
    invariants.  A delete batch under the same limit reports RETRY for the
    keys it did not remove, which are still found.  Locks are never waited
    on, so every kernel ends; at the default limit the retried keys then
    succeed."""
    import torch
    from paper_1712_09624_amd.ckpp import MAX_RETRY_LIMIT, RETRY
    keys = W.distinct_five_tuples(16, 140)
    vals = W.insertion_values(16, 50)
    t = new_table(1)
    assert t.retry_limit() == MAX_RETRY_LIMIT
    t.set_retry_limit(1)
    assert t.retry_limit() == 1
    say("retry limit 1: contended insert of 16 keys into 2 buckets")
    st, nfail = insert_batches(t, keys, vals, 16)
    assert set(np.unique(st)) <= {O.INSERTED, RETRY}
    ins = st == O.INSERTED
    assert ins.any() and (~ins).any(), f"statuses {st}"
    assert nfail == 0
    assert t.stats()["retry_exhausted"] == int((~ins).sum())
    f, v = t.lookup(to_dev(keys))
    assert np.array_equal(u8(f), ins.astype(np.uint8))
    assert np.array_equal(u64(v), np.where(ins, vals, 0).astype(np.uint64))
    check_gpu_image(t, 1)
    say("default limit: the retried keys")
    t.set_retry_limit(MAX_RETRY_LIMIT)
    st2, _ = insert_batches(t, keys[~ins], vals[~ins], 16)
    assert (st2 == O.INSERTED).all()
    t.set_retry_limit(1)
    say("retry limit 1: contended delete of the 16 keys")
    d = u8(t.delete(to_dev(keys)))
    torch.cuda.synchronize()
    assert set(np.unique(d)) <= {0, 1, RETRY}
    removed = d == 1
    assert removed.any() and (d == RETRY).any() and not (d == 0).any(), f"outcomes {d}"
    f, v = t.lookup(to_dev(keys))
    assert np.array_equal(u8(f), (~removed).astype(np.uint8))
    check_gpu_image(t, 1)
    t.set_retry_limit(MAX_RETRY_LIMIT)
    d2 = u8(t.delete(to_dev(keys)))
    assert np.array_equal(d2, (~removed).astype(np.uint8))
    assert t.stats()["live"] == 0
    t.close()


def test_duplicate_deletes_in_one_batch():
    B = 8
    n = W.keys_at_load(B, 0.9)
    keys = W.distinct_five_tuples(n, 120)
    t = new_table(B)
    insert_batches(t, keys, W.insertion_values(n), n)
    dup = np.concatenate([keys[:100], keys[:100]])
    say("duplicate deletes")
    d = u8(t.delete(to_dev(dup)))
    assert (d[:100] + d[100:] == 1).all()
    check_gpu_image(t, B)
    t.close()


def test_zero_kicks():
    """max_kicks 0: a key fails as soon as both of its buckets are full."""
    keys = W.distinct_five_tuples(17, 5)
    t = new_table(1, max_kicks=0)
    st, _ = insert_batches(t, keys[:16], W.insertion_values(16), 16)
    assert (st == O.INSERTED).all()
    st, _ = insert_batches(t, keys[16:], W.insertion_values(1), 1)
    assert st[0] == O.FAILED
    t.close()


def test_clear():
    B = 8
    keys = W.distinct_five_tuples(500, 130)
    t = new_table(B)
    insert_batches(t, keys, W.insertion_values(500), 500)
    t.clear()
    s = t.stats()
    assert s["live"] == 0
    f, _ = t.lookup(to_dev(keys))
    assert not u8(f).any()
    t.close()


@pytest.mark.parametrize("B,timed", [(6, False), (9, False), (7, True), (9, True)])
def test_churn_near_capacity(B, timed):
    """Forty batches alternate fresh inserts that bring the table to load
    0.97 (many keys need cuckoo paths, many lanes contend for the same
    buckets) with deletes of a random third of the stored keys and of some
    absent keys.  After every batch the table holds exactly what the
    statuses say (INSERTED kept, FAILED absent) with its values, every
    delete reports presence, the invariants hold and no lane gave up on a
    lock.  With timers the clock advances 60 units a batch and expiration
    times are up to 1023 units ahead, so entries expire, are reused lazily
    and are removed by a scan every ten batches."""
    import torch
    from paper_1712_09624_amd.ckpp import Table
    rng = np.random.default_rng(B + (100 if timed else 0))
    cap = 8 << B
    universe = W.distinct_five_tuples(24 * cap, 300 + B)
    t = Table(B, W.HASH_SEED, W.MAX_KICKS, device=0, timers=timed)
    live = {}  # row -> (value, expiry)
    nxt, now = 0, 65000

    def alive(row):
        return row in live and (not timed or ((live[row][1] - now) & 0xFFFF) < 1024)

    for r in range(40):
        if timed:
            now = (now + 60) & 0xFFFF
            for row in [x for x in live if not alive(x)]:
                del live[row]
            if r % 10 == 9:
                t.expire_scan(now)
        want = int(0.97 * cap) - len(live)
        if want > 0:
            rows = np.arange(nxt, nxt + want)
            nxt += want
            vals = rng.integers(0, 1 << 40, size=want).astype(np.uint64)
            exp = ((now + rng.integers(0, 1024, size=want)) & 0xFFFF).astype(np.uint16)
            say(f"churn B={B} timed={timed} round={r} insert {want}")
            if timed:
                st, nf = t.insert_at(to_dev(universe[rows]), vals_dev(vals),
                                     to_dev(exp.view(np.int16)), now)
            else:
                st, nf = t.insert(to_dev(universe[rows]), vals_dev(vals))
            torch.cuda.synchronize()
            st = u8(st)
            assert set(np.unique(st)) <= {O.INSERTED, O.FAILED}
            assert int(nf.item()) == int((st == O.FAILED).sum())
            for i in np.flatnonzero(st == O.INSERTED):
                live[int(rows[i])] = (int(vals[i]), int(exp[i]))
        stored = np.array(sorted(live), dtype=np.int64)
        drop = rng.choice(stored, size=len(stored) // 3, replace=False) if len(stored) else stored
        absent = rng.integers(nxt, len(universe), size=50)
        drows = np.concatenate([drop, absent])
        say(f"churn B={B} timed={timed} round={r} delete {len(drows)}")
        d = u8(t.delete_at(to_dev(universe[drows]), now) if timed
               else t.delete(to_dev(universe[drows])))
        assert np.array_equal(d, np.array([alive(int(x)) for x in drows], np.uint8))
        for x in drop:
            live.pop(int(x), None)
        probe = universe[:nxt]
        f, v = t.lookup_at(to_dev(probe), now) if timed else t.lookup(to_dev(probe))
        wf = np.array([alive(i) for i in range(nxt)], np.uint8)
        wv = np.array([live[i][0] if alive(i) else 0 for i in range(nxt)], np.uint64)
        assert np.array_equal(u8(f), wf), f"round {r}: found flags"
        assert np.array_equal(u64(v), wv), f"round {r}: values"
        b, k = t.export()
        rc, msg = O.check_image(b, k, B, W.HASH_SEED, timed=timed)
        assert rc == 0, f"round {r}: invariant {rc}: {msg}"
    s = t.stats()
    assert s["locked"] == 0 and s["retry_exhausted"] == 0
    t.close()
