"""GPU tables with timers (Sec. 4.2) against the oracle.

Lookups and the anti-revival scan on oracle-built images are bit-exact with
the oracle: the found flag and value of every key, and, after a refreshing
lookup or a scan, the whole table image byte for byte.  GPU-built timed
tables (inserts, refreshing lookups, deletes and scans while the 16-bit
clock advances and wraps) are compared by what is unique: every key's found
flag and value, every insert's status, and the image invariants."""

import numpy as np
import pytest

from gpu_util import say, to_dev, u64, u8, vals_dev
from oracle import oracle as O
from paper_1712_09624_amd import workload as W

pytestmark = pytest.mark.gpu

MODES = [("cuckoopp", O.MODE_CUCKOOPP), ("both", O.MODE_BOTH), ("optimistic", O.MODE_OPTIMISTIC)]


def alive(expiry, now):
    return ((np.asarray(expiry, np.int64) - int(now)) & 0xFFFF) < O.MAX_DELAY


def new_timed(B, plain=False):
    from paper_1712_09624_amd.ckpp import Table
    return Table(B, W.HASH_SEED, W.MAX_KICKS, plain=plain, device=0, timers=True)


def exp_dev(e):
    return to_dev(np.ascontiguousarray(e, dtype=np.uint16).view(np.int16))


def gpu_from(ref):
    t = new_timed(ref.log2_buckets, ref.plain)
    b, k = ref.image()
    t.import_image(b, k)
    return t


def check_timed_image(t, B, plain=False):
    b, k = t.export()
    rc, msg = O.check_image(b, k, B, W.HASH_SEED, plain, timed=True)
    assert rc == 0, f"GPU image invariant {rc}: {msg}"
    return b, k


@pytest.fixture(scope="module")
def timed_cfg1():
    """2^14 buckets at load 0.8 with timers: expiration times uniform over
    the 1024 units after now0 = 65000 (so the window wraps), 2^20 lookups
    with half of them fresh keys."""
    B, now0 = 14, 65000
    n = W.keys_at_load(B, 0.8)
    keys = W.distinct_five_tuples(n, 1)
    vals = W.insertion_values(n)
    exp = W.times_after(n, now0, 1024, 1)
    ref = O.OracleTable(B, W.HASH_SEED, W.MAX_KICKS, timed=True)
    assert (ref.insert_at(keys, vals, exp, now0) == O.INSERTED).all()
    look, _, _ = W.lookup_mix(keys, 1 << 20, 0.5, 1)
    return B, now0, ref, keys, exp, look


@pytest.mark.parametrize("mode,omode", MODES, ids=[m[0] for m in MODES])
def test_timed_lookup_bit_exact(timed_cfg1, mode, omode):
    B, now0, ref, keys, exp, look = timed_cfg1
    t = gpu_from(ref)
    for dt in (0, 300, 700, 1023, 1024, 64512, 64513):
        now = (now0 + dt) & 0xFFFF
        want_f, want_v = ref.lookup_at(look, now, omode)
        say(f"timed lookup mode={mode} now={now}")
        f, v = t.lookup_at(to_dev(look), now, mode)
        assert np.array_equal(u8(f), want_f), f"found flags differ at now={now}"
        assert np.array_equal(u64(v), want_v), f"values differ at now={now}"
    # some entries alive and some expired at now0 + 500
    f, _ = ref.lookup_at(keys, (now0 + 500) & 0xFFFF)
    assert 0 < int(f.sum()) < len(keys)
    t.close()


@pytest.mark.parametrize("shape", [(8, 1, 64, 0), (8, 1, 256, 3), (8, 2, 64, 1), (8, 2, 256, 0),
                                   (4, 1, 64, 0), (4, 1, 256, 3), (4, 2, 128, 0),
                                   (1, 1, 64, 0), (1, 2, 128, 3), (1, 4, 256, 0)])
def test_timed_lookup_launch_shapes(timed_cfg1, shape):
    B, now0, ref, keys, exp, look = timed_cfg1
    now = (now0 + 400) & 0xFFFF
    want_f, want_v = ref.lookup_at(look[:100003], now)
    t = gpu_from(ref)
    t.set_lookup_launch(*shape)
    say(f"timed lookup shape={shape}")
    f, v = t.lookup_at(to_dev(look[:100003]), now)
    assert np.array_equal(u8(f), want_f) and np.array_equal(u64(v), want_v)
    t.close()


@pytest.mark.parametrize("mode,omode", MODES, ids=[m[0] for m in MODES])
def test_refreshing_lookup_image_bit_exact(timed_cfg1, mode, omode):
    """A refreshing lookup writes the new expiration time of every entry it
    finds and nothing else: the GPU image equals the oracle's byte for
    byte afterwards."""
    B, now0, _, keys, exp, look = timed_cfg1
    ref = O.OracleTable(B, W.HASH_SEED, W.MAX_KICKS, timed=True)
    assert (ref.insert_at(keys, W.insertion_values(len(keys)), exp, now0) == O.INSERTED).all()
    t = gpu_from(ref)
    now = (now0 + 500) & 0xFFFF
    new_exp = (now + 1000) & 0xFFFF
    want_f, want_v = ref.lookup_at(look, now, omode, refresh=new_exp)
    say(f"refreshing lookup mode={mode}")
    f, v = t.lookup_at(to_dev(look), now, mode, refresh=new_exp)
    assert np.array_equal(u8(f), want_f) and np.array_equal(u64(v), want_v)
    gb, gk = t.export()
    rb, rk = ref.image()
    assert np.array_equal(gb, rb), "bucket arrays differ after refresh"
    assert np.array_equal(gk, rk), "key/value arrays differ after refresh"
    # refreshed entries are alive until new_exp, the others expire
    f2, _ = t.lookup_at(to_dev(keys), (now + 999) & 0xFFFF)
    wf2, _ = ref.lookup_at(keys, (now + 999) & 0xFFFF)
    assert np.array_equal(u8(f2), wf2) and int(wf2.sum()) > 0
    t.close()


@pytest.mark.parametrize("shape", [(1, 1, 64, 0), (1, 4, 256, 0), (4, 1, 128, 0), (4, 2, 64, 0), (8, 1, 256, 0)])
def test_refreshing_lookup_shapes(timed_cfg1, shape):
    """Refreshing lookups of the other kernels (one lane per lookup with
    bucket heads in registers, one lookup per lane with lines in LDS) leave
    the same image as the oracle."""
    B, now0, _, keys, exp, look = timed_cfg1
    ref = O.OracleTable(B, W.HASH_SEED, W.MAX_KICKS, timed=True)
    assert (ref.insert_at(keys, W.insertion_values(len(keys)), exp, now0) == O.INSERTED).all()
    t = gpu_from(ref)
    t.set_lookup_launch(*shape)
    now = (now0 + 300) & 0xFFFF
    new_exp = (now + 700) & 0xFFFF
    want_f, want_v = ref.lookup_at(look, now, O.MODE_CUCKOOPP, refresh=new_exp)
    say(f"refreshing lookup shape={shape}")
    f, v = t.lookup_at(to_dev(look), now, "cuckoopp", refresh=new_exp)
    assert np.array_equal(u8(f), want_f) and np.array_equal(u64(v), want_v)
    gb, gk = t.export()
    rb, rk = ref.image()
    assert np.array_equal(gb, rb) and np.array_equal(gk, rk), "images differ after refresh"
    t.close()


@pytest.mark.parametrize("plain", [False, True], ids=["cuckoopp", "plain"])
def test_expire_scan_image_bit_exact(plain):
    """The scan on an image at load 0.95 (many displaced entries) removes
    exactly the oracle's entries with the same counter and filter updates."""
    B, now0 = 12, 100
    n = W.keys_at_load(B, 0.95)
    keys = W.distinct_five_tuples(n, 61)
    exp = W.times_after(n, now0, 1024, 61)
    ref = O.OracleTable(B, W.HASH_SEED, W.MAX_KICKS, plain, timed=True)
    assert (ref.insert_at(keys, W.insertion_values(n), exp, now0) == O.INSERTED).all()
    assert plain or ref.stats()["in_secondary"] > 0
    t = gpu_from(ref)
    now = now0 + 600
    removed_want = ref.expire_scan(now)
    say(f"expire scan plain={plain}")
    removed = t.expire_scan(now)
    assert int(removed.item()) == removed_want > 0
    gb, gk = t.export()
    rb, rk = ref.image()
    assert np.array_equal(gb, rb), "bucket arrays differ after the scan"
    assert np.array_equal(gk, rk), "key/value arrays differ after the scan"
    check_timed_image(t, B, plain)
    st = t.stats()
    assert st["live"] == int(alive(exp, now).sum())
    t.close()


def test_lazy_reuse_two_buckets():
    """Two buckets, 16 entries expiring at 110: at 111, 16 fresh keys take
    the expired slots (no failure, the table still holds 16), the 17th
    fails, the old keys are gone and the counters are exact."""
    import torch
    keys = W.distinct_five_tuples(33, 41, check=True)
    t = new_timed(1)
    say("lazy reuse: fill")
    st, _ = t.insert_at(to_dev(keys[:16]), vals_dev(W.insertion_values(16)),
                        exp_dev(np.full(16, 110)), 100)
    assert (u8(st) == O.INSERTED).all()
    st, _ = t.insert_at(to_dev(keys[16:17]), vals_dev(W.insertion_values(1)),
                        exp_dev(np.full(1, 110)), 100)
    assert u8(st)[0] == O.FAILED
    say("lazy reuse: 16 fresh keys at 111")
    st, nf = t.insert_at(to_dev(keys[17:33]), vals_dev(W.insertion_values(16, 100)),
                         exp_dev(np.full(16, 200)), 111)
    torch.cuda.synchronize()
    assert (u8(st) == O.INSERTED).all() and int(nf.item()) == 0
    assert t.stats()["live"] == 16
    f, v = t.lookup_at(to_dev(keys), 111)
    f, v = u8(f), u64(v)
    assert not f[:17].any() and f[17:].all()
    assert np.array_equal(v[17:], W.insertion_values(16, 100))
    check_timed_image(t, 1)
    t.close()


@pytest.mark.parametrize("B,plain", [(4, False), (10, False), (8, True)])
def test_timed_dictionary_vs_oracle(B, plain):
    """Random batches of inserts, refreshing lookups and deletes while the
    clock advances and wraps, with a scan at least every 30000 units, on the
    GPU and on the oracle: every insert status and every key's answer agree
    after each round; the GPU image keeps its invariants.  The universe is
    85% of the slots, so no insert fails for lack of room and the statuses
    are unique.  Some insert values are 2^48 or more: the GPU's device
    layout refuses them (a documented precondition of its tables with
    timers: status FAILED, nothing changes for that key), which the test
    models by giving the oracle only the other keys of the batch."""
    import torch
    rng = np.random.default_rng(B)
    cap = 8 << B
    universe = W.distinct_five_tuples(int(0.85 * cap), 70 + B)
    ref = O.OracleTable(B, W.HASH_SEED, W.MAX_KICKS, plain, timed=True)
    t = new_timed(B, plain)
    now = 65300
    since_scan = 0
    for r in range(24):
        op = rng.choice(["ins", "ins", "del", "look", "tick"])
        k = int(rng.integers(1, max(2, len(universe) // 3)))
        rows = rng.choice(len(universe), size=k, replace=False)
        keys = universe[rows]
        say(f"timed dict B={B} plain={plain} round={r} op={op} n={k} now={now}")
        if op == "tick":
            step = int(rng.choice([int(rng.integers(1, 64)), int(rng.integers(200, 3000))]))
            if since_scan + step > 30000:
                want = ref.expire_scan(now)
                got = t.expire_scan(now)
                assert int(got.item()) == want
                since_scan = 0
            now = (now + step) & 0xFFFF
            since_scan += step
        elif op == "ins":
            vals = rng.integers(0, 1 << 48, size=k, dtype=np.int64).astype(np.uint64)
            wide = rng.random(k) < 0.03
            vals[wide] |= np.uint64(1 << 62)
            exp = ((now + rng.integers(0, 1024, size=k)) & 0xFFFF).astype(np.uint16)
            want = np.full(k, O.FAILED, np.uint8)
            if (~wide).any():
                want[~wide] = ref.insert_at(keys[~wide], vals[~wide], exp[~wide], now)
            st, nf = t.insert_at(to_dev(keys), vals_dev(vals), exp_dev(exp), now)
            torch.cuda.synchronize()
            assert np.array_equal(u8(st), want), "insert statuses differ"
            assert int(nf.item()) == int((want == O.FAILED).sum())
        elif op == "del":
            want = ref.delete_at(keys, now)
            got = t.delete_at(to_dev(keys), now)
            assert np.array_equal(u8(got), want), "delete results differ"
        else:
            e = (now + int(rng.integers(0, 1024))) & 0xFFFF
            mode, omode = MODES[r % 3]
            wf, wv = ref.lookup_at(keys, now, omode, refresh=e)
            f, v = t.lookup_at(to_dev(keys), now, mode, refresh=e)
            assert np.array_equal(u8(f), wf) and np.array_equal(u64(v), wv)
        for mode, omode in MODES:
            wf, wv = ref.lookup_at(universe, now, omode)
            f, v = t.lookup_at(to_dev(universe), now, mode)
            assert np.array_equal(u8(f), wf), f"round {r} {mode}: found differs"
            assert np.array_equal(u64(v), wv), f"round {r} {mode}: values differ"
        check_timed_image(t, B, plain)
    st = t.stats()
    assert st["locked"] == 0 and st["retry_exhausted"] == 0
    t.close()


@pytest.mark.parametrize("B", [3, 9])
def test_wide_values_device_limit(B):
    """The device-layout limit of tables with timers, as include/ckpp.h states
    it: an insert of a value of 2^48 or more stores nothing and reports
    FAILED for that key (counted in nfailed) -- an absent key stays absent,
    a present key keeps its old value and time -- while the other keys of
    the batch are inserted or updated as usual; and ckpp_import refuses an
    image (built by the oracle, whose dictionary takes 64-bit values) with
    such a value in an occupied slot, leaving the table unchanged."""
    import torch
    rng = np.random.default_rng(40 + B)
    now = 700
    n = int(0.5 * (8 << B))
    keys = W.distinct_five_tuples(n, 90 + B)
    vals = rng.integers(0, 1 << 48, size=n, dtype=np.int64).astype(np.uint64)
    exp = ((now + rng.integers(0, 1024, size=n)) & 0xFFFF).astype(np.uint16)
    t = new_timed(B)
    say(f"wide values B={B}: first batch")
    st, nf = t.insert_at(to_dev(keys), vals_dev(vals), exp_dev(exp), now)
    torch.cuda.synchronize()
    assert (u8(st) == O.INSERTED).all() and int(nf.item()) == 0
    # a second batch: updates of half of the keys and fresh keys, a third of
    # each with a value of 2^48 or more
    fresh = W.distinct_five_tuples(n // 2, 95 + B, stream=W.STREAM_FRESH)
    k2 = np.concatenate([keys[: n // 2], fresh])
    v2 = rng.integers(0, 1 << 48, size=len(k2), dtype=np.int64).astype(np.uint64)
    wide = rng.random(len(k2)) < 1 / 3
    wide[0] = wide[-1] = True
    v2[wide] |= rng.integers(1, 1 << 16, size=int(wide.sum()),
                             dtype=np.int64).astype(np.uint64) << np.uint64(48)
    e2 = np.full(len(k2), (now + 5) & 0xFFFF, np.uint16)
    say(f"wide values B={B}: mixed batch")
    st, nf = t.insert_at(to_dev(k2), vals_dev(v2), exp_dev(e2), now)
    torch.cuda.synchronize()
    st = u8(st)
    assert (st[wide] == O.FAILED).all(), "a value of 2^48 or more must be refused"
    upd = ~wide & (np.arange(len(k2)) < n // 2)
    assert (st[upd] == O.UPDATED).all() and (st[~wide & ~upd] == O.INSERTED).all()
    assert int(nf.item()) == int(wide.sum())
    # the dictionary: refused updates keep the old value, refused fresh keys
    # are absent
    want = {kk.tobytes(): int(v) for kk, v in zip(keys, vals)}
    for i in np.flatnonzero(~wide):
        want[k2[i].tobytes()] = int(v2[i])
    probe = np.concatenate([keys, fresh])
    f, v = t.lookup_at(to_dev(probe), now)
    assert np.array_equal(u8(f), np.array([p.tobytes() in want for p in probe], np.uint8))
    assert np.array_equal(u64(v), np.array([want.get(p.tobytes(), 0) for p in probe], np.uint64))
    check_timed_image(t, B)
    # an oracle image holding a wide value is refused; the table is unchanged
    ref = O.OracleTable(B, W.HASH_SEED, W.MAX_KICKS, timed=True)
    ref.insert_at(k2, v2, e2, now)
    rb, rk = ref.image()
    from paper_1712_09624_amd.ckpp import CkppError, check_image
    assert not check_image(B, rb, rk, timers=True)
    assert check_image(B, rb, rk, timers=False)
    gb, gk = t.export()
    with pytest.raises(CkppError):
        t.import_image(rb, rk)
    gb2, gk2 = t.export()
    assert np.array_equal(gb, gb2) and np.array_equal(gk, gk2)
    t.close()


def test_timed_argument_checks():
    """Calls that do not fit the table's kind, and refresh times outside the
    window, are refused; an image with a too-wide value or time is refused
    and leaves the table unchanged."""
    from paper_1712_09624_amd.ckpp import CkppError, Table
    keys = to_dev(W.distinct_five_tuples(4, 81))
    vals = vals_dev(W.insertion_values(4))
    t = new_timed(6)
    u = Table(6, W.HASH_SEED, device=0)
    say("timed argument checks")
    with pytest.raises(CkppError):
        t.lookup(keys)
    with pytest.raises(CkppError):
        t.insert(keys, vals)
    with pytest.raises(CkppError):
        t.delete(keys)
    with pytest.raises(CkppError):
        u.lookup_at(keys, 5)
    with pytest.raises(CkppError):
        u.expire_scan(5)
    with pytest.raises(CkppError):
        t.lookup_at(keys, 100, refresh=100 + 1024)
    with pytest.raises(CkppError):
        t.lookup_at(keys, 100, refresh=99)
    t.lookup_at(keys, 100, refresh=100 + 1023)
    ref = O.OracleTable(6, W.HASH_SEED, W.MAX_KICKS, timed=True)
    ref.insert_at(W.distinct_five_tuples(4, 81), W.insertion_values(4), np.full(4, 300), 0)
    b, k = ref.image()
    t.import_image(b, k)
    bad = k.copy().reshape(-1, 32)
    busy_rec = int(np.flatnonzero(bad[:, 16:24].any(axis=1) | bad[:, 24:32].any(axis=1))[0])
    bad[busy_rec, 30] = 1  # reserved word >= 2^16
    with pytest.raises(CkppError):
        t.import_image(b, bad.reshape(-1))
    gb, gk = t.export()
    assert np.array_equal(gb, b) and np.array_equal(gk, k)
    t.close()
    u.close()
