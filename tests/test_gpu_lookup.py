"""GPU lookups against the oracle, bit-exact (the lookups of one image have a
unique answer: found flag and value of every key).

The table image is built by the oracle and imported, so the comparison is
free of any insert-order effect."""

import numpy as np
import pytest

from gpu_util import say, to_dev, u64, u8
from oracle import oracle as O
from paper_1712_09624_amd import workload as W

pytestmark = pytest.mark.gpu

MODES = [("cuckoopp", O.MODE_CUCKOOPP), ("both", O.MODE_BOTH), ("optimistic", O.MODE_OPTIMISTIC)]
SHAPES = [(8, per, block, bpc) for per in (1, 2) for block in (64, 128, 256) for bpc in (0, 1, 3)]
SHAPES += [(4, per, block, bpc) for per in (1, 2) for block in (64, 128, 256) for bpc in (0, 3)]
SHAPES += [(1, per, block, bpc) for per in (1, 2, 4) for block in (64, 256) for bpc in (0, 3)]
# the default shape and one of each other form, for the degenerate tables
FORMS = [None, (8, 1, 64, 0), (4, 1, 128, 0), (4, 2, 64, 0), (1, 2, 64, 0)]


@pytest.fixture(scope="module")
def cfg1():
    """Plain method, small: 2^14 buckets at load 0.8 (104858 keys), 2^20
    lookups with half of them fresh keys, seed 1."""
    B = 14
    n = W.keys_at_load(B, 0.8)
    keys = W.distinct_five_tuples(n, 1)
    vals = W.insertion_values(n)
    ref = O.OracleTable(B, W.HASH_SEED, W.MAX_KICKS)
    assert (ref.insert(keys, vals) == O.INSERTED).all()
    look, neg, idx = W.lookup_mix(keys, 1 << 20, 0.5, 1)
    return B, ref, keys, look, neg, idx


def gpu_table_from(ref, plain=False):
    from paper_1712_09624_amd.ckpp import Table
    t = Table(ref.log2_buckets, W.HASH_SEED, W.MAX_KICKS, plain=plain, device=0)
    b, k = ref.image()
    t.import_image(b, k)
    return t


def test_hash_vectors():
    from paper_1712_09624_amd.ckpp import Table
    import oracle_pins as P
    rows = P.read_golden("hash_vectors.txt")
    keys = np.stack([np.frombuffer(bytes.fromhex(r[0]), np.uint8) for r in rows])
    say("ckpp_hash_batch on golden keys")
    t = Table(14, W.HASH_SEED, device=0)
    h = u64(t.hash(to_dev(keys)))
    assert [int(x) for x in h] == [int(r[1], 16) for r in rows]
    t.close()


@pytest.mark.parametrize("mode,omode", MODES, ids=[m[0] for m in MODES])
def test_cfg1_lookup_bit_exact(cfg1, mode, omode):
    B, ref, keys, look, neg, idx = cfg1
    want_f, want_v, _, _ = ref.lookup(look, omode)
    say(f"cfg1 lookup mode={mode} n={len(look)}")
    t = gpu_table_from(ref)
    f, v = t.lookup(to_dev(look), mode)
    assert np.array_equal(u8(f), want_f)
    assert np.array_equal(u64(v), want_v)
    # and the dictionary meaning of the answers
    assert int(want_f.sum()) == int((~neg).sum())
    assert np.array_equal(want_v[~neg], idx[~neg].astype(np.uint64))
    t.close()


@pytest.mark.parametrize("shape", SHAPES, ids=[f"l{s[0]}k{s[1]}b{s[2]}g{s[3]}" for s in SHAPES])
def test_launch_shapes_ragged(cfg1, shape):
    """Every launch shape, on a batch that spans many tiles and ends in a
    ragged tail (n = 2^17 + 77), in every mode."""
    B, ref, keys, look, neg, idx = cfg1
    n = (1 << 17) + 77
    q = look[:n]
    t = gpu_table_from(ref)
    t.set_lookup_launch(*shape)
    for mode, omode in MODES:
        want_f, want_v, _, _ = ref.lookup(q, omode)
        say(f"shape {shape} mode={mode} n={n}")
        f, v = t.lookup(to_dev(q), mode)
        assert np.array_equal(u8(f), want_f), f"{shape} {mode}"
        assert np.array_equal(u64(v), want_v), f"{shape} {mode}"
    t.close()


@pytest.mark.parametrize("n", [1, 2, 63, 65, 255, 257, 1000])
def test_small_batches(cfg1, n):
    B, ref, keys, look, neg, idx = cfg1
    q = look[:n]
    want_f, want_v, _, _ = ref.lookup(q)
    say(f"small batch n={n}")
    t = gpu_table_from(ref)
    f, v = t.lookup(to_dev(q))
    assert np.array_equal(u8(f), want_f) and np.array_equal(u64(v), want_v)
    t.close()


def test_empty_batch_is_noop(cfg1):
    import torch
    from paper_1712_09624_amd.ckpp import Table
    t = Table(8, W.HASH_SEED, device=0)
    z = torch.zeros((0, 16), dtype=torch.uint8, device="cuda:0")
    f, v = t.lookup(z)
    st, nf = t.insert(z, torch.zeros(0, dtype=torch.int64, device="cuda:0"))
    d = t.delete(z)
    torch.cuda.synchronize()
    assert f.numel() == 0 and v.numel() == 0 and st.numel() == 0 and d.numel() == 0
    assert int(nf.item()) == 0
    t.close()


def test_default_launch_shape():
    from paper_1712_09624_amd import ckpp
    t = ckpp.Table(8, W.HASH_SEED, device=0)
    assert t.get_lookup_launch() == ckpp.DEFAULT_LAUNCH
    t.set_lookup_launch(8, 1, 256, 3)
    assert t.get_lookup_launch() == {"lanes_per_lookup": 8, "lookups_per_lane": 1, "block": 256,
                                     "blocks_per_cu": 3}
    t.close()


def test_lookup_launch_rejects_bad_shapes():
    from paper_1712_09624_amd import ckpp
    t = ckpp.Table(8, W.HASH_SEED, device=0)
    for shape in ((2, 1, 128, 0), (4, 3, 128, 0), (4, 4, 128, 0), (8, 4, 128, 0), (1, 3, 128, 0),
                  (8, 1, 96, 0), (4, 1, 512, 0)):
        with pytest.raises(ckpp.CkppError):
            t.set_lookup_launch(*shape)
    assert t.get_lookup_launch() == ckpp.DEFAULT_LAUNCH
    t.close()


def test_empty_table_misses_everything():
    from paper_1712_09624_amd.ckpp import Table
    q = W.five_tuples(5000, 3)
    t = Table(12, W.HASH_SEED, device=0)
    for mode, _ in MODES:
        say(f"empty table mode={mode}")
        f, v = t.lookup(to_dev(q), mode)
        assert not u8(f).any() and not u64(v).any()
    t.close()


@pytest.mark.parametrize("form", FORMS, ids=lambda s: "default" if s is None else f"l{s[0]}k{s[1]}")
@pytest.mark.parametrize("B,load", [(1, 1.0), (2, 0.95), (3, 0.9), (6, 0.95), (10, 0.95)])
def test_tiny_and_full_tables(B, load, form):
    """Degenerate sizes: 2 buckets (every key shares the pair), and tables
    filled to high load, where many keys sit in their secondary bucket."""
    n = W.keys_at_load(B, load)
    keys = W.distinct_five_tuples(n, 40 + B)
    ref = O.OracleTable(B, W.HASH_SEED, W.MAX_KICKS)
    st = ref.insert(keys, W.insertion_values(n))
    look = np.concatenate([keys, W.five_tuples(4 * n + 10, 50 + B)])
    t = gpu_table_from(ref)
    if form:
        t.set_lookup_launch(*form)
    for mode, omode in MODES:
        want_f, want_v, _, _ = ref.lookup(look, omode)
        assert int(want_f[:n].sum()) == int((st == O.INSERTED).sum())
        say(f"tiny B={B} load={load} mode={mode} shape={form}")
        f, v = t.lookup(to_dev(look), mode)
        assert np.array_equal(u8(f), want_f) and np.array_equal(u64(v), want_v)
    t.close()


@pytest.mark.parametrize("form", FORMS, ids=lambda s: "default" if s is None else f"l{s[0]}k{s[1]}")
def test_colliding_keys(form):
    """Keys sharing bucket, tag and the first 8 bytes keep their own values."""
    import oracle_pins as P
    k1, k2 = P.colliding_pair(O.load())
    keys = np.stack([k1, k2])
    ref = O.OracleTable(1, W.HASH_SEED, W.MAX_KICKS)
    ref.insert(keys, np.array([11, 22], np.uint64))
    t = gpu_table_from(ref)
    if form:
        t.set_lookup_launch(*form)
    for mode, _ in MODES:
        say(f"colliding keys mode={mode} shape={form}")
        f, v = t.lookup(to_dev(keys), mode)
        assert list(u8(f)) == [1, 1] and list(u64(v)) == [11, 22]
    t.close()


def test_plain_table_lookup():
    """A plain table (no filters) answers like the oracle's plain table; its
    default lookup probes both buckets."""
    B = 12
    n = W.keys_at_load(B, 0.95)
    keys = W.distinct_five_tuples(n, 61)
    ref = O.OracleTable(B, W.HASH_SEED, W.MAX_KICKS, plain=True)
    ref.insert(keys, W.insertion_values(n))
    look, _, _ = W.lookup_mix(keys, 1 << 16, 0.5, 62)
    t = gpu_table_from(ref, plain=True)
    for mode, omode in MODES:
        want_f, want_v, _, _ = ref.lookup(look, omode)
        say(f"plain table mode={mode}")
        f, v = t.lookup(to_dev(look), mode)
        assert np.array_equal(u8(f), want_f) and np.array_equal(u64(v), want_v)
    t.close()


@pytest.mark.parametrize("load", [0.6, 0.95])
def test_mall_sized_table(load):
    """2^20 buckets (64 MiB of buckets: cache-resident size class) at low and
    high load, 2^22 lookups at negative rate 0.5."""
    B = 20
    n = W.keys_at_load(B, load)
    keys = W.distinct_five_tuples(n, 70)
    ref = O.OracleTable(B, W.HASH_SEED, W.MAX_KICKS)
    assert (ref.insert(keys, W.insertion_values(n)) == O.INSERTED).all()
    look, neg, idx = W.lookup_mix(keys, 1 << 22, 0.5, 71)
    t = gpu_table_from(ref)
    for mode, omode in MODES:
        want_f, want_v, _, _ = ref.lookup(look, omode)
        say(f"B=20 load={load} mode={mode}")
        f, v = t.lookup(to_dev(look), mode)
        assert np.array_equal(u8(f), want_f) and np.array_equal(u64(v), want_v)
    t.close()


def test_image_round_trip_and_stats(cfg1):
    """export(import(image)) reproduces the oracle's image byte for byte (the
    device layout differs from the interchange layout), and the device
    statistics of the imported table equal the oracle's."""
    B, ref, keys, look, neg, idx = cfg1
    b, k = ref.image()
    say("import/export round trip")
    t = gpu_table_from(ref)
    b2, k2 = t.export()
    assert np.array_equal(b, b2), "bucket image differs after the round trip"
    assert np.array_equal(k, k2), "record image differs after the round trip"
    s, want = t.stats(), ref.stats()
    for f in ("live", "in_secondary", "bloom_pc_sum", "bloom_pc2_sum", "locked", "moved_hist"):
        assert s[f] == want[f], f
    busy = b.reshape(-1, 64)[:, 26]
    sec = b.reshape(-1, 64)[:, 27]
    assert s["high_slots"] == int(np.unpackbits(busy & 0xF0).sum())
    assert s["high_slots_secondary"] == int(np.unpackbits(sec & 0xF0).sum())
    t.close()
