"""Pins of the reference oracle (CPU only)."""

import numpy as np
import pytest

import oracle_pins as P
from oracle import oracle as O
from paper_1712_09624_amd import workload as W


@pytest.fixture(scope="module")
def lib():
    return O.load()


def test_splitmix_finalizer(lib):
    P.pin_splitmix_finalizer(lib)


def test_hash_composition(lib):
    P.pin_hash_composition(lib)


def test_split_properties(lib):
    P.pin_split_properties(lib)


def test_hash_uniformity(lib):
    P.pin_hash_uniformity(lib)


@pytest.mark.parametrize("B", [1, 2, 3, 5, 8])
def test_dict_differential_cuckoopp(lib, B):
    P.pin_dict_differential(lib, B=B, rounds=30, seed=B)


@pytest.mark.parametrize("B", [1, 3, 6])
def test_dict_differential_plain(lib, B):
    P.pin_dict_differential(lib, B=B, rounds=20, seed=100 + B, plain=True)


def test_two_bucket_capacity(lib):
    P.pin_two_bucket_capacity(lib)


def test_lookup_costs(lib):
    P.pin_lookup_costs(lib)


def test_fpr_closed_form(lib):
    P.pin_fpr_closed_form(lib)


def test_empty_batches(lib):
    t = O.OracleTable(4, W.HASH_SEED, lib=lib)
    z = np.zeros((0, 16), np.uint8)
    assert len(t.insert(z, np.zeros(0, np.uint64))) == 0
    f, v, bl, kl = t.lookup(z)
    assert len(f) == 0 and bl == 0 and kl == 0
    assert len(t.delete(z)) == 0
    assert t.check() == (0, "")


def test_zero_kicks_fails_when_both_buckets_full(lib):
    # with max_kicks 0 no path is searched: a key fails as soon as both of
    # its buckets are full, and the table is unchanged
    keys = W.distinct_five_tuples(17, 5, check=True)
    t = O.OracleTable(1, W.HASH_SEED, 0, lib=lib)
    assert (t.insert(keys[:16], W.insertion_values(16)) == O.INSERTED).all()
    assert t.insert(keys[16:], W.insertion_values(1))[0] == O.FAILED


def test_delete_cycle(lib):
    P.pin_delete_cycle(lib)


def test_check_image_detects_corruption(lib):
    B = 8
    n = W.keys_at_load(B, 0.9)
    keys = W.distinct_five_tuples(n, 9, check=True)
    t = O.OracleTable(B, W.HASH_SEED, lib=lib)
    t.insert(keys, W.insertion_values(n))
    b, k = t.image()
    assert O.check_image(b, k, B, W.HASH_SEED)[0] == 0
    bk = b.reshape(-1, 64)
    # a displaced key's bloom bits cleared -> I4 or I5
    i = int(np.flatnonzero(bk[:, 24:26].copy().view(np.uint16)[:, 0] > 0)[0])
    bad = b.copy().reshape(-1, 64)
    bad[i, 16:24] = 0
    assert O.check_image(bad.reshape(-1), k, B, W.HASH_SEED)[0] in (4, 5)
    # a tag changed -> I1
    j = int(np.flatnonzero(bk[:, 26])[0])
    bad = b.copy().reshape(-1, 64)
    s = int(np.flatnonzero(np.unpackbits(bad[j, 26:27], bitorder="little"))[0])
    bad[j, 2 * s] ^= 1
    assert O.check_image(bad.reshape(-1), k, B, W.HASH_SEED)[0] == 1
    # a lock left set -> I9
    bad = b.copy().reshape(-1, 64)
    bad[3, 28] = 1
    assert O.check_image(bad.reshape(-1), k, B, W.HASH_SEED)[0] == 9


@pytest.mark.slow
def test_paper_statistics_32M(lib):
    P.pin_paper_statistics(P.paper_statistics(lib, B=22))


def test_full_key_compare(lib):
    P.pin_full_key_compare(lib)


def test_paper_statistics_small_table(lib):
    # the statistics hardly depend on the table size; 2^17 buckets is the
    # size the planted-mistake runs use
    P.pin_paper_statistics(P.paper_statistics(lib, B=17))


def test_hash_vectors_regression(lib):
    # the frozen vectors the GPU hash is compared with still come out of the
    # oracle (they were written by tests/golden/make_golden.py)
    rows = P.read_golden("hash_vectors.txt")
    assert len(rows) >= 32
    for key_hex, h_hex, p14, a14, tag, p24, a24 in rows:
        k = np.frombuffer(bytes.fromhex(key_hex), np.uint8).reshape(1, 16)
        h = int(O.hash_keys(k, W.HASH_SEED, lib=lib)[0])
        assert h == int(h_hex, 16)
        s14, s24 = O.split(h, 14, lib=lib), O.split(h, 24, lib=lib)
        assert (s14["p"], s14["a"], s14["tag"]) == (int(p14), int(a14), int(tag))
        assert (s24["p"], s24["a"]) == (int(p24), int(a24))


@pytest.mark.parametrize("B,plain", [(1, False), (3, False), (5, False), (4, True)])
def test_timer_dict_differential(lib, B, plain):
    P.pin_timer_dict_differential(lib, B=B, rounds=60, seed=20 + B, plain=plain)


def test_timer_revival(lib):
    P.pin_timer_revival(lib)


def test_timer_lazy_reuse(lib):
    P.pin_timer_lazy_reuse(lib)


def test_timer_reduces_to_untimed(lib):
    P.pin_timer_reduces_to_untimed(lib)
