"""Seeded synthetic workloads: 16-byte 5-tuple keys, values and lookup mixes.

This module only draws random inputs; it holds none of the hash table's
arithmetic (no hashing, no bucket indexing), so that the oracle and the GPU
library, which are both fed from here, share nothing else.

Keys follow the paper's connection-tracking setting: a 5-tuple (protocol,
source and destination address, source and destination port) packed in 128
bits (Sec. 1 and Sec. 5, common parameters: randomly generated keys, 128-bit
keys).  Byte layout, as four little-endian u32 words:

    w0 = source IPv4 address          (uniform u32)
    w1 = destination IPv4 address     (uniform u32)
    w2 = source port | dest port << 16 (uniform u16 each)
    w3 = protocol in the low byte      (6 or 17, equally likely), 3 zero bytes

Random numbers come from numpy's PCG64 bit generator (M. E. O'Neill, 2014)
through ``random_raw``, whose output stream is fixed by the algorithm's
definition, with ``SeedSequence(seed, spawn_key=(stream,))`` separating the
streams of one workload (keys, lookup mix, delete choice, fresh keys).
"""

from __future__ import annotations

import numpy as np

# Fixed hash seed of every table built by the tests and the benchmark.
HASH_SEED = 0x243F6A8885A308D3
# Paper-scale cuckoo path bound used by the configurations (max kick chain).
MAX_KICKS = 500

# Stream numbers of one workload.
STREAM_KEYS = 0
STREAM_MIX = 1
STREAM_DELETE = 2
STREAM_FRESH = 3
STREAM_NEGATIVE = 4
STREAM_TABLES = 5
STREAM_TIMES = 6


def raw_u64(seed: int, stream: int, n: int) -> np.ndarray:
    """n raw 64-bit draws of PCG64 stream ``stream`` of workload ``seed``."""
    bg = np.random.PCG64(np.random.SeedSequence(seed, spawn_key=(stream,)))
    return bg.random_raw(int(n)).astype(np.uint64, copy=False)


def five_tuples(n: int, seed: int, stream: int = STREAM_KEYS) -> np.ndarray:
    """n random 5-tuple keys as a C-contiguous uint8 array of shape (n, 16)."""
    n = int(n)
    r = raw_u64(seed, stream, 2 * n).reshape(n, 2) if n else np.zeros((0, 2), np.uint64)
    w = np.empty((n, 4), dtype=np.uint32)
    w[:, 0] = (r[:, 0] & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    w[:, 1] = (r[:, 0] >> np.uint64(32)).astype(np.uint32)
    w[:, 2] = (r[:, 1] & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    udp = ((r[:, 1] >> np.uint64(32)) & np.uint64(1)).astype(bool)
    w[:, 3] = np.where(udp, np.uint32(17), np.uint32(6))
    return w.view(np.uint8).reshape(n, 16)


def all_distinct(keys: np.ndarray) -> bool:
    """True when the rows of an (n, 16) uint8 key array are pairwise distinct."""
    if len(keys) < 2:
        return True
    k = np.ascontiguousarray(keys).view(np.uint64).reshape(-1, 2)
    order = np.lexsort((k[:, 1], k[:, 0]))
    s = k[order]
    same = (s[1:, 0] == s[:-1, 0]) & (s[1:, 1] == s[:-1, 1])
    return not bool(same.any())


def distinct_five_tuples(n: int, seed: int, stream: int = STREAM_KEYS,
                         check: bool | None = None) -> np.ndarray:
    """n pairwise distinct keys.

    Keys carry 97 random bits, so among 2^27 keys the chance of any repeat is
    below 1e-13.  Distinctness is verified exactly when ``check`` is true
    (default: for n <= 2^23); a repeat raises instead of being dropped, so the
    stream stays a pure function of (n, seed, stream).
    """
    keys = five_tuples(n, seed, stream)
    if check is None:
        check = n <= (1 << 23)
    if check and not all_distinct(keys):
        raise RuntimeError(f"repeated 5-tuple in stream (seed={seed}, stream={stream}, n={n})")
    return keys


def insertion_values(n: int, start: int = 0) -> np.ndarray:
    """Values are the insertion index of each key (uint64)."""
    return np.arange(start, start + int(n), dtype=np.uint64)


def keys_at_load(log2_buckets: int, load: float) -> int:
    """Number of keys that fills 2^B buckets x 8 slots to ``load``
    (round half up)."""
    slots = 8 << int(log2_buckets)
    return int(np.floor(load * slots + 0.5))


def bernoulli(n: int, rate: float, seed: int, stream: int) -> np.ndarray:
    """n independent booleans, each true with probability ``rate``."""
    if rate <= 0.0:
        return np.zeros(int(n), dtype=bool)
    if rate >= 1.0:
        return np.ones(int(n), dtype=bool)
    u = raw_u64(seed, stream, n) >> np.uint64(11)  # 53 uniform bits
    return u < np.uint64(int(rate * (1 << 53)))


def lookup_mix(live_keys: np.ndarray, n: int, neg_rate: float, seed: int,
               stream: int = STREAM_MIX):
    """A lookup stream over a table holding ``live_keys``.

    Each lookup is independently negative with probability ``neg_rate``
    (the paper's negative lookup rate is an average, Sec. 5 common
    parameters).  Positive lookups pick a live key uniformly with
    replacement; negative lookups are fresh random 5-tuples.

    Returns (keys (n,16) uint8, is_negative (n,) bool, index (n,) int64),
    where ``index`` is the row of ``live_keys`` a positive lookup drew
    (-1 for negatives).
    """
    n = int(n)
    neg = bernoulli(n, neg_rate, seed, stream)
    nneg = int(neg.sum())
    idx = np.full(n, -1, dtype=np.int64)
    keys = np.empty((n, 16), dtype=np.uint8)
    npos = n - nneg
    if npos:
        if len(live_keys) == 0:
            raise ValueError("positive lookups need live keys")
        pick = raw_u64(seed, stream + 100, npos) % np.uint64(len(live_keys))
        pos_rows = np.flatnonzero(~neg)
        idx[pos_rows] = pick.astype(np.int64)
        keys[pos_rows] = live_keys[pick.astype(np.int64)]
    if nneg:
        keys[neg] = five_tuples(nneg, seed, stream + 200)
    return keys, neg, idx


def choose_rows(n_total: int, k: int, seed: int, stream: int = STREAM_DELETE) -> np.ndarray:
    """k distinct row numbers out of n_total, in random order (a seeded
    permutation prefix)."""
    r = raw_u64(seed, stream, n_total)
    return np.argsort(r, kind="stable")[: int(k)]


def log_uniform_sizes(n: int, lo: int, hi: int, seed: int, stream: int) -> np.ndarray:
    """n integers log-uniform in [lo, hi] (burst sizes)."""
    u = (raw_u64(seed, stream, n) >> np.uint64(11)).astype(np.float64) / float(1 << 53)
    v = np.exp(np.log(lo) + u * (np.log(hi + 1) - np.log(lo)))
    return np.clip(np.floor(v).astype(np.int64), lo, hi)


def uniform01(n: int, seed: int, stream: int) -> np.ndarray:
    """n doubles uniform in [0, 1) (53-bit)."""
    return (raw_u64(seed, stream, n) >> np.uint64(11)).astype(np.float64) / float(1 << 53)


def many_tables(ntables: int, seed: int, log2_lo: int = 10, log2_hi: int = 18,
                load_lo: float = 0.6, load_hi: float = 0.95, batch_lo: int = 32,
                batch_hi: int = 4096) -> dict:
    """Parameters of a many-table batching workload: per table, a bucket
    count log-uniform over the powers of two 2^log2_lo..2^log2_hi (the
    exponent uniform), a load uniform in [load_lo, load_hi], a lookup batch
    size uniform in [batch_lo, batch_hi] and a negative-lookup rate uniform
    in [0, 1].  Returns arrays log2_buckets, load, batch, neg_rate."""
    n = int(ntables)
    u = uniform01(4 * n, seed, STREAM_TABLES).reshape(4, n) if n else np.zeros((4, 0))
    span = log2_hi - log2_lo + 1
    return {
        "log2_buckets": (log2_lo + np.floor(u[0] * span)).astype(np.int64),
        "load": load_lo + u[1] * (load_hi - load_lo),
        "batch": (batch_lo + np.floor(u[2] * (batch_hi - batch_lo + 1))).astype(np.int64),
        "neg_rate": u[3],
    }


def zipf_ranks(n: int, universe: int, s: float, seed: int, stream: int) -> np.ndarray:
    """n popularity ranks in [0, universe), rank r drawn with probability
    close to (r + 1)^-s / H(universe, s): the inverse of the continuous
    approximation (density proportional to x^-s on [1, universe + 1)),
    floored, for s != 1."""
    u = uniform01(n, seed, stream)
    a = 1.0 - s
    lo, hi = 1.0, float(universe) + 1.0
    x = (lo ** a + u * (hi ** a - lo ** a)) ** (1.0 / a)
    return np.minimum(np.floor(x).astype(np.int64) - 1, universe - 1)


def poisson_arrivals(n: int, rate: float, seed: int, stream: int) -> np.ndarray:
    """Arrival times (seconds) of n events of a Poisson process of the given
    rate, starting at the first inter-arrival gap."""
    u = uniform01(n, seed, stream)
    return np.cumsum(-np.log1p(-u) / rate)


def times_after(n: int, now: int, width: int, seed: int, stream: int = STREAM_TIMES) -> np.ndarray:
    """n 16-bit times uniform in [now, now + width) modulo 2^16 (expiration
    times set some units ahead of a 16-bit clock)."""
    r = raw_u64(seed, stream, n) % np.uint64(int(width))
    return ((r + np.uint64(int(now))) & np.uint64(0xFFFF)).astype(np.uint16)
