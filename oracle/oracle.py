"""ctypes view of the C reference oracle (``ckpp_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the
benchmark's CPU-baseline leg use this module; the product library never
does.  It shares no code with the GPU library.

Every function here only marshals numpy arrays into the C oracle; the
arithmetic is all in ``ckpp_oracle.c``.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ckpp_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

INSERTED, UPDATED, FAILED = 0, 1, 2
MODE_CUCKOOPP, MODE_BOTH, MODE_OPTIMISTIC = 0, 1, 2
MOVED_BINS = 66
MAX_DELAY = 1024  # expiration times lie within this many time units of now


def build(cc: str = "gcc") -> str:
    """Compiles the oracle into ``oracle/liboracle.so``."""
    tmp = LIB + ".tmp"
    cmd = [cc, "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp, SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


class _Stats(ctypes.Structure):
    _fields_ = [
        ("nbuckets", ctypes.c_uint64),
        ("live", ctypes.c_uint64),
        ("in_secondary", ctypes.c_uint64),
        ("bloom_pc_sum", ctypes.c_uint64),
        ("bloom_pc2_sum", ctypes.c_uint64),
        ("locked", ctypes.c_uint64),
        ("moved_hist", ctypes.c_uint64 * MOVED_BINS),
        ("fpr_from_moved_sum", ctypes.c_double),
    ]


class _Split(ctypes.Structure):
    _fields_ = [
        ("p", ctypes.c_uint64),
        ("a", ctypes.c_uint64),
        ("tag", ctypes.c_uint32),
        ("b1", ctypes.c_uint32),
        ("b2", ctypes.c_uint32),
        ("bloom_mask", ctypes.c_uint64),
    ]


_lib = None


def load(path: str | None = None) -> ctypes.CDLL:
    """Loads the oracle library, building it first if it is missing."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB
    if path is None and not os.path.exists(p):
        build()
    lib = ctypes.CDLL(p)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.orc_hash.restype = ctypes.c_uint64
    lib.orc_hash.argtypes = [u8p, ctypes.c_uint64]
    lib.orc_fmix64_export.restype = ctypes.c_uint64
    lib.orc_fmix64_export.argtypes = [ctypes.c_uint64]
    lib.orc_split.restype = None
    lib.orc_split.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(_Split)]
    lib.orc_create.restype = ctypes.c_void_p
    lib.orc_create.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int]
    lib.orc_destroy.restype = None
    lib.orc_destroy.argtypes = [ctypes.c_void_p]
    lib.orc_buckets_ptr.restype = ctypes.c_void_p
    lib.orc_buckets_ptr.argtypes = [ctypes.c_void_p]
    lib.orc_kv_ptr.restype = ctypes.c_void_p
    lib.orc_kv_ptr.argtypes = [ctypes.c_void_p]
    lib.orc_live.restype = ctypes.c_uint64
    lib.orc_live.argtypes = [ctypes.c_void_p]
    lib.orc_insert_batch.restype = None
    lib.orc_insert_batch.argtypes = [ctypes.c_void_p, u8p, u64p, ctypes.c_uint64, u8p]
    lib.orc_lookup_batch.restype = None
    lib.orc_lookup_batch.argtypes = [ctypes.c_void_p, u8p, ctypes.c_uint64, ctypes.c_int, u8p,
                                     u64p, u64p, u64p]
    lib.orc_delete_batch.restype = None
    lib.orc_delete_batch.argtypes = [ctypes.c_void_p, u8p, ctypes.c_uint64, u8p]
    u16p = ctypes.POINTER(ctypes.c_uint16)
    lib.orc_create_timed.restype = ctypes.c_void_p
    lib.orc_create_timed.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32,
                                     ctypes.c_int]
    lib.orc_insert_batch_at.restype = None
    lib.orc_insert_batch_at.argtypes = [ctypes.c_void_p, u8p, u64p, u16p, ctypes.c_uint64,
                                        ctypes.c_uint16, u8p]
    lib.orc_lookup_batch_at.restype = None
    lib.orc_lookup_batch_at.argtypes = [ctypes.c_void_p, u8p, ctypes.c_uint64, ctypes.c_int,
                                        ctypes.c_uint16, ctypes.c_int, ctypes.c_uint16, u8p, u64p]
    lib.orc_delete_batch_at.restype = None
    lib.orc_delete_batch_at.argtypes = [ctypes.c_void_p, u8p, ctypes.c_uint64, ctypes.c_uint16,
                                        u8p]
    lib.orc_expire_scan.restype = ctypes.c_uint64
    lib.orc_expire_scan.argtypes = [ctypes.c_void_p, ctypes.c_uint16]
    lib.orc_stats.restype = None
    lib.orc_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Stats)]
    lib.orc_image_stats.restype = None
    lib.orc_image_stats.argtypes = [u8p, ctypes.c_uint32, ctypes.POINTER(_Stats)]
    lib.orc_stats_size.restype = ctypes.c_uint64
    lib.orc_check_image.restype = ctypes.c_int
    lib.orc_check_image.argtypes = [u8p, u8p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int,
                                    ctypes.c_char_p, ctypes.c_uint64]
    if lib.orc_stats_size() != ctypes.sizeof(_Stats):
        raise RuntimeError("oracle stats struct size mismatch")
    if path is None:
        _lib = lib
    return lib


def _u8(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _u64(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _keys(keys: np.ndarray) -> np.ndarray:
    k = np.ascontiguousarray(keys, dtype=np.uint8)
    if k.ndim != 2 or k.shape[1] != 16:
        raise ValueError("keys must have shape (n, 16)")
    return k


def _stats_dict(st: _Stats) -> dict:
    nb = int(st.nbuckets)
    live = int(st.live)
    return {
        "nbuckets": nb,
        "live": live,
        "in_secondary": int(st.in_secondary),
        "f_sec": (int(st.in_secondary) / live) if live else 0.0,
        "bloom_pc_sum": int(st.bloom_pc_sum),
        "bloom_pc2_sum": int(st.bloom_pc2_sum),
        "expected_fpr": int(st.bloom_pc2_sum) / (4096.0 * nb),
        "locked": int(st.locked),
        "moved_hist": [int(x) for x in st.moved_hist],
        "moved_zero_fraction": int(st.moved_hist[0]) / nb,
        "fpr_from_moved": float(st.fpr_from_moved_sum) / nb,
    }


def hash_keys(keys: np.ndarray, seed: int, lib=None) -> np.ndarray:
    lib = lib or load()
    k = _keys(keys)
    out = np.empty(len(k), dtype=np.uint64)
    for i in range(len(k)):
        out[i] = lib.orc_hash(_u8(k[i]), ctypes.c_uint64(seed))
    return out


def split(h: int, log2_buckets: int, lib=None) -> dict:
    lib = lib or load()
    sp = _Split()
    lib.orc_split(ctypes.c_uint64(int(h)), log2_buckets, ctypes.byref(sp))
    return {"p": sp.p, "a": sp.a, "tag": sp.tag, "b1": sp.b1, "b2": sp.b2,
            "bloom_mask": sp.bloom_mask}


def fmix64(z: int, lib=None) -> int:
    lib = lib or load()
    return int(lib.orc_fmix64_export(ctypes.c_uint64(int(z))))


def check_image(buckets: np.ndarray, kv: np.ndarray, log2_buckets: int, seed: int,
                plain: bool = False, lib=None, timed: bool = False):
    """Runs the image invariant checker; returns (code, message), code 0 = ok."""
    lib = lib or load()
    b = np.ascontiguousarray(buckets, dtype=np.uint8).reshape(-1)
    k = np.ascontiguousarray(kv, dtype=np.uint8).reshape(-1)
    nb = 1 << log2_buckets
    if b.size != nb * 64 or k.size != nb * 256:
        raise ValueError("image size does not match log2_buckets")
    msg = ctypes.create_string_buffer(512)
    flags = (1 if plain else 0) | (2 if timed else 0)
    rc = lib.orc_check_image(_u8(b), _u8(k), log2_buckets, ctypes.c_uint64(seed), flags, msg,
                             512)
    return int(rc), msg.value.decode()


def image_stats(buckets: np.ndarray, log2_buckets: int, lib=None) -> dict:
    lib = lib or load()
    b = np.ascontiguousarray(buckets, dtype=np.uint8).reshape(-1)
    st = _Stats()
    lib.orc_image_stats(_u8(b), log2_buckets, ctypes.byref(st))
    return _stats_dict(st)


class OracleTable:
    """Single-threaded reference cuckoo table (see ``ckpp_oracle.c``)."""

    def __init__(self, log2_buckets: int, seed: int, max_kicks: int = 500,
                 plain: bool = False, lib=None, timed: bool = False):
        self.lib = lib or load()
        self.log2_buckets = int(log2_buckets)
        self.nbuckets = 1 << self.log2_buckets
        self.seed = int(seed)
        self.plain = bool(plain)
        self.timed = bool(timed)
        create = self.lib.orc_create_timed if timed else self.lib.orc_create
        self._t = create(self.log2_buckets, ctypes.c_uint64(self.seed), int(max_kicks),
                         1 if plain else 0)
        if not self._t:
            raise MemoryError("orc_create failed")

    def close(self):
        if self._t:
            self.lib.orc_destroy(self._t)
            self._t = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def live(self) -> int:
        return int(self.lib.orc_live(self._t))

    def insert(self, keys: np.ndarray, values: np.ndarray) -> np.ndarray:
        k = _keys(keys)
        v = np.ascontiguousarray(values, dtype=np.uint64)
        if len(v) != len(k):
            raise ValueError("keys and values differ in length")
        st = np.empty(len(k), dtype=np.uint8)
        self.lib.orc_insert_batch(self._t, _u8(k), _u64(v), len(k), _u8(st))
        return st

    def lookup(self, keys: np.ndarray, mode: int = MODE_CUCKOOPP):
        """Returns (found u8, values u64, bucket_lines_total, kv_lines_total)."""
        k = _keys(keys)
        f = np.empty(len(k), dtype=np.uint8)
        v = np.empty(len(k), dtype=np.uint64)
        bl = np.zeros(1, dtype=np.uint64)
        kl = np.zeros(1, dtype=np.uint64)
        self.lib.orc_lookup_batch(self._t, _u8(k), len(k), int(mode), _u8(f), _u64(v),
                                  _u64(bl), _u64(kl))
        return f, v, int(bl[0]), int(kl[0])

    def delete(self, keys: np.ndarray) -> np.ndarray:
        k = _keys(keys)
        f = np.empty(len(k), dtype=np.uint8)
        self.lib.orc_delete_batch(self._t, _u8(k), len(k), _u8(f))
        return f

    # -- tables with timers (Sec. 4.2); `now` and expiration times are u16

    def insert_at(self, keys: np.ndarray, values: np.ndarray, expiry: np.ndarray,
                  now: int) -> np.ndarray:
        k = _keys(keys)
        v = np.ascontiguousarray(values, dtype=np.uint64)
        e = np.ascontiguousarray(expiry, dtype=np.uint16)
        if len(v) != len(k) or len(e) != len(k):
            raise ValueError("keys, values and expiry differ in length")
        st = np.empty(len(k), dtype=np.uint8)
        self.lib.orc_insert_batch_at(self._t, _u8(k), _u64(v),
                                     e.ctypes.data_as(ctypes.POINTER(ctypes.c_uint16)), len(k),
                                     int(now) & 0xFFFF, _u8(st))
        return st

    def lookup_at(self, keys: np.ndarray, now: int, mode: int = MODE_CUCKOOPP,
                  refresh: int | None = None):
        """Returns (found u8, values u64); with `refresh` set, every alive
        entry found gets that expiration time."""
        k = _keys(keys)
        f = np.empty(len(k), dtype=np.uint8)
        v = np.empty(len(k), dtype=np.uint64)
        self.lib.orc_lookup_batch_at(self._t, _u8(k), len(k), int(mode), int(now) & 0xFFFF,
                                     0 if refresh is None else 1,
                                     0 if refresh is None else int(refresh) & 0xFFFF,
                                     _u8(f), _u64(v))
        return f, v

    def delete_at(self, keys: np.ndarray, now: int) -> np.ndarray:
        k = _keys(keys)
        f = np.empty(len(k), dtype=np.uint8)
        self.lib.orc_delete_batch_at(self._t, _u8(k), len(k), int(now) & 0xFFFF, _u8(f))
        return f

    def expire_scan(self, now: int) -> int:
        return int(self.lib.orc_expire_scan(self._t, int(now) & 0xFFFF))

    def stats(self) -> dict:
        st = _Stats()
        self.lib.orc_stats(self._t, ctypes.byref(st))
        return _stats_dict(st)

    def image(self):
        """Copies of the bucket array (nb*64 bytes) and key/value array
        (nb*256 bytes)."""
        nb = self.nbuckets
        bp = self.lib.orc_buckets_ptr(self._t)
        kp = self.lib.orc_kv_ptr(self._t)
        b = np.ctypeslib.as_array((ctypes.c_uint8 * (nb * 64)).from_address(bp)).copy()
        k = np.ctypeslib.as_array((ctypes.c_uint8 * (nb * 256)).from_address(kp)).copy()
        return b, k

    def check(self):
        b, k = self.image()
        return check_image(b, k, self.log2_buckets, self.seed, self.plain, lib=self.lib,
                           timed=self.timed)
