"""Python binding of ``libckpp.so`` (the C ABI declared in ``include/ckpp.h``).

Argument marshalling only: every step of every operation runs in the HIP
library.  Device buffers are torch tensors (PyTorch provides device memory
and streams); there is no CPU fallback -- without the built library every
call raises.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libckpp.so")

OK, EINVAL, ENOMEM, EDEVICE = 0, 1, 2, 3
INSERTED, UPDATED, FAILED = 0, 1, 2
# gave up after the table's retry limit on contended locks (insert status, and
# the delete outcome beside 0/1): nothing changed for that key
RETRY = 3
MAX_RETRY_LIMIT = 1 << 20
PLAIN = 1
TIMERS = 2  # entries carry 16-bit expiration times (Sec. 4.2); device limit: values < 2^48
MAX_DELAY = 1024
LOOKUP_DEFAULT, LOOKUP_BOTH, LOOKUP_OPTIMISTIC = 0, 1, 2
MODES = {"cuckoopp": LOOKUP_DEFAULT, "default": LOOKUP_DEFAULT, "both": LOOKUP_BOTH,
         "plain": LOOKUP_BOTH, "pessimistic": LOOKUP_BOTH, "optimistic": LOOKUP_OPTIMISTIC}
MOVED_BINS = 66
DEFAULT_HASH_SEED = 0x243F6A8885A308D3
# lookup launch shape a new table starts with (ckpp_create sets the same)
DEFAULT_LAUNCH = {"lanes_per_lookup": 8, "lookups_per_lane": 2, "block": 128, "blocks_per_cu": 0}


def lookup_kernel_name(launch: dict, mode: str = "cuckoopp") -> str:
    """Name of the lookup kernel a launch shape selects for a lookup mode."""
    if launch["lanes_per_lookup"] == 1:
        return "lookup_reg"
    if launch["lanes_per_lookup"] == 4:
        return "lookup_quad"
    if launch["lookups_per_lane"] == 2 and mode != "both":
        return "lookup_dual"
    return "lookup_lds"


class CkppError(RuntimeError):
    pass


class _Stats(ctypes.Structure):
    _fields_ = [
        ("nbuckets", ctypes.c_uint64),
        ("live", ctypes.c_uint64),
        ("in_secondary", ctypes.c_uint64),
        ("bloom_pc_sum", ctypes.c_uint64),
        ("bloom_pc2_sum", ctypes.c_uint64),
        ("locked", ctypes.c_uint64),
        ("high_slots", ctypes.c_uint64),
        ("high_slots_secondary", ctypes.c_uint64),
        ("retry_exhausted", ctypes.c_uint64),
        ("moved_hist", ctypes.c_uint64 * MOVED_BINS),
    ]


class _Info(ctypes.Structure):
    _fields_ = [
        ("log2_buckets", ctypes.c_uint32),
        ("max_kicks", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("device", ctypes.c_int),
        ("hash_seed", ctypes.c_uint64),
        ("image_bucket_bytes", ctypes.c_uint64),
        ("image_kv_bytes", ctypes.c_uint64),
        ("device_bytes", ctypes.c_uint64),
        ("d_table", ctypes.c_void_p),
    ]


class _Launch(ctypes.Structure):
    _fields_ = [
        ("lanes_per_lookup", ctypes.c_uint32),
        ("lookups_per_lane", ctypes.c_uint32),
        ("block", ctypes.c_uint32),
        ("blocks_per_cu", ctypes.c_uint32),
    ]


class _PlanLaunch(ctypes.Structure):
    _fields_ = [
        ("lookups_per_lane", ctypes.c_uint32),
        ("block", ctypes.c_uint32),
        ("blocks_per_cu", ctypes.c_uint32),
        ("passes_per_item", ctypes.c_uint32),
        ("schedule", ctypes.c_uint32),
        ("lanes_per_lookup", ctypes.c_uint32),
    ]


class _PlanInfo(ctypes.Structure):
    _fields_ = [
        ("ntables", ctypes.c_uint32),
        ("nitems", ctypes.c_uint32),
        ("lookups", ctypes.c_uint64),
        ("key_span", ctypes.c_uint64),
    ]


class _ServerConfig(ctypes.Structure):
    _fields_ = [
        ("capacity", ctypes.c_uint64),
        ("budget", ctypes.c_uint64),
        ("mode", ctypes.c_uint32),
        ("blocks_per_cu", ctypes.c_uint32),
        ("idle_ms", ctypes.c_uint32),
        ("ttl", ctypes.c_uint32),
    ]


class _ServerRings(ctypes.Structure):
    _fields_ = [
        ("d_lookup_keys", ctypes.c_void_p),
        ("d_lookup_found", ctypes.c_void_p),
        ("d_lookup_values", ctypes.c_void_p),
        ("d_insert_keys", ctypes.c_void_p),
        ("d_insert_values", ctypes.c_void_p),
        ("d_insert_status", ctypes.c_void_p),
        ("d_delete_keys", ctypes.c_void_p),
        ("d_delete_found", ctypes.c_void_p),
        ("capacity", ctypes.c_uint64),
    ]


class _ServerStatus(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64),
        ("completed", ctypes.c_uint64),
        ("lookup_tail", ctypes.c_uint64),
        ("insert_tail", ctypes.c_uint64),
        ("delete_tail", ctypes.c_uint64),
        ("rounds", ctypes.c_uint64),
        ("launches", ctypes.c_uint64),
        ("state", ctypes.c_uint32),
        ("grid", ctypes.c_uint32),
        ("lookup_ns", ctypes.c_uint64),
        ("insert_ns", ctypes.c_uint64),
        ("delete_ns", ctypes.c_uint64),
        ("boundary_ns", ctypes.c_uint64),
        ("wait_ns", ctypes.c_uint64),
    ]


EBUSY, ETIMEOUT = 4, 5
SERVER_STOPPED, SERVER_RUNNING, SERVER_EXITING, SERVER_ABORTED = 0, 1, 2, 3
SERVER_REFRESH = 1 << 16

# launch shape a new plan starts with (ckpp_plan_create sets the same)
PLAN_STATIC, PLAN_DYNAMIC = 0, 1
DEFAULT_PLAN_LAUNCH = {"lookups_per_lane": 1, "block": 128, "blocks_per_cu": 8,
                       "passes_per_item": 1, "schedule": PLAN_STATIC, "lanes_per_lookup": 8}

_lib = None

# (name, restype, argtypes) of every exported entry point
_VP, _U32, _U64, _I = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
SIGNATURES = [
    ("ckpp_create", _I, [ctypes.POINTER(_VP), _U32, _U64, _U32, _U32, _I]),
    ("ckpp_destroy", _I, [_VP]),
    ("ckpp_clear", _I, [_VP, _VP]),
    ("ckpp_insert_batch", _I, [_VP, _VP, _VP, _U64, _VP, _VP, _VP]),
    ("ckpp_insert_batch_noalloc", _I, [_VP, _VP, _VP, _U64, _VP, _VP, _VP]),
    ("ckpp_lookup_batch", _I, [_VP, _VP, _U64, _U32, _VP, _VP, _VP]),
    ("ckpp_delete_batch", _I, [_VP, _VP, _U64, _VP, _VP]),
    ("ckpp_insert_batch_at", _I, [_VP, _VP, _VP, _VP, _U64, ctypes.c_uint16, _VP, _VP, _VP]),
    ("ckpp_lookup_batch_at", _I, [_VP, _VP, _U64, _U32, ctypes.c_uint16, _U32, ctypes.c_uint16,
                                  _VP, _VP, _VP]),
    ("ckpp_delete_batch_at", _I, [_VP, _VP, _U64, ctypes.c_uint16, _VP, _VP]),
    ("ckpp_expire_scan", _I, [_VP, ctypes.c_uint16, _VP, _VP]),
    ("ckpp_export", _I, [_VP, _VP, _VP, _VP]),
    ("ckpp_import", _I, [_VP, _VP, _VP, _VP]),
    ("ckpp_stats", _I, [_VP, ctypes.POINTER(_Stats), _VP]),
    ("ckpp_hash_batch", _I, [_VP, _VP, _U64, _VP, _VP]),
    ("ckpp_info", _I, [_VP, ctypes.POINTER(_Info)]),
    ("ckpp_set_lookup_launch", _I, [_VP, ctypes.POINTER(_Launch)]),
    ("ckpp_get_lookup_launch", _I, [_VP, ctypes.POINTER(_Launch)]),
    ("ckpp_set_retry_limit", _I, [_VP, _U32]),
    ("ckpp_get_retry_limit", _I, [_VP, ctypes.POINTER(_U32)]),
    ("ckpp_check_image", _I, [_U32, _U32, _VP, _VP]),
    ("ckpp_plan_create", _I, [ctypes.POINTER(_VP), ctypes.POINTER(_VP), _U32, _VP, _VP, _VP]),
    ("ckpp_plan_destroy", _I, [_VP]),
    ("ckpp_plan_lookup", _I, [_VP, _VP, _VP, _VP, _VP]),
    ("ckpp_plan_lookup_at", _I, [_VP, _VP, _VP, _VP, ctypes.c_uint16, _U32, ctypes.c_uint16,
                                 _VP]),
    ("ckpp_plan_set_launch", _I, [_VP, ctypes.POINTER(_PlanLaunch)]),
    ("ckpp_plan_get_launch", _I, [_VP, ctypes.POINTER(_PlanLaunch)]),
    ("ckpp_plan_info", _I, [_VP, ctypes.POINTER(_PlanInfo)]),
    ("ckpp_server_create", _I, [ctypes.POINTER(_VP), _VP, ctypes.POINTER(_ServerConfig)]),
    ("ckpp_server_rings", _I, [_VP, ctypes.POINTER(_ServerRings)]),
    ("ckpp_server_put", _I, [_VP, _U32, _U64, _VP, _VP, _U32, _VP]),
    ("ckpp_server_get", _I, [_VP, _U32, _U64, _U32, _VP, _VP, _VP]),
    ("ckpp_server_submit", _I, [_VP, _U32, _U32, _U32, ctypes.POINTER(_U64)]),
    ("ckpp_server_status", _I, [_VP, ctypes.POINTER(_ServerStatus)]),
    ("ckpp_server_wait", _I, [_VP, _U64, _U32]),
    ("ckpp_server_set_time", _I, [_VP, ctypes.c_uint16]),
    ("ckpp_server_replay", _I, [_VP, _U64, _VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_double]),
    ("ckpp_server_destroy", _I, [_VP]),
    ("ckpp_probe_random_reads", _I, [_VP, _U64, _U32, _U64, _U32, _U32, _U32, _U32, _U64, _VP,
                                     _VP]),
    ("ckpp_probe_latency", _I, [_VP, _U64, _U32, _U32, _U64, _VP, _VP]),
    ("ckpp_strerror", ctypes.c_char_p, [_I]),
]


def load(path: str | None = None) -> ctypes.CDLL:
    """Loads the HIP library; raises when it has not been built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise CkppError(f"{p} is not built: run `python -m paper_1712_09624_amd.build` "
                        "(there is no CPU fallback)")
    lib = ctypes.CDLL(p)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


def _check(rc: int, what: str):
    if rc != OK:
        msg = load().ckpp_strerror(rc).decode()
        raise CkppError(f"{what}: {msg} (status {rc})")


def _torch():
    import torch
    return torch


def _stream_handle(stream) -> int:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _keys_ptr(keys) -> tuple[int, int]:
    """(device pointer, n) of a contiguous (n, 16) byte tensor (any 16-byte
    row dtype view is accepted)."""
    torch = _torch()
    if not keys.is_cuda:
        raise CkppError("keys must be a device tensor")
    if not keys.is_contiguous():
        raise CkppError("keys must be contiguous")
    nbytes = keys.numel() * keys.element_size()
    if nbytes % 16:
        raise CkppError("keys must be a whole number of 16-byte rows")
    if keys.data_ptr() % 16:
        raise CkppError("keys must be 16-byte aligned")
    del torch
    return keys.data_ptr(), nbytes // 16


def check_image(log2_buckets: int, buckets: np.ndarray, kv: np.ndarray, plain: bool = False,
                timers: bool = False) -> bool:
    """Host-only image check of ckpp_check_image (the one ckpp_import
    applies): True when the library would accept the image."""
    b = np.ascontiguousarray(buckets, dtype=np.uint8).reshape(-1)
    k = np.ascontiguousarray(kv, dtype=np.uint8).reshape(-1)
    if b.size != 64 << log2_buckets or k.size != 256 << log2_buckets:
        raise CkppError("image size does not match the bucket count")
    flags = (PLAIN if plain else 0) | (TIMERS if timers else 0)
    rc = load().ckpp_check_image(int(log2_buckets), flags, b.ctypes.data, k.ctypes.data)
    if rc not in (OK, EINVAL):
        _check(rc, "ckpp_check_image")
    return rc == OK


class Table:
    """A Cuckoo++ hash table in device memory (see include/ckpp.h)."""

    def __init__(self, log2_buckets: int, hash_seed: int = DEFAULT_HASH_SEED,
                 max_kicks: int = 500, plain: bool = False, device: int | None = None,
                 timers: bool = False):
        torch = _torch()
        self.lib = load()
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        self.log2_buckets = int(log2_buckets)
        self.nbuckets = 1 << self.log2_buckets
        self.hash_seed = int(hash_seed)
        self.plain = bool(plain)
        self.timers = bool(timers)
        h = ctypes.c_void_p()
        rc = self.lib.ckpp_create(ctypes.byref(h), self.log2_buckets,
                                  ctypes.c_uint64(self.hash_seed), int(max_kicks),
                                  (PLAIN if plain else 0) | (TIMERS if timers else 0),
                                  self.device)
        _check(rc, "ckpp_create")
        self._h = h

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.ckpp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self) -> int:
        return self._h.value

    def _dev(self):
        return _torch().device("cuda", self.device)

    # -- batches
    def insert(self, keys, values, status=None, nfailed=None, stream=None):
        """Enqueues an insert batch; returns (status u8[n], nfailed i64[1])."""
        torch = _torch()
        kp, n = _keys_ptr(keys)
        if values.numel() != n or values.element_size() != 8 or not values.is_contiguous():
            raise CkppError("values must be n contiguous 64-bit integers")
        if status is None:
            status = torch.empty(n, dtype=torch.uint8, device=self._dev())
        if nfailed is None:
            nfailed = torch.zeros(1, dtype=torch.int64, device=self._dev())
        rc = self.lib.ckpp_insert_batch(self._h, kp, values.data_ptr(), n, status.data_ptr(),
                                        nfailed.data_ptr(), _stream_handle(stream))
        _check(rc, "ckpp_insert_batch")
        return status, nfailed

    def insert_noalloc(self, keys, values, status, nfailed, stream=None):
        """ckpp_insert_batch_noalloc: the insert without any allocation; the
        caller passes the status (u8[n]) and nfailed (i64[1]) buffers."""
        kp, n = _keys_ptr(keys)
        if values.numel() != n or values.element_size() != 8 or not values.is_contiguous():
            raise CkppError("values must be n contiguous 64-bit integers")
        if status.numel() < n or nfailed.numel() < 1:
            raise CkppError("status needs n bytes and nfailed one 64-bit word")
        rc = self.lib.ckpp_insert_batch_noalloc(self._h, kp, values.data_ptr(), n,
                                                status.data_ptr(), nfailed.data_ptr(),
                                                _stream_handle(stream))
        _check(rc, "ckpp_insert_batch_noalloc")
        return status, nfailed

    def lookup(self, keys, mode="cuckoopp", found=None, values=None, stream=None):
        """Enqueues a lookup batch; returns (found u8[n], values i64[n])."""
        torch = _torch()
        kp, n = _keys_ptr(keys)
        m = MODES[mode] if isinstance(mode, str) else int(mode)
        if found is None:
            found = torch.empty(n, dtype=torch.uint8, device=self._dev())
        if values is None:
            values = torch.empty(n, dtype=torch.int64, device=self._dev())
        rc = self.lib.ckpp_lookup_batch(self._h, kp, n, m, found.data_ptr(), values.data_ptr(),
                                        _stream_handle(stream))
        _check(rc, "ckpp_lookup_batch")
        return found, values

    def delete(self, keys, found=None, stream=None):
        """Enqueues a delete batch; returns found u8[n]."""
        torch = _torch()
        kp, n = _keys_ptr(keys)
        if found is None:
            found = torch.empty(n, dtype=torch.uint8, device=self._dev())
        rc = self.lib.ckpp_delete_batch(self._h, kp, n, found.data_ptr(), _stream_handle(stream))
        _check(rc, "ckpp_delete_batch")
        return found

    # -- batches on a table with timers (Sec. 4.2); now and times are u16
    def insert_at(self, keys, values, expiry, now, status=None, nfailed=None, stream=None):
        """Enqueues an insert batch with one expiration time per key (u16
        tensor); returns (status u8[n], nfailed i64[1])."""
        torch = _torch()
        kp, n = _keys_ptr(keys)
        if values.numel() != n or values.element_size() != 8 or not values.is_contiguous():
            raise CkppError("values must be n contiguous 64-bit integers")
        if expiry.numel() != n or expiry.element_size() != 2 or not expiry.is_contiguous():
            raise CkppError("expiry must be n contiguous 16-bit integers")
        if status is None:
            status = torch.empty(n, dtype=torch.uint8, device=self._dev())
        if nfailed is None:
            nfailed = torch.zeros(1, dtype=torch.int64, device=self._dev())
        rc = self.lib.ckpp_insert_batch_at(self._h, kp, values.data_ptr(), expiry.data_ptr(), n,
                                           int(now) & 0xFFFF, status.data_ptr(),
                                           nfailed.data_ptr(), _stream_handle(stream))
        _check(rc, "ckpp_insert_batch_at")
        return status, nfailed

    def lookup_at(self, keys, now, mode="cuckoopp", refresh=None, found=None, values=None,
                  stream=None):
        """Enqueues a lookup batch at time `now`; with `refresh` (a u16 time)
        every entry found gets that expiration time.  Returns (found, values)."""
        torch = _torch()
        kp, n = _keys_ptr(keys)
        m = MODES[mode] if isinstance(mode, str) else int(mode)
        if found is None:
            found = torch.empty(n, dtype=torch.uint8, device=self._dev())
        if values is None:
            values = torch.empty(n, dtype=torch.int64, device=self._dev())
        rc = self.lib.ckpp_lookup_batch_at(self._h, kp, n, m, int(now) & 0xFFFF,
                                           0 if refresh is None else 1,
                                           0 if refresh is None else int(refresh) & 0xFFFF,
                                           found.data_ptr(), values.data_ptr(),
                                           _stream_handle(stream))
        _check(rc, "ckpp_lookup_batch_at")
        return found, values

    def delete_at(self, keys, now, found=None, stream=None):
        """Enqueues a delete batch at time `now`; returns found u8[n]."""
        torch = _torch()
        kp, n = _keys_ptr(keys)
        if found is None:
            found = torch.empty(n, dtype=torch.uint8, device=self._dev())
        rc = self.lib.ckpp_delete_batch_at(self._h, kp, n, int(now) & 0xFFFF, found.data_ptr(),
                                           _stream_handle(stream))
        _check(rc, "ckpp_delete_batch_at")
        return found

    def expire_scan(self, now, removed=None, stream=None):
        """Enqueues the anti-revival scan; returns the removed-entry counter
        (i64[1], incremented)."""
        torch = _torch()
        if removed is None:
            removed = torch.zeros(1, dtype=torch.int64, device=self._dev())
        rc = self.lib.ckpp_expire_scan(self._h, int(now) & 0xFFFF, removed.data_ptr(),
                                       _stream_handle(stream))
        _check(rc, "ckpp_expire_scan")
        return removed

    def hash(self, keys, stream=None):
        torch = _torch()
        kp, n = _keys_ptr(keys)
        out = torch.empty(n, dtype=torch.int64, device=self._dev())
        rc = self.lib.ckpp_hash_batch(self._h, kp, n, out.data_ptr(), _stream_handle(stream))
        _check(rc, "ckpp_hash_batch")
        return out

    def clear(self, stream=None):
        _check(self.lib.ckpp_clear(self._h, _stream_handle(stream)), "ckpp_clear")

    # -- inspection
    def export(self, stream=None):
        """Host copies (numpy uint8) of the bucket and key/value arrays."""
        b = np.empty(64 * self.nbuckets, dtype=np.uint8)
        k = np.empty(256 * self.nbuckets, dtype=np.uint8)
        rc = self.lib.ckpp_export(self._h, b.ctypes.data, k.ctypes.data, _stream_handle(stream))
        _check(rc, "ckpp_export")
        return b, k

    def import_image(self, buckets: np.ndarray, kv: np.ndarray, stream=None):
        b = np.ascontiguousarray(buckets, dtype=np.uint8).reshape(-1)
        k = np.ascontiguousarray(kv, dtype=np.uint8).reshape(-1)
        if b.size != 64 * self.nbuckets or k.size != 256 * self.nbuckets:
            raise CkppError("image size does not match the table")
        rc = self.lib.ckpp_import(self._h, b.ctypes.data, k.ctypes.data, _stream_handle(stream))
        _check(rc, "ckpp_import")

    def set_retry_limit(self, limit: int):
        """Attempts per key on contended bucket locks before CKPP_RETRY."""
        _check(self.lib.ckpp_set_retry_limit(self._h, int(limit)), "ckpp_set_retry_limit")

    def retry_limit(self) -> int:
        out = ctypes.c_uint32()
        _check(self.lib.ckpp_get_retry_limit(self._h, ctypes.byref(out)), "ckpp_get_retry_limit")
        return int(out.value)

    def stats(self, stream=None) -> dict:
        st = _Stats()
        _check(self.lib.ckpp_stats(self._h, ctypes.byref(st), _stream_handle(stream)),
               "ckpp_stats")
        nb = int(st.nbuckets)
        live = int(st.live)
        hist = [int(x) for x in st.moved_hist]
        return {
            "nbuckets": nb,
            "live": live,
            "in_secondary": int(st.in_secondary),
            "f_sec": int(st.in_secondary) / live if live else 0.0,
            "bloom_pc_sum": int(st.bloom_pc_sum),
            "bloom_pc2_sum": int(st.bloom_pc2_sum),
            "expected_fpr": int(st.bloom_pc2_sum) / (4096.0 * nb),
            "locked": int(st.locked),
            "high_slots": int(st.high_slots),
            "high_slots_secondary": int(st.high_slots_secondary),
            "retry_exhausted": int(st.retry_exhausted),
            "moved_hist": hist,
            "moved_zero_fraction": hist[0] / nb,
        }

    def info(self) -> dict:
        inf = _Info()
        _check(self.lib.ckpp_info(self._h, ctypes.byref(inf)), "ckpp_info")
        return {f: getattr(inf, f) for f, _ in _Info._fields_}

    def set_lookup_launch(self, lanes_per_lookup=DEFAULT_LAUNCH["lanes_per_lookup"],
                          lookups_per_lane=DEFAULT_LAUNCH["lookups_per_lane"],
                          block=DEFAULT_LAUNCH["block"],
                          blocks_per_cu=DEFAULT_LAUNCH["blocks_per_cu"]):
        cfg = _Launch(lanes_per_lookup, lookups_per_lane, block, blocks_per_cu)
        _check(self.lib.ckpp_set_lookup_launch(self._h, ctypes.byref(cfg)),
               "ckpp_set_lookup_launch")

    def get_lookup_launch(self) -> dict:
        cfg = _Launch()
        _check(self.lib.ckpp_get_lookup_launch(self._h, ctypes.byref(cfg)),
               "ckpp_get_lookup_launch")
        return {f: getattr(cfg, f) for f, _ in _Launch._fields_}


class Plan:
    """Lookup batches of many tables served by one persistent launch (see
    ckpp_plan_create in include/ckpp.h).  ``offsets[i]``/``counts[i]`` place
    table i's batch in the concatenated key array; ``modes`` (names or
    numbers, default Cuckoo++) gives each table's lookup mode."""

    def __init__(self, tables, offsets, counts, modes=None):
        self.lib = load()
        self.tables = list(tables)  # kept alive for the plan's lifetime
        nt = len(self.tables)
        handles = (ctypes.c_void_p * nt)(*[t.handle for t in self.tables])
        off = np.ascontiguousarray(offsets, dtype=np.uint64)
        cnt = np.ascontiguousarray(counts, dtype=np.uint64)
        if off.size != nt or cnt.size != nt:
            raise CkppError("one offset and one count per table")
        md = None
        if modes is not None:
            md = np.ascontiguousarray([MODES[m] if isinstance(m, str) else int(m) for m in modes],
                                      dtype=np.uint32)
            if md.size != nt:
                raise CkppError("one mode per table")
        h = ctypes.c_void_p()
        rc = self.lib.ckpp_plan_create(ctypes.byref(h), handles, nt, off.ctypes.data,
                                       cnt.ctypes.data, md.ctypes.data if md is not None else None)
        _check(rc, "ckpp_plan_create")
        self._h = h
        self.device = self.tables[0].device
        self.key_span = self.info()["key_span"]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.ckpp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def lookup(self, keys, found=None, values=None, stream=None, now=None, refresh=None):
        """Enqueues the plan's lookups; returns (found u8[span], values i64[span]).
        A plan with tables with timers runs at time `now` (required), and with
        `refresh` (a u16 time) every entry found on them gets that expiration
        time."""
        torch = _torch()
        kp, n = _keys_ptr(keys)
        if n < self.key_span:
            raise CkppError(f"the plan reads {self.key_span} keys, got {n}")
        dev = torch.device("cuda", self.device)
        if found is None:
            found = torch.zeros(self.key_span, dtype=torch.uint8, device=dev)
        if values is None:
            values = torch.zeros(self.key_span, dtype=torch.int64, device=dev)
        if found.numel() < self.key_span or values.numel() < self.key_span:
            raise CkppError("output arrays shorter than the plan's key span")
        if now is None:
            rc = self.lib.ckpp_plan_lookup(self._h, kp, found.data_ptr(), values.data_ptr(),
                                           _stream_handle(stream))
            _check(rc, "ckpp_plan_lookup")
        else:
            rc = self.lib.ckpp_plan_lookup_at(self._h, kp, found.data_ptr(), values.data_ptr(),
                                              int(now) & 0xFFFF, 0 if refresh is None else 1,
                                              0 if refresh is None else int(refresh) & 0xFFFF,
                                              _stream_handle(stream))
            _check(rc, "ckpp_plan_lookup_at")
        return found, values

    def set_launch(self, lookups_per_lane=DEFAULT_PLAN_LAUNCH["lookups_per_lane"],
                   block=DEFAULT_PLAN_LAUNCH["block"],
                   blocks_per_cu=DEFAULT_PLAN_LAUNCH["blocks_per_cu"],
                   passes_per_item=DEFAULT_PLAN_LAUNCH["passes_per_item"],
                   schedule=DEFAULT_PLAN_LAUNCH["schedule"],
                   lanes_per_lookup=DEFAULT_PLAN_LAUNCH["lanes_per_lookup"]):
        cfg = _PlanLaunch(lookups_per_lane, block, blocks_per_cu, passes_per_item, schedule,
                          lanes_per_lookup)
        _check(self.lib.ckpp_plan_set_launch(self._h, ctypes.byref(cfg)), "ckpp_plan_set_launch")

    def get_launch(self) -> dict:
        cfg = _PlanLaunch()
        _check(self.lib.ckpp_plan_get_launch(self._h, ctypes.byref(cfg)), "ckpp_plan_get_launch")
        return {f: getattr(cfg, f) for f, _ in _PlanLaunch._fields_}

    def info(self) -> dict:
        inf = _PlanInfo()
        _check(self.lib.ckpp_plan_info(self._h, ctypes.byref(inf)), "ckpp_plan_info")
        return {f: getattr(inf, f) for f, _ in _PlanInfo._fields_}


class Server:
    """A device-resident serving loop over one table (see ckpp_server_create
    in include/ckpp.h).  ``put`` copies a burst's operations into the rings
    at the next positions, ``submit`` hands the burst to the loop, ``get``
    copies results out once the burst is complete."""

    KINDS = {"lookup": 0, "insert": 1, "delete": 2}

    def __init__(self, table, capacity=1 << 20, budget=None, mode="cuckoopp", blocks_per_cu=1,
                 idle_ms=200, ttl=0, refresh=False):
        """ttl / refresh: tables with timers only (the entry lifetime, and
        whether lookups that find an entry renew it)."""
        self.lib = load()
        self.table = table
        cfg = _ServerConfig(int(capacity), int(budget or capacity),
                            MODES[mode] if isinstance(mode, str) else int(mode),
                            int(blocks_per_cu), int(idle_ms),
                            int(ttl) | (SERVER_REFRESH if refresh else 0))
        h = ctypes.c_void_p()
        _check(self.lib.ckpp_server_create(ctypes.byref(h), table.handle, ctypes.byref(cfg)),
               "ckpp_server_create")
        self._h = h
        r = _ServerRings()
        _check(self.lib.ckpp_server_rings(self._h, ctypes.byref(r)), "ckpp_server_rings")
        self.capacity = int(r.capacity)
        self._stage = [0, 0, 0]  # op numbers where put_burst stages next

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.ckpp_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def status(self) -> dict:
        st = _ServerStatus()
        _check(self.lib.ckpp_server_status(self._h, ctypes.byref(st)), "ckpp_server_status")
        return {f: int(getattr(st, f)) for f, _ in _ServerStatus._fields_}

    def put(self, kind: str, pos: int, keys, values=None, stream=None):
        """Copies ops (device tensors) into the ring slots of op numbers
        pos .. pos + n - 1 of a kind, then waits for the copies."""
        kp, n = _keys_ptr(keys)
        vp = None
        if values is not None:
            if values.numel() != n or values.element_size() != 8 or not values.is_contiguous():
                raise CkppError("values must be n contiguous 64-bit integers")
            vp = values.data_ptr()
        torch = _torch()
        if stream is None:
            stream = torch.cuda.current_stream(self.table.device)
        _check(self.lib.ckpp_server_put(self._h, self.KINDS[kind], int(pos), kp, vp, n,
                                        _stream_handle(stream)), "ckpp_server_put")
        stream.synchronize()

    def put_burst(self, lookup_keys=None, insert_keys=None, insert_values=None,
                  delete_keys=None):
        """Stages one burst's operations after those already staged or
        submitted (bursts may be staged ahead of their submission, in
        submission order, as long as they fit the rings); returns the counts
        for submit() and the first op number of each kind."""
        st = self.status()
        counts, first = [], []
        for k, (kind, keys, vals) in enumerate((("lookup", lookup_keys, None),
                                                ("insert", insert_keys, insert_values),
                                                ("delete", delete_keys, None))):
            n = 0 if keys is None else int(keys.shape[0])
            pos = max(self._stage[k], st[f"{kind}_tail"])
            if n:
                self.put(kind, pos, keys, vals)
            self._stage[k] = pos + n
            counts.append(n)
            first.append(pos)
        return counts, first

    def submit(self, n_lookup, n_insert=0, n_delete=0):
        """Returns the burst number, or None when the budget does not admit it."""
        b = ctypes.c_uint64()
        rc = self.lib.ckpp_server_submit(self._h, int(n_lookup), int(n_insert), int(n_delete),
                                         ctypes.byref(b))
        if rc == EBUSY:
            return None
        _check(rc, "ckpp_server_submit")
        return int(b.value)

    def set_time(self, now):
        """Time of the bursts submitted from now on (tables with timers);
        False when the burst that carries a due scan is not admitted yet."""
        rc = self.lib.ckpp_server_set_time(self._h, int(now) & 0xffff)
        if rc == EBUSY:
            return False
        _check(rc, "ckpp_server_set_time")
        return True

    def wait(self, burst, timeout_ms=10000):
        _check(self.lib.ckpp_server_wait(self._h, int(burst), int(timeout_ms)), "ckpp_server_wait")

    def get(self, kind: str, pos: int, n: int, stream=None):
        """Results of ops pos .. pos + n - 1 of a kind: (found, values) for
        lookups, status for inserts, found for deletes (device tensors,
        ready once the stream is synchronized)."""
        torch = _torch()
        dev = torch.device("cuda", self.table.device)
        flags = torch.empty(int(n), dtype=torch.uint8, device=dev)
        vals = torch.empty(int(n), dtype=torch.int64, device=dev) if kind == "lookup" else None
        _check(self.lib.ckpp_server_get(self._h, self.KINDS[kind], int(pos), int(n),
                                        flags.data_ptr(), vals.data_ptr() if vals is not None
                                        else None, _stream_handle(stream)), "ckpp_server_get")
        return (flags, vals) if kind == "lookup" else flags

    def replay(self, nlookup, ninsert, ndelete, arrival_s, timeout_s=60.0):
        """Open-loop replay of a pre-staged stream; returns (admit_s, done_s)."""
        n = len(arrival_s)
        nl = np.ascontiguousarray(nlookup, dtype=np.uint32)
        ni = np.ascontiguousarray(ninsert, dtype=np.uint32)
        nd = np.ascontiguousarray(ndelete, dtype=np.uint32)
        ar = np.ascontiguousarray(arrival_s, dtype=np.float64)
        adm = np.zeros(n, np.float64)
        done = np.zeros(n, np.float64)
        _check(self.lib.ckpp_server_replay(self._h, n, nl.ctypes.data, ni.ctypes.data,
                                           nd.ctypes.data, ar.ctypes.data, adm.ctypes.data,
                                           done.ctypes.data, float(timeout_s)),
               "ckpp_server_replay")
        return adm, done


def probe_random_reads(buf, granule: int, nreads: int, per_lane: int, block: int, grid: int,
                       seed: int, sink, cooperative: bool = False, stream=None):
    """Launches the random-read probe over the device tensor ``buf``."""
    lib = load()
    nbytes = buf.numel() * buf.element_size()
    rc = lib.ckpp_probe_random_reads(buf.data_ptr(), nbytes, granule, nreads, per_lane,
                                     1 if cooperative else 0, block, grid,
                                     ctypes.c_uint64(seed), sink.data_ptr(),
                                     _stream_handle(stream))
    _check(rc, "ckpp_probe_random_reads")


LATENCY_KINDS = ("load", "atomic_load", "cas", "load_store_wait", "cas_pair", "load_batch32",
                 "atomic_load_batch32")


def probe_latency(buf, kind: str, steps: int, seed: int, out, stream=None):
    """Launches the dependent-access latency probe over the device tensor
    ``buf`` (kinds: LATENCY_KINDS); ``out`` (two int64) receives the elapsed
    10 ns ticks and a fold of the values read."""
    lib = load()
    nbytes = buf.numel() * buf.element_size()
    rc = lib.ckpp_probe_latency(buf.data_ptr(), nbytes, LATENCY_KINDS.index(kind), int(steps),
                                ctypes.c_uint64(seed), out.data_ptr(), _stream_handle(stream))
    _check(rc, "ckpp_probe_latency")
