"""The C ABI library loads on a machine without a GPU and exports every
entry point include/ckpp.h declares; the binding covers each of them and its
structures match the header's (checked by compiling the header with gcc).
No compute call is made here."""

import ctypes
import os
import re
import subprocess
import tempfile

import pytest

from paper_1712_09624_amd import ckpp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ckpp.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ckpp_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(ckpp.LIB_PATH):
        from paper_1712_09624_amd import build
        build.build()
    return ckpp.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ckpp_create", "ckpp_insert_batch", "ckpp_lookup_batch",
                     "ckpp_delete_batch", "ckpp_destroy"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} declared in ckpp.h but not exported"


def test_binding_covers_every_declared_symbol():
    bound = {s[0] for s in ckpp.SIGNATURES}
    assert set(declared_functions()) == bound


def test_strerror_needs_no_device(lib):
    assert lib.ckpp_strerror(0) == b"ok"
    assert lib.ckpp_strerror(1) == b"invalid argument"


def test_argument_checks_need_no_device(lib):
    # invalid arguments are rejected before any device work
    h = ctypes.c_void_p()
    assert lib.ckpp_create(None, 10, 1, 500, 0, 0) == ckpp.EINVAL
    assert lib.ckpp_create(ctypes.byref(h), 0, 1, 500, 0, 0) == ckpp.EINVAL
    assert lib.ckpp_create(ctypes.byref(h), 30, 1, 500, 0, 0) == ckpp.EINVAL
    assert lib.ckpp_create(ctypes.byref(h), 10, 1, 500, 4, 0) == ckpp.EINVAL
    assert lib.ckpp_insert_batch(None, None, None, 5, None, None, None) == ckpp.EINVAL
    assert lib.ckpp_lookup_batch(None, None, 5, 0, None, None, None) == ckpp.EINVAL
    assert lib.ckpp_delete_batch(None, None, 5, None, None) == ckpp.EINVAL
    assert lib.ckpp_insert_batch_at(None, None, None, None, 5, 0, None, None, None) == ckpp.EINVAL
    assert lib.ckpp_lookup_batch_at(None, None, 5, 0, 0, 0, 0, None, None, None) == ckpp.EINVAL
    assert lib.ckpp_delete_batch_at(None, None, 5, 0, None, None) == ckpp.EINVAL
    assert lib.ckpp_expire_scan(None, 0, None, None) == ckpp.EINVAL
    assert lib.ckpp_set_lookup_launch(None, None) == ckpp.EINVAL
    assert lib.ckpp_set_retry_limit(None, 5) == ckpp.EINVAL
    assert lib.ckpp_get_retry_limit(None, None) == ckpp.EINVAL
    assert lib.ckpp_check_image(10, 0, None, None) == ckpp.EINVAL
    assert lib.ckpp_destroy(None) == ckpp.OK
    assert lib.ckpp_probe_random_reads(None, 64, 64, 1, 1, 0, 256, 1, 0, None, None) == ckpp.EINVAL
    assert lib.ckpp_probe_latency(None, 256, 0, 1, 0, None, None) == ckpp.EINVAL
    offs = (ctypes.c_uint64 * 1)(0)
    cnts = (ctypes.c_uint64 * 1)(1)
    tabs = (ctypes.c_void_p * 1)(None)
    assert lib.ckpp_plan_create(None, tabs, 1, offs, cnts, None) == ckpp.EINVAL
    assert lib.ckpp_plan_create(ctypes.byref(h), None, 1, offs, cnts, None) == ckpp.EINVAL
    assert lib.ckpp_plan_create(ctypes.byref(h), tabs, 0, offs, cnts, None) == ckpp.EINVAL
    assert lib.ckpp_plan_create(ctypes.byref(h), tabs, 1, offs, cnts, None) == ckpp.EINVAL
    assert lib.ckpp_plan_lookup(None, None, None, None, None) == ckpp.EINVAL
    assert lib.ckpp_plan_lookup_at(None, None, None, None, 0, 0, 0, None) == ckpp.EINVAL
    assert lib.ckpp_plan_set_launch(None, None) == ckpp.EINVAL
    assert lib.ckpp_plan_destroy(None) == ckpp.OK
    assert lib.ckpp_server_create(None, None, None) == ckpp.EINVAL
    assert lib.ckpp_server_submit(None, 1, 0, 0, None) == ckpp.EINVAL
    assert lib.ckpp_server_put(None, 0, 0, None, None, 1, None) == ckpp.EINVAL
    assert lib.ckpp_server_set_time(None, 0) == ckpp.EINVAL
    assert lib.ckpp_server_destroy(None) == ckpp.OK


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(ckpp.CkppError):
        ckpp.load(str(tmp_path / "absent.so"))


def test_struct_layouts_match_header():
    prog = r"""
#include <stdio.h>
#include <stddef.h>
#include "ckpp.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(ckpp_stats_t),
         offsetof(ckpp_stats_t, moved_hist), sizeof(ckpp_info_t), sizeof(ckpp_launch_t),
         sizeof(ckpp_plan_launch_t), sizeof(ckpp_plan_info_t), offsetof(ckpp_plan_info_t, key_span),
         sizeof(ckpp_server_config_t), sizeof(ckpp_server_rings_t), sizeof(ckpp_server_status_t),
         offsetof(ckpp_server_status_t, lookup_ns));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(prog)
        subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), "-o", exe, c],
                       check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    (sz_stats, off_hist, sz_info, sz_launch, sz_pl, sz_pi, off_span, sz_sc, sz_sr, sz_ss,
     off_lns) = map(int, out)
    assert sz_stats == ctypes.sizeof(ckpp._Stats)
    assert off_hist == ckpp._Stats.moved_hist.offset
    assert sz_info == ctypes.sizeof(ckpp._Info)
    assert sz_launch == ctypes.sizeof(ckpp._Launch)
    assert sz_pl == ctypes.sizeof(ckpp._PlanLaunch)
    assert sz_pi == ctypes.sizeof(ckpp._PlanInfo)
    assert off_span == ckpp._PlanInfo.key_span.offset
    assert sz_sc == ctypes.sizeof(ckpp._ServerConfig)
    assert sz_sr == ctypes.sizeof(ckpp._ServerRings)
    assert sz_ss == ctypes.sizeof(ckpp._ServerStatus)
    assert off_lns == ckpp._ServerStatus.lookup_ns.offset


def test_check_image_rejects_wild_images(lib):
    """ckpp_check_image (the check ckpp_import applies, host-only): an image
    the oracle built is accepted; a lock word left set, a sec bit outside
    busy, an occupied slot whose other bucket lies outside the table, and on
    a table with timers an occupied slot's value of 2^48 or more or a
    reserved word above 16 bits are refused; a wide value in a free slot is
    not looked at."""
    import numpy as np
    from oracle import oracle as O
    from paper_1712_09624_amd import workload as W
    B = 6
    n = W.keys_at_load(B, 0.8)
    keys = W.distinct_five_tuples(n, 11)
    for timed in (False, True):
        ref = O.OracleTable(B, W.HASH_SEED, W.MAX_KICKS, timed=timed)
        if timed:
            ref.insert_at(keys, W.insertion_values(n), np.full(n, 300, np.uint16), 0)
        else:
            ref.insert(keys, W.insertion_values(n))
        b, k = ref.image()
        assert ckpp.check_image(B, b, k, timers=timed)
        bk = b.reshape(-1, 64)
        rec = k.reshape(-1, 32)
        busy = bk[:, 26]
        bb = int(np.flatnonzero(busy)[0])
        s0 = int(np.flatnonzero([(busy[bb] >> i) & 1 for i in range(8)])[0])

        def refused(bm=None, km=None):
            b2, k2 = bk.copy(), rec.copy()
            if bm:
                bm(b2)
            if km:
                km(k2)
            return not ckpp.check_image(B, b2, k2, timers=timed)

        assert refused(bm=lambda x: x.__setitem__((bb, 29), 1))               # lock word
        free = int(np.flatnonzero(busy != 0xFF)[0])
        fslot = int(next(i for i in range(8) if not (busy[free] >> i) & 1))
        assert refused(bm=lambda x: x.__setitem__((free, 27), x[free, 27] | (1 << fslot)))
        big = np.frombuffer(np.uint32(1 << B).tobytes(), np.uint8)
        assert refused(bm=lambda x: x.__setitem__((bb, slice(32 + 4 * s0, 36 + 4 * s0)), big))
        if timed:
            r = bb * 8 + s0
            assert refused(km=lambda x: x.__setitem__((r, 23), 1))            # value >= 2^56
            assert refused(km=lambda x: x.__setitem__((r, 26), 1))            # time >= 2^16
            fr = free * 8 + fslot
            k3 = rec.copy()
            k3[fr, 23] = 0x80
            assert ckpp.check_image(B, bk, k3, timers=True)
