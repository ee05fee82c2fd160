"""Benchmark of the Cuckoo++ hot path on one MI355X.

A step is one pass of the whole path over one batch of synthetic input, on a
2^24-bucket x 8-slot table (134M slots, ~5 GiB of buckets and records,
HBM-resident) filled to load 0.9:
    insert_batch  65536 fresh keys (churn)
    lookup_batch  2^26 positive lookups   (Cuckoo++)
    lookup_batch  2^26 negative lookups   (Cuckoo++)
    delete_batch  the 65536 churn keys    (load back to 0.9)
value = lookups per second over the timed steps (Glookups/s), inputs resident
in device memory.  Around it (untimed): the plain-cuckoo and optimistic
lookups on the same table, a 2^20-bucket table (cache-resident bucket array),
the random-read line rate of the device (the lookups' roofline), single
burst latencies, and the oracle timed on the host.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1712_09624_amd import workload as W  # noqa: E402

METRIC = "Glookups/s @load 0.9 (pos & neg), % random-64B HBM peak; p99 burst latency"
HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth
LINE = 128  # bytes of one bucket line (half of a 256-byte device bucket)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2-buckets", type=int, default=24)
    ap.add_argument("--load", type=float, default=0.9)
    ap.add_argument("--lookups", type=int, default=1 << 26)
    ap.add_argument("--churn", type=int, default=65536)
    ap.add_argument("--core-only", action="store_true",
                    help="only the timed steps (for profiler runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency", action="store_true",
                    help="latency of one dependent access of each kind the updates make")
    ap.add_argument("--burst-latency", action="store_true",
                    help="only the burst-latency leg (plain calls and the serving loop)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run only a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--sweep", action="store_true",
                    help="lookup rate over loads x negative rates x modes (2^24 and 2^20 buckets)")
    ap.add_argument("--serve", type=int, default=0, metavar="BURSTS",
                    help="serving workload, BURSTS bursts per run: peak, then 25/50/75/100%% offered")
    ap.add_argument("--serve-log2-buckets", type=int, default=24,
                    help="with --serve: table size (2^B buckets; the table must hold more keys "
                         "than the 100M-flow universe, for the deletes)")
    ap.add_argument("--serve-load", type=float, default=0.85, help="with --serve: table load")
    ap.add_argument("--serve-blocks-per-cu", type=int, default=1,
                    help="with --serve: blocks of the loop kernel per compute unit (1..4)")
    ap.add_argument("--serve-timers", action="store_true",
                    help="with --serve: the table has timers (lookups renew entries; the loop "
                         "runs the anti-revival scan)")
    ap.add_argument("--many-tables", type=int, default=0, metavar="N",
                    help="batching workload over N tables: per-table calls vs one plan launch")
    ap.add_argument("--plan-shape", default=None, metavar="L,P,B,C,I,S",
                    help="with --many-tables: only the plan at this shape (lanes per lookup, "
                         "lookups per lane, block, blocks per CU, passes per item, schedule)")
    ap.add_argument("--insert-workload", action="store_true",
                    help="insert rate vs load in 65536-key batches, then delete 20%% and re-insert")
    ap.add_argument("--summarize-profiles", metavar="DIR", default=None,
                    help="write profiles/ summaries from rocprofv3 CSV output under DIR")
    ap.add_argument("--summarize-serve", metavar="JSON", default=None,
                    help="write the serving summary in profiles/ from a saved --serve 50000 line")
    ap.add_argument("--summarize-serve-trace", metavar="DIR", default=None,
                    help="with --summarize-serve: rocprofv3 output of the loop's kernel trace")
    ap.add_argument("--summarize-serve-counters", metavar="DIR", default=None,
                    help="with --summarize-serve: rocprofv3 --pmc output of the loop "
                         "(DIR/serve_a, DIR/serve_b) and the copy calibration (DIR/p4_copy_*)")
    ap.add_argument("--summarize-serve-timers", metavar="JSON", default=None,
                    help="write the timed serving summary in profiles/ from a saved "
                         "--serve 50000 --serve-timers line")
    ap.add_argument("--summarize-many-tables", metavar="JSON", default=None,
                    help="write the many-table batching summary in profiles/ from a saved "
                         "--many-tables 1024 line")
    ap.add_argument("--summarize-latency", metavar="JSON", default=None,
                    help="write the latency probe summary in profiles/ from a saved --latency line")
    ap.add_argument("--summarize-insert-workload", metavar="JSON", default=None,
                    help="write the insert workload summary in profiles/ from a saved "
                         "--insert-workload line")
    ap.add_argument("--summarize-plan-profiles", metavar="DIR", default=None,
                    help="write the plan kernel's profiles/ summary from rocprofv3 CSV output "
                         "under DIR")
    ap.add_argument("--tune", action="store_true",
                    help="time every lookup launch shape, print them, keep the fastest")
    ap.add_argument("--lanes", type=int, default=None)
    ap.add_argument("--per-lane", type=int, default=None)
    ap.add_argument("--block", type=int, default=None)
    ap.add_argument("--blocks-per-cu", type=int, default=None)
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def to_dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def lookup_source_digest() -> str:
    h = hashlib.sha256()
    for f in ("ckpp_lookup.hip", "ckpp_lookup_dev.h", "ckpp_device.h"):
        with open(os.path.join(ROOT, "paper_1712_09624_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def expected_lines(stats: dict) -> dict:
    """Algorithmic 128-byte lines read per lookup (Sec. 2 and 4.1 on the
    device layout: a bucket's first line holds its metadata and slots 0..3,
    its second line slots 4..7).  A positive Cuckoo++ lookup reads the first
    line of its primary bucket, plus the second line when the key sits in a
    slot 4..7, plus the secondary bucket's line(s) when the key was displaced
    there: per key 1 + f_high + f_sec, f_high = share of entries in slots
    4..7, f_sec = share in their secondary bucket.  A negative Cuckoo++
    lookup reads one line, plus a line of the secondary when the filter
    passes (rate FPR).  A busy slot 4..7 whose tag matches by chance
    (2^-16 per slot) costs one more line.  The pessimistic lookup reads the
    first lines of both buckets always; the optimistic one reads the
    secondary whenever the key is not in the primary."""
    nb, live = stats["nbuckets"], max(1, stats["live"])
    f_sec, fpr = stats["f_sec"], stats["expected_fpr"]
    f_high = stats["high_slots"] / live
    eps = (stats["high_slots"] / nb) / 65536.0  # false tag matches in slots 4..7 per bucket
    return {
        "cuckoopp_pos": 1.0 + f_high + f_sec + eps * f_sec,
        "cuckoopp_neg": 1.0 + fpr + eps * (1.0 + fpr),
        "plain_pos": 2.0 + f_high + eps,
        "plain_neg": 2.0 + 2.0 * eps,
        "optimistic_pos": 1.0 + f_high + f_sec + eps * f_sec,
        "optimistic_neg": 2.0 + 2.0 * eps,
    }


STREAM_BYTES = 16 + 1 + 8  # key in, found + value out, per lookup
ALG_LINE = 64  # the method's unit of memory access: a 64-byte cache line


def algorithmic_lines_64(stats: dict) -> dict:
    """Lines of 64 bytes a lookup must touch in the paper's layout (a 64-byte
    bucket line, and a separate 32-byte key/value record, Sec. 4.3), the
    unit of the roofline's algorithmic bytes: a positive Cuckoo++ lookup
    reads its primary bucket and the record of its key, plus the secondary
    bucket when the key was displaced there (f_sec), 2 + f_sec; a negative
    one reads its primary bucket, plus the secondary when the filter passes
    (FPR), 1 + FPR (Sec. 4.1).  Each probed bucket adds a record read per
    false 16-bit tag match, eps = (busy slots per bucket) * 2^-16.  The
    pessimistic lookup always reads both buckets: 3 + eps positive, 2 + 2 eps
    negative; the optimistic one reads the secondary whenever the key is not
    in the primary."""
    nb, live = stats["nbuckets"], max(1, stats["live"])
    f_sec, fpr = stats["f_sec"], stats["expected_fpr"]
    eps = (live / nb) / 65536.0
    return {
        "cuckoopp_pos": 2.0 + f_sec + eps * (1.0 + f_sec),
        "cuckoopp_neg": 1.0 + fpr + eps * (1.0 + fpr),
        "plain_pos": 3.0 + eps,
        "plain_neg": 2.0 + 2.0 * eps,
        "optimistic_pos": 2.0 + f_sec + eps * (1.0 + f_sec),
        "optimistic_neg": 2.0 + 2.0 * eps,
    }


def build_table(B, load, seed, dev, batch=1 << 22, expiry=None, now=0):
    """A table of 2^B buckets filled to `load` with the keys of workload
    `seed` (values = insertion index); with `expiry` (one u16 time per key)
    a table with timers, built at time `now`."""
    import torch
    from paper_1712_09624_amd.ckpp import Table
    n = W.keys_at_load(B, load)
    log(f"generating {n} keys for 2^{B} buckets at load {load}")
    keys = W.distinct_five_tuples(n, seed)
    vals = W.insertion_values(n)
    t = Table(B, W.HASH_SEED, W.MAX_KICKS, device=dev.index, timers=expiry is not None)
    nfail = torch.zeros(1, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(0, n, batch):
        dk = to_dev(keys[s:s + batch], dev)
        dv = to_dev(vals[s:s + batch].view(np.int64), dev)
        if expiry is None:
            t.insert(dk, dv, nfailed=nfail)
        else:
            de = to_dev(expiry[s:s + batch].view(np.int16), dev)
            t.insert_at(dk, dv, de, now, nfailed=nfail)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    nf = int(nfail.item())
    if nf:
        raise RuntimeError(f"{nf} inserts failed while building the table")
    log(f"built in {dt:.2f}s ({n / dt / 1e6:.0f} M inserts/s incl. transfers)")
    return t, keys, vals, dt


def timed(fn, reps, dev):
    """Mean ms of fn() measured with events on the current stream."""
    import torch
    s = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    fn()
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def probe_rand_peak(dev, gib=8, nreads=1 << 26):
    """Measured random-read rate: aligned 32/64/128-byte reads at uniformly
    random positions of a buffer far larger than every cache, read either by
    one lane (16-byte loads) or cooperatively (one 16-byte piece per lane,
    one coalesced request per granule); several reads in flight per lane;
    best launch shape per granule and form."""
    import torch
    from paper_1712_09624_amd import ckpp
    nbytes = gib << 30
    buf = torch.empty(nbytes // 8, dtype=torch.int64, device=dev)
    ncu = torch.cuda.get_device_properties(dev).multi_processor_count
    best = {}
    for coop in (False, True):
        for granule in (32, 64, 128):
            rates = []
            for per_lane in (2, 4, 8):
                for bpc in (8, 16):
                    grid = ncu * bpc
                    sink = torch.empty(grid * 256, dtype=torch.int64, device=dev)
                    ms = timed(lambda: ckpp.probe_random_reads(buf, granule, nreads, per_lane, 256,
                                                               grid, 12345, sink, coop), 3, dev)
                    rates.append((nreads / (ms * 1e-3), per_lane, bpc))
            r = max(rates)
            key = f"{granule}{'_coop' if coop else '_lane'}"
            best[key] = {"reads_per_s": r[0], "GBps": r[0] * granule / 1e9,
                         "per_lane": r[1], "blocks_per_cu": r[2]}
            log(f"random {key} reads: {r[0] / 1e9:.2f} G/s = {r[0] * granule / 1e9:.0f} GB/s")
    del buf
    torch.cuda.empty_cache()
    return best


def probe_line_peak(dev, nbytes, nreads=1 << 26):
    """Measured rate of random 128-byte line reads (cooperative, the lookups'
    request shape) at uniformly random positions of a buffer of nbytes;
    best launch shape.  On a buffer the size of a table it is that table's
    random-line ceiling: HBM for 4 GiB, the last-level cache (256 MiB) for
    tables that fit it."""
    import torch
    from paper_1712_09624_amd import ckpp
    buf = torch.empty(nbytes // 8, dtype=torch.int64, device=dev)
    buf.zero_()
    ncu = torch.cuda.get_device_properties(dev).multi_processor_count
    best = 0.0
    for per_lane in (4, 8):
        for bpc in (8, 16):
            grid = ncu * bpc
            sink = torch.empty(grid * 256, dtype=torch.int64, device=dev)
            ms = timed(lambda: ckpp.probe_random_reads(buf, 128, nreads, per_lane, 256, grid,
                                                       12345, sink, True), 3, dev)
            best = max(best, nreads / (ms * 1e-3))
    del buf
    torch.cuda.empty_cache()
    return best


def cache_resident_table(dev, lookups, B=20):
    """A table of 2^B buckets at load 0.9 whose buckets fit the 256 MiB
    last-level cache (B = 20: 256 MiB, the cache's size, so only partly
    resident; B = 19: 128 MiB), with its own random-line ceiling measured on
    a buffer of the table's size."""
    import torch
    t, keys, _, _ = build_table(B, 0.9, 77, dev)
    n = lookups
    pos, _, _ = W.lookup_mix(keys, n, 0.0, 78)
    neg = W.five_tuples(n, 79, stream=W.STREAM_NEGATIVE)
    dp, dn = to_dev(pos, dev), to_dev(neg, dev)
    f = torch.empty(n, dtype=torch.uint8, device=dev)
    v = torch.empty(n, dtype=torch.int64, device=dev)
    out = {"log2_buckets": B, "load": 0.9, "lookups": n, "table_bytes": 256 << B}
    st = t.stats()
    out["f_sec"] = st["f_sec"]
    lines = expected_lines(st)
    out["random_line_peak_same_size_per_s"] = peak = probe_line_peak(dev, 256 << B)
    for mode, lk in (("cuckoopp", "cuckoopp"), ("both", "plain")):
        for name, d in (("pos", dp), ("neg", dn)):
            ms = timed(lambda: t.lookup(d, mode, found=f, values=v), 5, dev)
            rate = n / (ms * 1e-3)
            out[f"{mode}_{name}_glookups"] = rate / 1e9
            out[f"{mode}_{name}_frac_same_size_peak"] = rate * lines[f"{lk}_{name}"] / peak
    t.close()
    return out


def timers_leg(dev, B, load, n, dpos, dneg, pos_idx, untimed):
    """Tables with timers (Sec. 4.2) on the same workload: the table is built
    with expiration times uniform over the 1024 units after now0, and the
    positive and negative lookup batches are timed at now0 (every entry
    alive: the answers equal those of the table without timers, so the time
    difference is the overhead of the timer check), at now0 + 512 (about
    half the entries expired), and at now0 + 512 with a refresh of every
    entry found (each timed call sets a time other than the previous call's,
    so every hit writes; then once more with the time the entries already
    hold, which writes nothing).  Then the anti-revival scan over the whole
    table once every entry has expired.  Answers are checked on a sample: found iff the key's
    entry is alive, value = insertion index."""
    import torch
    now0 = 65000
    nkeys = W.keys_at_load(B, load)
    exp = W.times_after(nkeys, now0, 1024, 1)
    t, keys, vals, build_s = build_table(B, load, 1, dev, expiry=exp, now=now0)
    f = torch.empty(n, dtype=torch.uint8, device=dev)
    v = torch.empty(n, dtype=torch.int64, device=dev)
    out = {"log2_buckets": B, "load": load, "lookups": n, "build_s": build_s,
           "expiry": "uniform over [now0, now0 + 1023], now0 = 65000 (the window wraps)"}
    chk = np.arange(0, n, max(1, n // 65536))
    # the anti-revival scan at now0, when every entry is alive: a read of the
    # whole table that removes nothing
    removed0 = torch.zeros(1, dtype=torch.int64, device=dev)
    out["scan_nothing_ms"] = timed(lambda: t.expire_scan(now0, removed=removed0), 3, dev)
    if int(removed0.item()) != 0:
        raise RuntimeError("the scan removed entries that were alive")
    half = (now0 + 512) & 0xFFFF
    for label, now, refresh in (("", now0, None), ("half_expired_", half, None),
                                ("refresh_", half, (half + 1023) & 0xFFFF)):
        for name, d in (("pos", dpos), ("neg", dneg)):
            last = [refresh]

            def run():
                if refresh is not None:
                    # alternate between two times in the window
                    last[0] = (refresh - 1) & 0xFFFF if last[0] == refresh else refresh
                t.lookup_at(d, now, found=f, values=v, refresh=last[0])

            ms = timed(run, 5, dev)
            out[f"{label}{name}_glookups"] = n / (ms * 1e-3) / 1e9
            if refresh is not None and name == "pos":
                ms = timed(lambda: t.lookup_at(d, now, found=f, values=v, refresh=last[0]), 5,
                           dev)
                out["refresh_unchanged_pos_glookups"] = n / (ms * 1e-3) / 1e9
            fo = f.cpu().numpy()[chk]
            if name == "neg":
                ok = not fo.any()
            else:
                # a refresh keeps alive what it finds, so the answers stay
                # those of the times before it
                e = exp[pos_idx[chk]].astype(np.int64)
                want = (((e - now) & 0xFFFF) < 1024).astype(np.uint8)
                vo = v.cpu().numpy().view(np.uint64)[chk]
                ok = np.array_equal(fo, want) and np.array_equal(
                    vo[want == 1], vals[pos_idx[chk]][want == 1])
                if refresh is not None:
                    found_rows = np.unique(pos_idx[f.cpu().numpy() == 1])
                    exp[found_rows] = last[0]
            if not ok:
                raise RuntimeError(f"timed lookups ({label}{name}) returned a wrong answer")
    for name in ("pos", "neg"):
        out[f"overhead_{name}"] = untimed[f"cuckoopp_{name}_glookups"] / out[f"{name}_glookups"] - 1
    removed = torch.zeros(1, dtype=torch.int64, device=dev)
    later = (half + 2000) & 0xFFFF
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    t.expire_scan(later, removed=removed)
    e1.record()
    e1.synchronize()
    out["scan_ms"] = e0.elapsed_time(e1)
    out["scan_removed"] = int(removed.item())
    out["scan_table_GBps"] = (256 << B) / (out["scan_ms"] * 1e-3) / 1e9
    if t.stats()["live"] != 0 or out["scan_removed"] != nkeys:
        raise RuntimeError("the scan did not remove every expired entry")
    t.close()
    return out


def burst_latency(dev, keys, B=24, load=0.85, nbursts=10_000, neg_rate=0.5, warm=100):
    """Single-kernel burst latency on a 2^B-bucket table at `load`: nbursts
    synchronous lookup_batch calls, burst sizes log-uniform in [1, 2048]
    (the serving workload's burst-size law), each lookup of a burst
    independently negative with probability neg_rate (positives uniform over
    the stored keys); p50/p99 of submit -> completion on the host clock.
    The table holds the first keys_at_load(B, load) keys of `keys` (the
    benchmark's key stream).  The first `warm` bursts are not counted."""
    import torch
    n = W.keys_at_load(B, load)
    from paper_1712_09624_amd.ckpp import Table
    t = Table(B, W.HASH_SEED, W.MAX_KICKS, device=dev.index)
    nfail = torch.zeros(1, dtype=torch.int64, device=dev)
    for s0 in range(0, n, 1 << 22):
        s1 = min(n, s0 + (1 << 22))
        t.insert(to_dev(keys[s0:s1], dev),
                 to_dev(W.insertion_values(s1 - s0, s0).view(np.int64), dev), nfailed=nfail)
    torch.cuda.synchronize()
    if int(nfail.item()):
        raise RuntimeError("inserts failed while building the burst-latency table")
    sizes = W.log_uniform_sizes(nbursts + warm, 1, 2048, 5, 0)
    total = int(sizes.sum())
    mix, isneg, idx = W.lookup_mix(keys[:n], total, neg_rate, 6)
    dmix = to_dev(mix, dev)
    f = torch.empty(total, dtype=torch.uint8, device=dev)
    v = torch.empty(total, dtype=torch.int64, device=dev)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    # the caller waits on the stream its lookup was issued on: a device-wide
    # synchronize has a slow mode (about 30 us) for over a tenth of the
    # waits, on MI355X with ROCm 7.2
    st = torch.cuda.current_stream(dev)
    torch.cuda.synchronize()
    lat = []
    for i in range(len(sizes)):
        a, b = int(offs[i]), int(offs[i + 1])
        q = dmix[a:b]
        t0 = time.perf_counter()
        t.lookup(q, "cuckoopp", found=f[a:b], values=v[a:b], stream=st)
        st.synchronize()
        lat.append(time.perf_counter() - t0)
    fo = f.cpu().numpy()
    vo = v.cpu().numpy().view(np.uint64)
    want_f = (~isneg).astype(np.uint8)
    want_v = np.where(isneg, 0, idx).astype(np.uint64)  # values = insertion index
    if not (np.array_equal(fo, want_f) and np.array_equal(vo, want_v)):
        raise RuntimeError("burst lookups returned a wrong answer")
    loop = loop_burst_latency(t, dmix, sizes, warm, dev, want_f, want_v)
    t.close()
    lat = np.array(lat[warm:]) * 1e6
    counted = int(offs[-1] - offs[warm])
    return {"p50_us": float(np.percentile(lat, 50)), "p99_us": float(np.percentile(lat, 99)),
            "mean_us": float(lat.mean()), "bursts": int(len(lat)),
            "sizes": "log-uniform [1, 2048]", "mean_burst": counted / len(lat),
            "log2_buckets": B, "load": load, "neg_rate": neg_rate,
            "realized_neg_rate": float(isneg[int(offs[warm]):].mean()),
            "form": "one ckpp_lookup_batch per burst, then a wait on its stream "
                    "(submit -> completion)",
            "serving_loop": loop}


def loop_burst_latency(t, dmix, sizes, warm, dev, want_f, want_v, gap_us=100.0):
    """The burst-latency bursts through the serving loop, one at a time:
    the lookups are staged in the loop's ring first, then the native replay
    submits burst i at time i * gap_us (far apart enough that each burst is
    complete before the next arrives) and notes when the loop reports it
    complete; latency = completion - arrival on the host clock (a submit is
    a store to pinned host memory, a completion a load from it, so no HIP
    call is on the path).  Every answer is checked."""
    import torch
    from paper_1712_09624_amd.ckpp import Server
    total = int(sizes.sum())
    srv = Server(t, capacity=1 << (total - 1).bit_length(), budget=1 << 20, idle_ms=2000)
    pos = srv.status()["lookup_tail"]
    srv.put("lookup", pos, dmix)
    n = len(sizes)
    zero = np.zeros(n, np.uint32)
    arrival = np.arange(n, dtype=np.float64) * (gap_us * 1e-6)
    s_before = srv.status()
    _, done = srv.replay(sizes.astype(np.uint32), zero, zero, arrival, 60.0)
    s_after = srv.status()
    rounds = max(1, s_after["rounds"] - s_before["rounds"])
    phase_us = {k[:-3]: (s_after[k] - s_before[k]) / 1e3 / rounds
                for k in ("lookup_ns", "boundary_ns")}
    f, v = srv.get("lookup", pos, total)
    torch.cuda.current_stream(dev).synchronize()
    if not (np.array_equal(f.cpu().numpy(), want_f)
            and np.array_equal(v.cpu().numpy().view(np.uint64), want_v)):
        raise RuntimeError("burst lookups through the serving loop returned a wrong answer")
    srv.close()
    lat = (done - arrival)[warm:] * 1e6
    late = int((lat > gap_us).sum())
    return {"p50_us": float(np.percentile(lat, 50)), "p99_us": float(np.percentile(lat, 99)),
            "mean_us": float(lat.mean()), "bursts": int(len(lat)), "gap_us": gap_us,
            "bursts_over_gap": late, "rounds": s_after["rounds"] - s_before["rounds"],
            "us_per_round": phase_us,
            "form": "the same bursts submitted one at a time to the resident serving loop "
                    "(arrival -> completion seen in host memory)"}


def host_cpu() -> dict:
    """The host's CPU: model, sockets, physical cores (lscpu), the CPUs this
    process may run on (affinity, and the cgroup's CPU quota when one is
    set), and its memory size (/proc/meminfo)."""
    import subprocess
    info = {}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        kv = dict(line.split(":", 1) for line in txt.splitlines() if ":" in line)
        kv = {k.strip(): v.strip() for k, v in kv.items()}
        info["model"] = kv.get("Model name")
        sockets = int(kv.get("Socket(s)", "1") or 1)
        cps = int(kv.get("Core(s) per socket", "0") or 0)
        info["sockets"] = sockets
        info["physical_cores"] = sockets * cps
        info["threads_per_core"] = int(kv.get("Thread(s) per core", "1") or 1)
        info["numa_nodes"] = int(kv.get("NUMA node(s)", "1") or 1)
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    try:
        aff = sorted(os.sched_getaffinity(0))
    except AttributeError:
        aff = list(range(os.cpu_count() or 1))
    info["cpus_allowed"] = len(aff)
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as fh:
            q, per = fh.read().split()
            if q != "max":
                quota = int(q) / int(per)
    except (OSError, ValueError):
        pass
    info["cgroup_cpu_quota"] = quota
    try:
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal:"):
                    info["mem_total_gib"] = int(line.split()[1]) / 2**20
    except OSError:
        pass
    # cores this process may use: the allowed CPUs, at most the quota, one
    # thread per physical core, and at most the host's CPU share for this
    # job when the environment states one (OMP_NUM_THREADS: a shared host
    # gives each GPU's jobs a share of its cores)
    usable = len(aff)
    if quota:
        usable = min(usable, max(1, int(quota)))
    usable = max(1, usable // max(1, info.get("threads_per_core", 1)))
    share = os.environ.get("OMP_NUM_THREADS", "")
    if share.isdigit() and int(share) > 0:
        info["cpu_share"] = int(share)
        usable = min(usable, int(share))
    info["usable_cores"] = usable
    return info


def cpu_baseline(keys, pos, neg, B=24, load=0.9, single_sample=1 << 22):
    """The oracle (single-threaded C, as it stands) timed on the host on the
    benchmark's own workload: the oracle builds its own 2^B-bucket table
    from the same key stream (single-threaded; setup, reported), then runs
    the same positive and negative lookup streams split over one host
    thread per usable physical core (each a plain oracle lookup call on its
    own slice; the calls release the interpreter lock and only read the
    table).  The multi-threaded rate is the reported value; the one-thread
    rate is timed on the first single_sample lookups of each stream."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O
    cpu = host_cpu()
    threads = cpu["usable_cores"]
    nk = W.keys_at_load(B, load)
    t = O.OracleTable(B, W.HASH_SEED, W.MAX_KICKS)
    t0 = time.perf_counter()
    st = t.insert(keys[:nk], W.insertion_values(nk))
    t_ins = time.perf_counter() - t0
    if not (st == O.INSERTED).all():
        raise RuntimeError("the oracle failed to build the benchmark table")
    n = len(pos)
    m = min(single_sample, n)
    t0 = time.perf_counter()
    fp, _, _, _ = t.lookup(pos[:m])
    fn, _, _, _ = t.lookup(neg[:m])
    dt1 = time.perf_counter() - t0
    if not (fp.all() and not fn.any()):
        raise RuntimeError("oracle lookups returned a wrong answer")
    chunks = [a for q in (pos, neg) for a in np.array_split(q, 4 * threads)]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        t0 = time.perf_counter()
        res = list(ex.map(lambda q: t.lookup(q)[0], chunks))
        dtn = time.perf_counter() - t0
    if int(sum(int(r.sum()) for r in res)) != n:
        raise RuntimeError("oracle lookups returned a wrong answer")
    t.close()
    return {"value": 2 * n / dtn / 1e9, "unit": "Glookups/s", "cores": threads, "kind": "oracle",
            "sample": f"the benchmark's own workload: an oracle table of 2^{B} buckets x 8 "
                      f"slots at load {load} built from the same {nk} keys ({t_ins:.1f} s, "
                      f"one thread), the same {n} positive + {n} negative Cuckoo++ lookups "
                      f"split over {threads} host threads on {cpu.get('model')}",
            "single_thread_value": 2 * m / dt1 / 1e9,
            "single_thread_sample": f"{m} positive + {m} negative lookups",
            "insert_per_s": nk / t_ins, "host": cpu}


def latency_probe(dev, steps=4000):
    """Latency of one dependent access of each kind the insert and delete
    paths make (ckpp_probe_latency: plain load, agent-scope atomic load,
    compare-and-swap, load + store + wait, two compare-and-swaps at once,
    and 32 independent loads at once, plain or atomic), on an idle GPU,
    over a 4 GiB buffer (HBM) and a 1 MiB one (cache), in ns per step."""
    import torch
    from paper_1712_09624_amd import ckpp
    out = {}
    for label, nbytes in (("4GiB", 4 << 30), ("1MiB", 1 << 20)):
        buf = torch.zeros(nbytes // 8, dtype=torch.int64, device=dev)
        res = torch.zeros(2, dtype=torch.int64, device=dev)
        r = {}
        for i, kind in enumerate(ckpp.LATENCY_KINDS):
            # step k visits line mix64(seed + k + value): seeds 2^32 apart give
            # the warm-up and the timed chain (and each kind) lines of their own
            ckpp.probe_latency(buf, kind, steps, ((2 * i + 1) << 32), res)   # warm-up
            ckpp.probe_latency(buf, kind, steps, ((2 * i + 2) << 32), res)
            torch.cuda.synchronize()
            r[kind + "_ns"] = int(res[0].item()) * 10.0 / steps
        out[label] = r
        log(f"latency {label}: " + " ".join(f"{k} {v:.0f}" for k, v in r.items()))
        del buf
        torch.cuda.empty_cache()
    return out


def copy_calibration(dev):
    import torch
    a = torch.empty(1 << 27, dtype=torch.int64, device=dev)  # 1 GiB
    b = torch.empty_like(a)
    a.fill_(1)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": 1 << 30, "dispatches": 5}))


def sweep(dev, lookups, probe_peak):
    """Lookup rate of Cuckoo++ and plain lookups over loads {0.6 .. 0.95} and
    negative rates {0 .. 1}, `lookups` (2^26) per point, on a 2^24-bucket
    (4 GiB, HBM-resident), a 2^20-bucket (256 MiB, the size of the
    last-level cache) and a 2^19-bucket (128 MiB, cache-resident) table
    built incrementally.  Each point's frac is given against the HBM
    random-line peak and against the random-line peak measured on a buffer
    of the table's size, and on the method's algorithmic bytes (64-byte
    lines) against 8 TB/s.  Ends with a table of the points on stderr."""
    import torch
    from paper_1712_09624_amd.ckpp import Table
    loads = (0.6, 0.7, 0.8, 0.9, 0.95)
    rates = (0.0, 0.25, 0.5, 0.75, 1.0)
    rows = []
    for B, nlook in ((24, lookups), (20, lookups), (19, lookups)):
        size_peak = probe_line_peak(dev, 256 << B)
        log(f"sweep B={B}: random-line peak on a {256 << B >> 20} MiB buffer "
            f"{size_peak / 1e9:.2f} G/s")
        nmax = W.keys_at_load(B, max(loads))
        keys = W.distinct_five_tuples(nmax, 21 + B, check=False)
        t = Table(B, W.HASH_SEED, W.MAX_KICKS, device=dev.index)
        nf = torch.zeros(1, dtype=torch.int64, device=dev)
        done = 0
        neg_pool = to_dev(W.five_tuples(nlook, 40 + B, stream=W.STREAM_NEGATIVE), dev)
        f = torch.empty(nlook, dtype=torch.uint8, device=dev)
        v = torch.empty(nlook, dtype=torch.int64, device=dev)
        for ld in loads:
            n = W.keys_at_load(B, ld)
            for s0 in range(done, n, 1 << 22):
                s1 = min(n, s0 + (1 << 22))
                t.insert(to_dev(keys[s0:s1], dev),
                         to_dev(W.insertion_values(s1 - s0, s0).view(np.int64), dev), nfailed=nf)
            done = n
            torch.cuda.synchronize()
            st = t.stats()
            lines = expected_lines(st)
            alg = algorithmic_lines_64(st)
            pick = W.raw_u64(50 + B, int(ld * 100), nlook) % np.uint64(n)
            pos_pool = to_dev(keys[pick.astype(np.int64)], dev)
            for r in rates:
                neg = torch.from_numpy(W.bernoulli(nlook, r, 60 + B, int(r * 100))).to(dev)
                q = torch.where(neg[:, None], neg_pool, pos_pool).contiguous()
                for mode, lk in (("cuckoopp", "cuckoopp"), ("both", "plain")):
                    ms = timed(lambda: t.lookup(q, mode, found=f, values=v), 3, dev)
                    req = (1 - r) * lines[f"{lk}_pos"] + r * lines[f"{lk}_neg"]
                    alg_lines = (1 - r) * alg[f"{lk}_pos"] + r * alg[f"{lk}_neg"]
                    rate = nlook / (ms * 1e-3)
                    rows.append({"log2_buckets": B, "load": ld, "neg_rate": r, "mode": lk,
                                 "glookups": rate / 1e9, "lines_per_lookup": req,
                                 "frac_random_line_peak": rate * req / probe_peak,
                                 "same_size_peak_per_s": size_peak,
                                 "frac_same_size_peak": rate * req / size_peak,
                                 "alg_lines_64B": alg_lines,
                                 "frac_hbm_8TBps": rate * (ALG_LINE * alg_lines + STREAM_BYTES)
                                 / (HBM_PEAK_GBS * 1e9),
                                 "failed_inserts": int(nf.item())})
            del pos_pool
            log(f"sweep B={B} load={ld}: " + " ".join(
                f"{x['mode'][0]}{x['neg_rate']}:{x['glookups']:.1f}" for x in rows[-10:]))
        t.close()
        del neg_pool
        torch.cuda.empty_cache()
    log(f"{'B':>3} {'load':>5} {'r':>5} {'mode':>9} {'Glk/s':>7} {'lines128':>8} "
        f"{'frac_peak':>9} {'frac_size':>9} {'lines64':>7} {'frac8TB':>7}")
    for x in rows:
        log(f"{x['log2_buckets']:>3} {x['load']:>5.2f} {x['neg_rate']:>5.2f} {x['mode']:>9} "
            f"{x['glookups']:>7.2f} {x['lines_per_lookup']:>8.3f} {x['frac_random_line_peak']:>9.3f} "
            f"{x['frac_same_size_peak']:>9.3f} {x['alg_lines_64B']:>7.3f} {x['frac_hbm_8TBps']:>7.3f}")
    return rows


def insert_workload(dev, B=24, batch=65536):
    """Insert rate vs load (empty table -> load 0.95 in batches of 65536
    keys), then delete of a random 20% and re-insert of as many fresh keys."""
    import torch
    from paper_1712_09624_amd.ckpp import Table
    n = W.keys_at_load(B, 0.95)
    keys = W.distinct_five_tuples(n, 11, check=False)
    vals = W.insertion_values(n)
    t = Table(B, W.HASH_SEED, W.MAX_KICKS, device=dev.index)
    dk, dv = to_dev(keys, dev), to_dev(vals.view(np.int64), dev)
    st = torch.empty(n, dtype=torch.uint8, device=dev)
    nf = torch.zeros(1, dtype=torch.int64, device=dev)
    s = torch.cuda.current_stream(dev)
    nb = (n + batch - 1) // batch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(nb + 1)]
    torch.cuda.synchronize()
    ev[0].record(s)
    for b in range(nb):
        lo, hi = b * batch, min(n, (b + 1) * batch)
        t.insert(dk[lo:hi], dv[lo:hi], status=st[lo:hi], nfailed=nf)
        ev[b + 1].record(s)
    torch.cuda.synchronize()
    ms = np.array([ev[b].elapsed_time(ev[b + 1]) for b in range(nb)])
    slots = 8 << B
    per_load = []
    for lo_ld in np.arange(0.0, 0.95, 0.05):
        sel = [b for b in range(nb) if lo_ld <= (b * batch) / slots < lo_ld + 0.05]
        if sel:
            k = sum(min(n, (b + 1) * batch) - b * batch for b in sel)
            per_load.append({"load_from": round(float(lo_ld), 2),
                             "minserts_per_s": k / (ms[sel].sum() * 1e-3) / 1e6})
    fails = int(nf.item())
    nd = n // 5
    rows = W.choose_rows(n, nd, 12)
    dd = to_dev(keys[rows], dev)
    fo = torch.empty(nd, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in range(0, nd, batch):
        t.delete(dd[b:b + batch], found=fo[b:b + batch])
    torch.cuda.synchronize()
    del_s = time.perf_counter() - t0
    fresh = to_dev(W.distinct_five_tuples(nd, 13, stream=W.STREAM_FRESH, check=False), dev)
    fv = to_dev(W.insertion_values(nd, n).view(np.int64), dev)
    st2 = torch.empty(nd, dtype=torch.uint8, device=dev)
    nf2 = torch.zeros(1, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b in range(0, nd, batch):
        t.insert(fresh[b:b + batch], fv[b:b + batch], status=st2[b:b + batch], nfailed=nf2)
    torch.cuda.synchronize()
    re_s = time.perf_counter() - t0
    stats = t.stats()
    t.close()
    return {"log2_buckets": B, "batch": batch, "keys": n, "build_ms": float(ms.sum()),
            "build_minserts_per_s": n / (ms.sum() * 1e-3) / 1e6, "build_failed": fails,
            "per_load": per_load, "deleted": nd, "deleted_found": int(fo.sum().item()),
            "delete_minserts_per_s": nd / del_s / 1e6,
            "reinserted": nd, "reinsert_failed": int(nf2.item()),
            "reinsert_minserts_per_s": nd / re_s / 1e6,
            "final_live": stats["live"], "f_sec": stats["f_sec"],
            "retry_exhausted": stats["retry_exhausted"]}


def many_table_bench(dev, ntables=1024, seed=4, reps=20, tune_reps=3, shape=None):
    """Batching workload: ntables independent tables (bucket counts
    log-uniform over 2^10..2^18, loads U[0.6, 0.95], lookup batches
    U[32, 4096], negative rates U[0, 1]), every table's batch served
    (a) by one lookup call per table, eagerly and captured in a HIP graph,
    and (b) by one plan launch, eagerly and captured in a HIP graph, after
    the plan's launch shape is autotuned.  All four give the same answers,
    checked against the workload's ground truth.  shape (lanes per lookup,
    lookups per lane, block, blocks per CU, passes per item, schedule): only
    the plan at that shape, `reps` launches, nothing else (for profiler
    runs)."""
    import torch
    from paper_1712_09624_amd import tune
    from paper_1712_09624_amd.ckpp import Plan, Table
    cfg = W.many_tables(ntables, seed)
    tables, offsets, counts, chunks, want_f, want_v, lines = [], [], [], [], [], [], []
    nkeys = 0
    t0 = time.perf_counter()
    nfail = torch.zeros(1, dtype=torch.int64, device=dev)
    pos = 0
    for i in range(ntables):
        B, load = int(cfg["log2_buckets"][i]), float(cfg["load"][i])
        n = W.keys_at_load(B, load)
        keys = W.distinct_five_tuples(n, seed * 10000 + i, check=False)
        vals = W.insertion_values(n, i << 32)
        t = Table(B, W.HASH_SEED, W.MAX_KICKS, device=dev.index)
        t.insert(to_dev(keys, dev), to_dev(vals.view(np.int64), dev), nfailed=nfail)
        look, neg, idx = W.lookup_mix(keys, int(cfg["batch"][i]), float(cfg["neg_rate"][i]),
                                      seed * 10000 + i)
        want_f.append((~neg).astype(np.uint8))
        want_v.append(np.where(neg, np.uint64(0), vals[np.maximum(idx, 0)]))
        tables.append(t)
        offsets.append(pos)
        counts.append(len(look))
        chunks.append(look)
        pos += len(look)
        nkeys += n
        if i % 128 == 127:
            log(f"many tables: built {i + 1}/{ntables} ({nkeys} keys, {time.perf_counter() - t0:.1f}s)")
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    if int(nfail.item()):
        raise RuntimeError(f"{int(nfail.item())} inserts failed while building the tables")
    # algorithmic lines per lookup of each table, from its own statistics
    neg_rate = np.array([1.0 - float(f.mean()) if len(f) else 0.0 for f in want_f])
    lines64 = []
    for i, t in enumerate(tables):
        st = t.stats()
        el, a64 = expected_lines(st), algorithmic_lines_64(st)
        lines.append(counts[i] * ((1.0 - neg_rate[i]) * el["cuckoopp_pos"]
                                  + neg_rate[i] * el["cuckoopp_neg"]))
        lines64.append(counts[i] * ((1.0 - neg_rate[i]) * a64["cuckoopp_pos"]
                                    + neg_rate[i] * a64["cuckoopp_neg"]))
    total = int(sum(counts))
    # the method's algorithmic bytes (64-byte lines), and the device layout's
    # 128-byte lines
    alg_bytes = ALG_LINE * float(sum(lines64)) + STREAM_BYTES * total
    dev_bytes = LINE * float(sum(lines)) + STREAM_BYTES * total
    keys_d = to_dev(np.concatenate(chunks), dev)
    wf, wv = np.concatenate(want_f), np.concatenate(want_v)
    found = torch.empty(total, dtype=torch.uint8, device=dev)
    vals_d = torch.empty(total, dtype=torch.int64, device=dev)
    views = [(keys_d[o:o + c], found[o:o + c], vals_d[o:o + c]) for o, c in zip(offsets, counts)]

    def check(what):
        torch.cuda.synchronize()
        if not (np.array_equal(found.cpu().numpy(), wf)
                and np.array_equal(vals_d.cpu().numpy().view(np.uint64), wv)):
            raise RuntimeError(f"{what}: wrong answers")
        found.fill_(0xAB)
        vals_d.fill_(-1)

    def per_table():
        for t, (k, f, v) in zip(tables, views):
            t.lookup(k, "cuckoopp", found=f, values=v)

    out = {"tables": ntables, "keys": nkeys, "lookups": total, "build_s": build_s,
           "device_table_bytes": int(sum(256 << int(b) for b in cfg["log2_buckets"])),
           "algorithmic_bytes": alg_bytes, "device_layout_bytes": dev_bytes}
    if shape is not None:
        plan = Plan(tables, offsets, counts)
        lanes, per, block, bpc, passes, sched = shape
        plan.set_launch(per, block, bpc, passes, sched, lanes)
        plan.lookup(keys_d, found, vals_d)
        check("plan (given shape)")
        out["plan_shape"] = plan.get_launch()
        out["plan_us"] = timed(lambda: plan.lookup(keys_d, found, vals_d), reps, dev) * 1e3
        plan.close()
        for t in tables:
            t.close()
        return out
    s = torch.cuda.current_stream(dev)
    # (a) one call per table
    per_table()
    check("per-table calls")
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ms = timed(per_table, reps, dev)
    out["per_table_eager_us"] = ms * 1e3
    out["per_table_eager_wall_us"] = (time.perf_counter() - w0) * 1e6 / (reps + 1)
    g_tab = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g_tab):
        per_table()
    g_tab.replay()
    check("per-table graph")
    out["per_table_graph_us"] = timed(g_tab.replay, reps, dev) * 1e3
    # (b) one plan launch
    plan = Plan(tables, offsets, counts)
    plan.lookup(keys_d, found, vals_d)
    check("plan (default shape)")
    out["plan_default_shape"] = plan.get_launch()
    out["plan_default_us"] = timed(lambda: plan.lookup(keys_d, found, vals_d), reps, dev) * 1e3
    ranked = tune.tune_plan(plan, keys_d, found, vals_d, reps=tune_reps)
    out["plan_tuned_shape"] = ranked[0][1]
    out["plan_tune_top"] = [{"us": r[0] * 1e3, **r[1]} for r in ranked[:8]]
    best_of = {}
    for ms_, sh in ranked:  # fastest shape per (lanes per lookup, lookups per lane, schedule)
        best_of.setdefault(f"lanes{sh['lanes_per_lookup']}_per{sh['lookups_per_lane']}"
                           f"_sched{sh['schedule']}", {"us": ms_ * 1e3, **sh})
    out["plan_tune_best_of"] = best_of
    plan.lookup(keys_d, found, vals_d)
    check("plan (tuned shape)")
    out["plan_eager_us"] = timed(lambda: plan.lookup(keys_d, found, vals_d), reps, dev) * 1e3
    g_plan = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g_plan):
        plan.lookup(keys_d, found, vals_d)
    for _ in range(3):  # every replay is checked
        g_plan.replay()
        check("plan graph replay")
    out["plan_graph_us"] = timed(g_plan.replay, reps, dev) * 1e3
    # a graph replay submits one launch from the host; when that submission
    # takes longer than the kernel, the device idles between replays.  A
    # graph of `reps` launches replayed once shows the launch's own time,
    # and the host's submission time of one replay is timed on the host
    g_many = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g_many):
        for _ in range(reps):
            plan.lookup(keys_d, found, vals_d)
    g_many.replay()
    check("plan graph of many launches")
    out["plan_graph_batched_us"] = timed(g_many.replay, 3, dev) * 1e3 / reps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g_plan.replay()
    out["plan_graph_host_submit_us"] = (time.perf_counter() - t0) * 1e6 / reps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.lookup(keys_d, found, vals_d)
    out["plan_eager_host_submit_us"] = (time.perf_counter() - t0) * 1e6 / reps
    torch.cuda.synchronize()
    del g_many
    del s
    for k in ("per_table_eager", "per_table_graph", "plan_eager", "plan_graph"):
        out[k + "_glookups"] = total / (out[k + "_us"] * 1e-6) / 1e9
    out["plan_graph_over_per_table_graph"] = out["per_table_graph_us"] / out["plan_graph_us"]
    out["plan_graph_over_per_table_eager"] = out["per_table_eager_us"] / out["plan_graph_us"]
    out["plan_achieved_GBps"] = alg_bytes / (out["plan_eager_us"] * 1e-6) / 1e9
    out["plan_frac_hbm_peak"] = out["plan_achieved_GBps"] / HBM_PEAK_GBS
    out["plan_frac_128B_granule"] = dev_bytes / (out["plan_eager_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS
    del g_plan, g_tab
    tuned = plan.get_launch()
    plan.close()
    for t in tables:
        t.close()
    # (c) the same tables with timers (Sec. 4.2): every entry's expiration
    # time uniform over the 1024 units after now0, so all are alive at now0
    # and the answers are those above; one plan launch at the tuned shape,
    # plain and refreshing
    now0 = 65000
    t0 = time.perf_counter()
    tables = []
    for i in range(ntables):
        B, load = int(cfg["log2_buckets"][i]), float(cfg["load"][i])
        n = W.keys_at_load(B, load)
        keys = W.distinct_five_tuples(n, seed * 10000 + i, check=False)
        vals = W.insertion_values(n, i << 32)
        exp = W.times_after(n, now0, 1024, seed * 10000 + i)
        t = Table(B, W.HASH_SEED, W.MAX_KICKS, device=dev.index, timers=True)
        t.insert_at(to_dev(keys, dev), to_dev(vals.view(np.int64), dev),
                    to_dev(exp.view(np.int16), dev), now0, nfailed=nfail)
        tables.append(t)
    torch.cuda.synchronize()
    out["timed_build_s"] = time.perf_counter() - t0
    if int(nfail.item()):
        raise RuntimeError(f"{int(nfail.item())} inserts failed while building the timed tables")
    plan = Plan(tables, offsets, counts)
    plan.set_launch(tuned["lookups_per_lane"], tuned["block"], tuned["blocks_per_cu"],
                    tuned["passes_per_item"], tuned["schedule"], tuned["lanes_per_lookup"])
    plan.lookup(keys_d, found, vals_d, now=now0)
    check("plan with timers")
    out["plan_timed_us"] = timed(lambda: plan.lookup(keys_d, found, vals_d, now=now0), reps,
                                 dev) * 1e3
    refresh = (now0 + 1000) & 0xFFFF
    plan.lookup(keys_d, found, vals_d, now=now0, refresh=refresh)
    check("refreshing plan with timers")
    # each timed launch sets a time other than the previous launch's, so
    # every hit writes (a hit that finds the time already set writes nothing)
    last = [refresh]

    def run_refresh():
        last[0] = (refresh - 1) & 0xFFFF if last[0] == refresh else refresh
        plan.lookup(keys_d, found, vals_d, now=now0, refresh=last[0])

    out["plan_timed_refresh_us"] = timed(run_refresh, reps, dev) * 1e3
    out["plan_timed_overhead"] = out["plan_timed_us"] / out["plan_eager_us"] - 1.0
    plan.close()
    for t in tables:
        t.close()
    return out


SERVE_UNIVERSE = 100_000_000
SERVE_SCRAMBLE = 2654435761  # odd, prime to 10^8: rank -> flow is a permutation


def serve_stream(nbursts, seed, keys, universe, vals, del_base):
    """One serving run's bursts: sizes log-uniform in [1, 2048]; each burst
    0.9 n lookups (rounded half up), 0.1 n inserts of new flows, 0.05 n
    deletes of expired flows.  Lookups pick flows of the universe by Zipf
    s = 1.1 popularity (rank r -> flow r * SERVE_SCRAMBLE mod universe);
    inserts are fresh keys; deletes take stored keys outside the universe,
    from del_base on."""
    size = W.log_uniform_sizes(nbursts, 1, 2048, seed, 20)
    nl = np.floor(0.9 * size + 0.5).astype(np.int64)
    ni = np.floor(0.1 * size + 0.5).astype(np.int64)
    nd = np.floor(0.05 * size + 0.5).astype(np.int64)
    ranks = W.zipf_ranks(int(nl.sum()), universe, 1.1, seed, 21)
    flows = (ranks.astype(np.uint64) * np.uint64(SERVE_SCRAMBLE)) % np.uint64(universe)
    flows = flows.astype(np.int64)
    ins = W.five_tuples(int(ni.sum()), seed, 22)
    dels = np.arange(del_base, del_base + int(nd.sum()), dtype=np.int64)
    if dels.size and dels[-1] >= len(keys):
        raise RuntimeError("not enough expired flows for the deletes")
    return {"nl": nl, "ni": ni, "nd": nd, "look": keys[flows], "look_val": vals[flows],
            "ins": ins, "ins_val": np.arange(int(ni.sum()), dtype=np.uint64) + np.uint64(1 << 40),
            "dels": keys[dels], "del_next": del_base + int(nd.sum())}


SERVE_NOW0, SERVE_TTL, SERVE_TICK = 1000, 1023, 50


def serve_bench(dev, nbursts=50000, B=24, load=0.85, fracs=(0.25, 0.5, 0.75, 1.0),
                budget=1 << 20, capacity=1 << 25, timers=False, blocks_per_cu=1):
    """Serving workload: a 2^24-bucket table at load 0.85 whose first 100M
    keys are the flow universe; a closed-loop run measures the loop's peak,
    then open-loop Poisson runs offer 25/50/75/100 % of it.  Every run's
    lookups, inserts and deletes are checked against the ground truth.
    timers: the table has timers (every key built to expire at time
    SERVE_NOW0 + SERVE_TTL); the server's entries live SERVE_TTL units and
    lookups renew them; run r runs at time SERVE_NOW0 + SERVE_TICK (r + 1),
    so every key stays alive.  The first time set starts with the loop's
    anti-revival scan of the whole table, timed on its own."""
    import torch
    from paper_1712_09624_amd.ckpp import Server
    n = W.keys_at_load(B, load)
    expiry = np.full(n, SERVE_NOW0 + SERVE_TTL, np.uint16) if timers else None
    t, keys, vals, build_s = build_table(B, load, 11, dev, expiry=expiry, now=SERVE_NOW0)
    universe = min(SERVE_UNIVERSE, len(keys))
    srv = Server(t, capacity=capacity, budget=budget, blocks_per_cu=blocks_per_cu, idle_ms=2000,
                 ttl=SERVE_TTL if timers else 0, refresh=timers)
    out = {"log2_buckets": B, "load": load, "stored_keys": len(keys), "universe": universe,
           "budget_ops": budget, "ring_capacity": capacity, "bursts_per_run": nbursts,
           "grid_blocks": srv.status()["grid"], "timers": timers, "runs": []}
    del_base = universe
    peak_lps = None
    for run, frac in enumerate((None,) + tuple(fracs)):
        st = serve_stream(nbursts, 100 + run, keys, universe, vals, del_base)
        del_base = st["del_next"]
        # stage the run's operations in the rings
        s0 = srv.status()
        pos = [s0["lookup_tail"], s0["insert_tail"], s0["delete_tail"]]
        srv.put("lookup", pos[0], to_dev(st["look"], dev))
        if len(st["ins"]):
            srv.put("insert", pos[1], to_dev(st["ins"], dev),
                    to_dev(st["ins_val"].view(np.int64), dev))
        if len(st["dels"]):
            srv.put("delete", pos[2], to_dev(st["dels"], dev))
        mean_l = float(st["nl"].mean())
        if timers:
            s_scan = srv.status()
            t0 = time.perf_counter()
            if not srv.set_time(SERVE_NOW0 + SERVE_TICK * (run + 1)):
                raise RuntimeError("the time change was not admitted")
            s_set = srv.status()
            if s_set["submitted"] > s_scan["submitted"]:  # the scan's empty burst
                srv.wait(s_set["submitted"] - 1, 60000)
                s_done = srv.status()
                out["scan"] = {"host_ms": (time.perf_counter() - t0) * 1e3,
                               "loop_ms": (s_done["boundary_ns"] - s_scan["boundary_ns"]) / 1e6,
                               "table_gib": (256 << B) / 2**30}
                log(f"scan in the loop: {out['scan']}")
        if frac is None:
            arrival = np.zeros(nbursts)
        else:
            arrival = W.poisson_arrivals(nbursts, frac * peak_lps / mean_l, 100 + run, 23)
        s_before = srv.status()
        adm, done = srv.replay(st["nl"], st["ni"], st["nd"], arrival, 120.0)
        s_after = srv.status()
        rounds = s_after["rounds"] - s_before["rounds"]
        phase_us = {k[:-3]: (s_after[k] - s_before[k]) / 1e3 / max(rounds, 1)
                    for k in ("lookup_ns", "insert_ns", "delete_ns", "boundary_ns")}
        # verify every result of the run
        f, v = srv.get("lookup", pos[0], len(st["look"]))
        ist = srv.get("insert", pos[1], len(st["ins"]))
        dfo = srv.get("delete", pos[2], len(st["dels"]))
        torch.cuda.current_stream(dev).synchronize()
        ok = (bool((f.cpu().numpy() == 1).all())
              and np.array_equal(v.cpu().numpy().view(np.uint64), st["look_val"])
              and bool((ist.cpu().numpy() == 0).all()) and bool((dfo.cpu().numpy() == 1).all()))
        if not ok:
            raise RuntimeError(f"serving run {run}: wrong results")
        span = float(done.max() - arrival.min())
        lat = (done - arrival) * 1e6
        nlook = int(st["nl"].sum())
        ops = nlook + int(st["ni"].sum()) + int(st["nd"].sum())
        rec = {"offered": "closed loop (peak)" if frac is None else frac,
               "offered_glookups": None if frac is None else frac * peak_lps / 1e9,
               "glookups": nlook / span / 1e9, "gops": ops / span / 1e9,
               "p50_us": float(np.percentile(lat, 50)), "p99_us": float(np.percentile(lat, 99)),
               "mean_us": float(lat.mean()), "rounds": rounds,
               "bursts_per_round": nbursts / max(rounds, 1), "us_per_round": phase_us,
               "lookups": nlook, "ops": ops,
               "span_s": span}
        if frac is None:
            peak_lps = nlook / span
        out["runs"].append(rec)
        log(f"serve run {run}: {rec}")
    srv.close()
    if timers:
        t.close()
        return out
    # the same kind of stream through the plain batch calls, burst by burst
    # (lookup, insert and delete batch of each burst, then a wait on their stream)
    nplain = min(5000, nbursts)
    st = serve_stream(nplain, 100 + len(out["runs"]), keys, universe, vals, del_base)
    out["plain_calls"] = plain_call_run(t, st, dev)
    log(f"plain calls: {out['plain_calls']}")
    t.close()
    return out


def plain_call_run(t, st, dev):
    """Bursts served one at a time by the plain batch calls, back to back
    (closed loop): per burst a lookup, an insert and a delete batch on the
    caller's stream and a wait on that stream.  Every result is checked."""
    import torch
    look, ins, dels = to_dev(st["look"], dev), to_dev(st["ins"], dev), to_dev(st["dels"], dev)
    ins_v = to_dev(st["ins_val"].view(np.int64), dev)
    nl, ni, nd = st["nl"], st["ni"], st["nd"]
    f = torch.empty(len(st["look"]), dtype=torch.uint8, device=dev)
    v = torch.empty(len(st["look"]), dtype=torch.int64, device=dev)
    ist = torch.empty(max(1, len(st["ins"])), dtype=torch.uint8, device=dev)
    dfo = torch.empty(max(1, len(st["dels"])), dtype=torch.uint8, device=dev)
    nf = torch.zeros(1, dtype=torch.int64, device=dev)
    lat = np.empty(len(nl))
    ol = oi = od = 0
    s = torch.cuda.current_stream(dev)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for b in range(len(nl)):
        t0 = time.perf_counter()
        a, c, e = int(nl[b]), int(ni[b]), int(nd[b])
        if a:
            t.lookup(look[ol:ol + a], found=f[ol:ol + a], values=v[ol:ol + a])
        if c:
            t.insert(ins[oi:oi + c], ins_v[oi:oi + c], status=ist[oi:oi + c], nfailed=nf)
        if e:
            t.delete(dels[od:od + e], found=dfo[od:od + e])
        s.synchronize()
        lat[b] = time.perf_counter() - t0
        ol, oi, od = ol + a, oi + c, od + e
    span = time.perf_counter() - t_start
    ok = (bool((f.cpu().numpy() == 1).all())
          and np.array_equal(v.cpu().numpy().view(np.uint64), st["look_val"])
          and bool((ist[:oi].cpu().numpy() == 0).all()) and bool((dfo[:od].cpu().numpy() == 1).all())
          and int(nf.item()) == 0)
    if not ok:
        raise RuntimeError("plain-call serving run: wrong results")
    lat *= 1e6
    return {"bursts": int(len(nl)), "glookups": ol / span / 1e9, "gops": (ol + oi + od) / span / 1e9,
            "p50_us": float(np.percentile(lat, 50)), "p99_us": float(np.percentile(lat, 99)),
            "mean_us": float(lat.mean()), "span_s": span}


PROFILE_CMDS = {
    "trace": "rocprofv3 --kernel-trace --stats --output-format csv -d DIR/p4_trace -o core -- "
             "python3 bench.py --core-only --steps 5 --warmup 2",
    "fetch": "rocprofv3 --pmc FETCH_SIZE --output-format csv -d DIR/p4_fetch -o core -- "
             "python3 bench.py --core-only --steps 5 --warmup 2",
    "write": "rocprofv3 --pmc WRITE_SIZE --output-format csv -d DIR/p4_write -o core -- "
             "python3 bench.py --core-only --steps 5 --warmup 2",
    "req": "rocprofv3 --pmc TCC_EA0_RDREQ_sum TCC_EA0_RDREQ_32B_sum TCC_EA0_RDREQ_64B_sum "
           "TCC_EA0_RDREQ_128B_sum --output-format csv -d DIR/p4_req -o core -- "
           "python3 bench.py --core-only --steps 5 --warmup 2",
    "copy": "the same three --pmc runs with -d DIR/p4_copy_{fetch,write,req} -o copy -- "
            "python3 bench.py --copy-calib",
}


def _pmc(path, kernel_part):
    import csv
    per = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if kernel_part in r["Kernel_Name"]:
                per.setdefault(int(r["Dispatch_Id"]), {})[r["Counter_Name"]] = float(r["Counter_Value"])
    return [per[k] for k in sorted(per)]


def summarize_profiles(d):
    """Writes profiles/ summaries from the rocprofv3 CSV output of the
    commands in PROFILE_CMDS (run from the repository root with DIR = d)."""
    import csv
    prof = os.path.join(ROOT, "profiles")
    from paper_1712_09624_amd import ckpp
    # the profiled runs use the default launch shape
    kname = ckpp.lookup_kernel_name(ckpp.DEFAULT_LAUNCH)
    # kernel trace
    rows = list(csv.DictReader(open(os.path.join(d, "p4_trace", "core_kernel_stats.csv"))))
    out = ["# rocprofv3 kernel-trace summary: Cuckoo++ step on a 2^24-bucket table at load 0.9",
           "# (bench.py --core-only: table build in 4M-key insert batches, then per step",
           "#  insert 65536 + lookup 2^26 positive + lookup 2^26 negative + delete 65536)",
           "# device layout: 256-byte buckets, two 128-byte lines; lookup kernel " + kname,
           "# command (repository root, TMPDIR=/tmp): " + PROFILE_CMDS["trace"].replace("DIR", d),
           f"{'kernel':<40} {'calls':>6} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'pct':>6}"]
    for r in rows:
        name = r["Name"].replace("void ", "", 1).replace("ckpp::(anonymous namespace)::", "")
        depth, cut = 0, len(name)
        for i, ch in enumerate(name):
            if ch == "<":
                depth += 1
            elif ch == ">":
                depth -= 1
            elif ch == "(" and depth == 0 and i > 0 and name[i - 1] != " ":
                cut = i
                break
        out.append(f"{name[:cut][:40]:<40} {int(r['Calls']):>6} {float(r['AverageNs']) / 1e3:>10.1f} "
                   f"{float(r['MinNs']) / 1e3:>10.1f} {float(r['MaxNs']) / 1e3:>10.1f} "
                   f"{float(r['Percentage']):>6.2f}")
    out.append(f"# {kname} launches alternate positive (the longer) and negative batches;")
    out.append("# their average is the avg_launch_ms bench.py reports in roofline.")
    with open(os.path.join(prof, f"{kname}_b24_load0.9_kernel_trace.txt"), "w") as fh:
        fh.write("\n".join(out) + "\n")
    # traffic
    lk = {k: _pmc(os.path.join(d, f"p4_{k}", "core_counter_collection.csv"), kname)
          for k in ("fetch", "write", "req")}
    cp = {k: _pmc(os.path.join(d, f"p4_copy_{k}", "copy_counter_collection.csv"), "copyBuffer")
          for k in ("fetch", "write", "req")}
    copy_bytes = 1 << 30
    f_fetch = copy_bytes / (cp["fetch"][0]["FETCH_SIZE"] * 1024)
    f_write = copy_bytes / (cp["write"][0]["WRITE_SIZE"] * 1024)
    def exact(v):
        return (v["TCC_EA0_RDREQ_32B_sum"] * 32 + v["TCC_EA0_RDREQ_64B_sum"] * 64 +
                v["TCC_EA0_RDREQ_128B_sum"] * 128)
    f_req = copy_bytes / exact(cp["req"][0])
    fetch = [v["FETCH_SIZE"] * 1024 * f_fetch for v in lk["fetch"]]
    write = [v["WRITE_SIZE"] * 1024 * f_write for v in lk["write"]]
    reqb = [exact(v) * f_req for v in lk["req"]]
    nreq = [v["TCC_EA0_RDREQ_sum"] for v in lk["req"]]
    per_launch = (sum(fetch) + sum(write)) / len(fetch)
    lines = [f"# HBM traffic of the Cuckoo++ lookup kernel ({kname}), 2^24 buckets at load 0.9,",
             "# 2^26 lookups per launch, launches alternating positive / negative batches",
             "# commands (repository root, TMPDIR=/tmp, one counter group per run):"]
    for k in ("fetch", "write", "req", "copy"):
        lines.append("#   " + PROFILE_CMDS[k].replace("DIR", d))
    lines += [f"# calibration on a 1 GiB device copy: FETCH_SIZE x {f_fetch:.4f}, WRITE_SIZE x {f_write:.4f},",
              f"#   request-size bytes (32*RDREQ_32B + 64*RDREQ_64B + 128*RDREQ_128B) x {f_req:.4f}",
              f"{'dispatch':>8} {'fetch_GB':>10} {'write_GB':>10} {'reqsize_GB':>11} {'rd_requests':>13}"]
    for i in range(len(fetch)):
        lines.append(f"{i:>8} {fetch[i] / 1e9:>10.3f} {write[i] / 1e9:>10.3f} {reqb[i] / 1e9:>11.3f} "
                     f"{nreq[i]:>13.0f}")
    lines.append(f"# mean HBM bytes per launch (calibrated fetch + write): {per_launch / 1e9:.3f} GB")
    with open(os.path.join(prof, f"{kname}_b24_load0.9_hbm_traffic.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    with open(os.path.join(prof, "lookup_traffic.json"), "w") as fh:
        json.dump({"source_digest": lookup_source_digest(),
                   "launch": dict(ckpp.DEFAULT_LAUNCH), "kernel": kname,
                   "hbm_bytes_per_launch": per_launch,
                   "fetch_factor": f_fetch, "write_factor": f_write,
                   "dispatches": len(fetch)}, fh, indent=1)
    print("\n".join(out + lines))


PLAN_PROFILE_CMD = "python3 bench.py --many-tables 1024 --plan-shape 1,1,128,8,1,0"


def summarize_plan_profiles(d):
    """Writes the profiles/ summary of the plan kernel from the rocprofv3 CSV
    output under d of: a kernel trace (d/plan_trace), FETCH_SIZE
    (d/plan_fetch), WRITE_SIZE (d/plan_write) and the read-request sizes
    (d/plan_req), each of PLAN_PROFILE_CMD, and the 1 GiB copy calibration
    of the lookup profiles (d/p4_copy_{fetch,write}, the PROFILE_CMDS
    "copy" runs)."""
    import csv
    rows = [r for r in csv.DictReader(open(os.path.join(d, "plan_trace", "plan_kernel_stats.csv")))
            if "lookup_plan" in r["Name"]]
    r = rows[0]
    fetch = [v["FETCH_SIZE"] for v in _pmc(os.path.join(d, "plan_fetch", "plan_counter_collection.csv"),
                                             "lookup_plan")]
    write = [v["WRITE_SIZE"] for v in _pmc(os.path.join(d, "plan_write", "plan_counter_collection.csv"),
                                             "lookup_plan")]
    req = _pmc(os.path.join(d, "plan_req", "plan_counter_collection.csv"), "lookup_plan")
    cpf = _pmc(os.path.join(d, "p4_copy_fetch", "copy_counter_collection.csv"), "copyBuffer")
    cpw = _pmc(os.path.join(d, "p4_copy_write", "copy_counter_collection.csv"), "copyBuffer")
    f_fetch = (1 << 30) / (cpf[0]["FETCH_SIZE"] * 1024)
    f_write = (1 << 30) / (cpw[0]["WRITE_SIZE"] * 1024)
    fb = float(np.mean(fetch)) * 1024 * f_fetch
    wb = float(np.mean(write)) * 1024 * f_write
    nreq = float(np.mean([v["TCC_EA0_RDREQ_sum"] for v in req]))
    n128 = float(np.mean([v["TCC_EA0_RDREQ_128B_sum"] for v in req]))
    n64 = float(np.mean([v["TCC_EA0_RDREQ_64B_sum"] for v in req]))
    n32 = float(np.mean([v["TCC_EA0_RDREQ_32B_sum"] for v in req]))
    lines = [
        "# lookup_plan: 1024 tables (2^10..2^18 buckets, loads 0.6..0.95, batches 32..4096,",
        "#   negative rates 0..1; 2,144,563 lookups) in one launch at the tuned shape",
        "#   (1 lane per lookup, 1 lookup per lane, block 128, 8 blocks/CU, 1 pass/item, static)",
        "# commands (repository root, TMPDIR=/tmp, one counter group per run):",
        f"#   rocprofv3 --kernel-trace --stats --output-format csv -d {d}/plan_trace -o plan -- "
        f"{PLAN_PROFILE_CMD}",
        f"#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d {d}/plan_fetch -o plan -- "
        f"{PLAN_PROFILE_CMD}",
        f"#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d {d}/plan_write -o plan -- "
        f"{PLAN_PROFILE_CMD}",
        f"#   rocprofv3 --pmc TCC_EA0_RDREQ_sum TCC_EA0_RDREQ_32B_sum TCC_EA0_RDREQ_64B_sum "
        f"TCC_EA0_RDREQ_128B_sum --output-format csv -d {d}/plan_req -o plan -- {PLAN_PROFILE_CMD}",
        "#   calibration: the copy runs of the lookup profiles (FETCH_SIZE x "
        f"{f_fetch:.4f}, WRITE_SIZE x {f_write:.4f})",
        f"kernel trace: {int(r['Calls'])} launches, average {float(r['AverageNs']) / 1e3:.1f} us, "
        f"min {float(r['MinNs']) / 1e3:.1f}, max {float(r['MaxNs']) / 1e3:.1f}",
        f"HBM traffic per launch (calibrated): fetch {fb / 1e6:.1f} MB, write {wb / 1e6:.1f} MB",
        f"read requests per launch: {nreq:.0f} (128 B: {n128:.0f}, 64 B: {n64:.0f}, "
        f"32 B: {n32:.0f}); {nreq / 2144563:.3f} per lookup",
    ]
    with open(os.path.join(ROOT, "profiles", "lookup_plan_1024_tables_trace_traffic.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


SERVE_COUNTER_CMDS = {
    "serve_a": "FETCH_SIZE SQ_WAVE_CYCLES SQ_WAIT_INST_ANY SQ_WAIT_ANY SQ_BUSY_CYCLES "
               "SQC_ICACHE_MISSES SQC_ICACHE_HITS",
    "serve_b": "WRITE_SIZE TCC_EA0_RDREQ_sum TCC_EA0_RDREQ_128B_sum",
}


def serve_counter_lines(d):
    """Summary lines of the serving loop's counter runs under d (one
    rocprofv3 --pmc run per SERVE_COUNTER_CMDS entry of
    `python3 bench.py --serve 20000`, plus the 1 GiB copy calibration of the
    lookup profiles): HBM bytes and read requests per operation served."""
    import csv
    tot, ops = {}, {}
    for run in SERVE_COUNTER_CMDS:
        for r in csv.DictReader(open(os.path.join(d, run, "serve_counter_collection.csv"))):
            if "serve_loop" in r["Kernel_Name"]:
                tot[r["Counter_Name"]] = tot.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        log_path = os.path.join(d, run + ".log")
        rec = [json.loads(x) for x in open(log_path) if x.startswith('{"serve"')][-1]["serve"]
        ops[run] = (sum(r["ops"] for r in rec["runs"]), sum(r["lookups"] for r in rec["runs"]),
                    sum(r["rounds"] for r in rec["runs"]))
    cpf = _pmc(os.path.join(d, "p4_copy_fetch", "copy_counter_collection.csv"), "copyBuffer")
    cpw = _pmc(os.path.join(d, "p4_copy_write", "copy_counter_collection.csv"), "copyBuffer")
    f_fetch = (1 << 30) / (cpf[0]["FETCH_SIZE"] * 1024)
    f_write = (1 << 30) / (cpw[0]["WRITE_SIZE"] * 1024)
    na, la, ra = ops["serve_a"]
    nb_, _, _ = ops["serve_b"]
    fetch = tot["FETCH_SIZE"] * 1024 * f_fetch / na
    write = tot["WRITE_SIZE"] * 1024 * f_write / nb_
    req = tot["TCC_EA0_RDREQ_sum"] / nb_
    r128 = tot["TCC_EA0_RDREQ_128B_sum"] / nb_
    out = ["# loop counters (rocprofv3 --pmc, one run per group, each the loop's dispatches of",
           "#   python3 bench.py --serve 20000; the profiler serializes dispatches, so the loop",
           "#   idles out and relaunches between runs and the runs' timings do not count):"]
    for run, cnt in SERVE_COUNTER_CMDS.items():
        out.append(f"#   rocprofv3 --pmc {cnt} --output-format csv -d {d}/{run} -o serve -- "
                   "python3 bench.py --serve 20000")
    out += [f"#   calibration: FETCH_SIZE x {f_fetch:.4f}, WRITE_SIZE x {f_write:.4f} (1 GiB copy)",
            f"HBM bytes per operation served: fetch {fetch:.0f}, write {write:.0f} "
            f"({na:,} operations, {la:,} of them lookups, {ra} rounds)",
            f"read requests per operation: {req:.2f} ({r128:.2f} of 128 bytes)",
            f"instruction cache: {tot['SQC_ICACHE_MISSES']:.0f} misses in "
            f"{tot['SQC_ICACHE_HITS']:.3g} hits; waves waiting for an instruction "
            f"{100 * tot['SQ_WAIT_INST_ANY'] / tot['SQ_WAVE_CYCLES']:.1f}% of wave cycles, "
            f"waiting on anything {100 * tot['SQ_WAIT_ANY'] / tot['SQ_WAVE_CYCLES']:.1f}%"]
    return out


def summarize_latency(path):
    """Writes profiles/dependent_access_latency.txt from the JSON line of
    `python3 bench.py --latency` saved at `path`."""
    rec = [json.loads(x) for x in open(path) if x.startswith("{")][-1]["latency_ns"]
    names = {"load_ns": "plain load", "atomic_load_ns": "relaxed agent-scope atomic load",
             "cas_ns": "compare-and-swap (expects 1, writes 1)",
             "load_store_wait_ns": "atomic load + atomic store + wait for the store",
             "cas_pair_ns": "two compare-and-swaps issued together",
             "load_batch32_ns": "32 independent plain loads, issued together",
             "atomic_load_batch32_ns": "32 independent atomic loads, issued together"}
    out = ["# Latency of one step of each access the insert and delete paths make, one lane of one",
           "# wavefront on an idle MI355X (ckpp_probe_latency; steps chained by their values, 4000",
           "# per kind; lines chosen at random in the buffer), ns per step",
           "# command (repository root): python3 bench.py --latency",
           f"{'access':<52} {'4 GiB (HBM)':>12} {'1 MiB (cache)':>14}"]
    for k, name in names.items():
        out.append(f"{name:<52} {rec['4GiB'][k]:>12.0f} {rec['1MiB'][k]:>14.0f}")
    out.append("# a batch of independent loads from one lane completes at about 80 ns per load in")
    out.append("#   either buffer: one lane's scattered loads are bounded by their issue, not by HBM")
    with open(os.path.join(ROOT, "profiles", "dependent_access_latency.txt"), "w") as fh:
        fh.write("\n".join(out) + "\n")
    print("\n".join(out))


# Earlier records of the same command, kept with the summary.
INSERT_WORKLOAD_HISTORY = [
    "# earlier path searches, same command: plain random walk (no lookahead) 734.9 ms = 173.5 M/s,",
    "#   band 0.85: 55.6, band 0.90: 17.9, re-insert 81.5 M/s; walk with lookahead only: 228.8 ms =",
    "#   557.3 M/s, band 0.85: 284.0, band 0.90: 180.2, re-insert 339.6 M/s; displacements inlined:",
    "#   211.2 ms, band 0.05: 764, band 0.85: 404, band 0.90: 302, re-insert 472 M/s",
    "#   pool-allocated path scratch for batches above 4096 lanes: 182.0 ms =",
    "#   700.5 M/s, band 0.05: 950, band 0.90: 305, re-insert 522 M/s",
    "#   agent-scope acquire/release fences around each critical section (an L2 invalidate and an L2",
    "#   write-back per lock cycle): 170.6 ms = 747.2 M/s, band 0.05: 1026, band 0.90:",
    "#   317, delete 1139 M/s, re-insert 547 M/s",
    "#   two-level lookahead over every candidate at once (104 loads): 99.4 ms =",
    "#   1282.2 M/s, band 0.85: 792.5, band 0.90: 510.5, re-insert 941.6 M/s",
    "#   one candidate at a time, walks for paths blocked by another lane's lock (previous record):",
    "#   92.8 ms = 1373.9 M/s, band 0.85: 937.1, band 0.90: 633.5, re-insert 1115.6 M/s",
]


def summarize_insert_workload(path):
    """Writes profiles/insert_workload_b24.txt from the JSON line of
    `python3 bench.py --insert-workload` saved at `path`."""
    rec = [json.loads(x) for x in open(path) if x.startswith("{")][-1]
    w = rec.get("insert_workload", rec)
    out = ["# Batched insert workload on MI355X: empty 2^24-bucket table -> load 0.95 in batches of 65536",
           "# keys (max kick chain 500), then delete of a random 20% and re-insert of as many fresh keys.",
           "# Per-batch times from HIP events; delete/re-insert times wall-clock around the batch loops.",
           "# cuckoo paths: up to two displacements done inside the locked DIRECT step when the primary's",
           "#   entries (one level, else two levels of lookahead, one candidate at a time) reach a free",
           "#   slot (a path blocked by another lane's lock is retried, up to 4 times); else a random walk",
           "#   with one step of lookahead, whose path (up to 8 displacements) is applied in one critical",
           "#   section; the rare paths are compiled out of line",
           "# path scratch: a buffer of the table's own (up to 1/32 of the table's memory, here all 2^16 lanes",
           "#   of a batch), allocated once; the stream-ordered pool only beyond that",
           "# locks: table words under a lock read and written with device-coherent (agent-scope) accesses,",
           "#   so taking and dropping a lock flushes no L2 cache",
           "# command (repository root): python3 bench.py --insert-workload",
           f"keys {w['keys']}  build {w['build_ms']:.1f} ms = {w['build_minserts_per_s']:.1f} M inserts/s  "
           f"failed {w['build_failed']}",
           f"delete {w['deleted']} (found {w['deleted_found']}) at {w['delete_minserts_per_s']:.0f} M/s",
           f"re-insert {w['reinserted']} (failed {w['reinsert_failed']}) at "
           f"{w['reinsert_minserts_per_s']:.1f} M/s",
           f"final live {w['final_live']}  entries in secondary {w['f_sec']:.4f}  "
           f"retry bound reached {w['retry_exhausted']}",
           "insert rate by load band:",
           " load from  M inserts/s"]
    for b in w["per_load"]:
        out.append(f"{b['load_from']:>10.2f} {b['minserts_per_s']:>13.1f}")
    out += INSERT_WORKLOAD_HISTORY
    with open(os.path.join(ROOT, "profiles", "insert_workload_b24.txt"), "w") as fh:
        fh.write("\n".join(out) + "\n")
    print("\n".join(out))


def summarize_many_tables(path):
    """Writes profiles/plan_1024_tables_batching.txt from the JSON line of
    `python3 bench.py --many-tables 1024` saved at `path`."""
    rec = [json.loads(x) for x in open(path) if x.startswith("{")][-1]
    m = rec.get("many_tables", rec)
    n = m["lookups"]
    g = lambda us: n / (us * 1e-6) / 1e9
    out = ["# Many-table batching: 1024 tables, one lookup batch each, served by one call per table",
           "# versus one plan launch (persistent lookup_plan kernel), MI355X, ROCm 7.2",
           "# workload: bucket counts 2^10..2^18 (exponent uniform), loads U[0.6, 0.95], batches U[32, 4096],",
           "#   negative rates U[0, 1], seed 4; every answer checked against the workload's ground truth",
           "# command (repository root): python3 bench.py --many-tables 1024",
           f"tables {m['tables']}  keys {m['keys']}  lookups {n}  table bytes "
           f"{m['device_table_bytes'] / 1e9:.1f} GB",
           f"{'form':<44} {'us':>8} {'Glookups/s':>11}",
           f"{'one call per table, eager':<44} {m['per_table_eager_us']:>8.1f} "
           f"{g(m['per_table_eager_us']):>11.2f}",
           f"{'one call per table, HIP graph':<44} {m['per_table_graph_us']:>8.1f} "
           f"{g(m['per_table_graph_us']):>11.2f}",
           f"{'plan, tuned shape, eager':<44} {m['plan_eager_us']:>8.1f} {g(m['plan_eager_us']):>11.2f}",
           f"{'plan, tuned shape, HIP graph (one replay)':<44} {m['plan_graph_us']:>8.1f} "
           f"{g(m['plan_graph_us']):>11.2f}",
           f"{'plan, tuned shape, HIP graph (replays queued)':<44} {m['plan_graph_batched_us']:>8.1f} "
           f"{g(m['plan_graph_batched_us']):>11.2f}",
           f"plan at its first shape {m['plan_default_shape']}: {m['plan_default_us']:.1f} us",
           f"tuned shape: {m['plan_tuned_shape']}",
           f"{'plan, tables with timers, tuned shape':<44} {m['plan_timed_us']:>8.1f} "
           f"{g(m['plan_timed_us']):>11.2f}",
           f"{'plan, tables with timers, refreshing':<44} {m['plan_timed_refresh_us']:>8.1f} "
           f"{g(m['plan_timed_refresh_us']):>11.2f}",
           f"plan algorithmic bytes (64-byte lines) {m['algorithmic_bytes'] / 1e6:.1f} MB -> "
           f"{m['algorithmic_bytes'] / (m['plan_eager_us'] * 1e-6) / 1e9:.0f} GB/s = "
           f"{m['plan_frac_hbm_peak']:.3f} of 8 TB/s; in the device layout's 128-byte lines "
           f"{m['device_layout_bytes'] / 1e6:.1f} MB = {m['plan_frac_128B_granule']:.3f}",
           "# fastest shape per (lanes per lookup, lookups per lane, schedule 0 static / 1 dynamic):"]
    best = m["plan_tune_best_of"]
    items = best.items() if isinstance(best, dict) else best
    for k, v in sorted(items, key=lambda kv: kv[1]["us"]):
        out.append(f"#   {k}: {v['us']:.1f} us  block {v['block']} blocks/CU {v['blocks_per_cu']} "
                   f"passes/item {v['passes_per_item']}")
    with open(os.path.join(ROOT, "profiles", "plan_1024_tables_batching.txt"), "w") as fh:
        fh.write("\n".join(out) + "\n")
    print("\n".join(out))


def summarize_serve_timers(path):
    """Writes profiles/serve_b24_load0.85_zipf1.1_timers.txt from the JSON
    line of `python3 bench.py --serve 50000 --serve-timers` saved at
    `path`."""
    rec = [json.loads(x) for x in open(path) if x.startswith("{")][-1]["serve"]
    out = ["# Serving loop on a table with timers (persistent cooperative kernel, rounds of lookups | inserts |",
           "# deletes), MI355X, ROCm 7.2",
           f"# table 2^24 buckets x 8 slots at load 0.85 ({rec['stored_keys']:,} keys), every key expiring at "
           f"time {SERVE_NOW0 + SERVE_TTL};",
           f"# server: entries live {SERVE_TTL} units, every lookup that finds an entry renews it;",
           f"# run r at time {SERVE_NOW0} + {SERVE_TICK} (r + 1): every key stays alive; flow universe = "
           "first 100M keys;",
           "# bursts log-uniform in [1, 2048] ops: 0.9 n lookups (Zipf s=1.1 over the universe), 0.1 n inserts of",
           "# new flows, 0.05 n deletes of expired flows (stored keys outside the universe); "
           f"{rec['bursts_per_run']:,} bursts per run;",
           f"# admission budget {rec['budget_ops']} ops per kind; loop grid {rec['grid_blocks']} blocks x 512 threads;",
           "# every lookup, insert status and delete result of every run checked against the ground truth",
           "# command (repository root): python3 bench.py --serve 50000 --serve-timers",
           "# latency = host-observed completion - arrival; us/round = the loop's own clock per phase",
           f"{'offered':>10} {'Glookups/s':>11} {'p50_us':>9} {'p99_us':>9} {'rounds':>7} {'bursts/rnd':>10} "
           f"{'lookup':>7} {'insert':>7} {'delete':>7} {'bound.':>6}"]
    for r in rec["runs"]:
        off = "peak" if r["offered"] == "closed loop (peak)" else f"{int(round(r['offered'] * 100))}%"
        u = r["us_per_round"]
        out.append(f"{off:>10} {r['glookups']:>11.3f} {r['p50_us']:>9.1f} {r['p99_us']:>9.1f} "
                   f"{r['rounds']:>7} {r['bursts_per_round']:>10.0f} {u['lookup']:>7.1f} "
                   f"{u['insert']:>7.1f} {u['delete']:>7.1f} {u['boundary']:>6.1f}")
    sc = rec["scan"]
    out += ["# the peak run submits all bursts at once (closed loop): its latency is queueing behind the budget",
            "# anti-revival scan inside the loop (first time set; 4 GiB table, nothing expired, one",
            f"#   pass, 16 buckets in flight per 16-lane group): {sc['loop_ms']:.2f} ms on the loop's clock, "
            f"{sc['host_ms']:.2f} ms host-observed",
            "# a renewing hit writes nothing when its entry already holds the new time (all rounds of a run",
            "#   share one time); the time store is a relaxed agent-scope atomic",
            "# the same workload without timers: serve_b24_load0.85_zipf1.1.txt"]
    with open(os.path.join(ROOT, "profiles", "serve_b24_load0.85_zipf1.1_timers.txt"), "w") as fh:
        fh.write("\n".join(out) + "\n")
    print("\n".join(out))


def summarize_serve(path, trace_dir=None, counter_dir=None):
    """Writes profiles/serve_b24_load0.85_zipf1.1.txt from the JSON line of
    `python3 bench.py --serve 50000` saved at `path` (and, with trace_dir,
    the loop kernel's line of a rocprofv3 kernel trace of
    `python3 bench.py --serve 20000` under trace_dir/serve_trace; with
    counter_dir, serve_counter_lines of it)."""
    import csv
    rec = [json.loads(x) for x in open(path) if x.startswith("{")][-1]["serve"]
    out = ["# Serving loop (persistent cooperative kernel, rounds of lookups | inserts | deletes), MI355X, ROCm 7.2",
           "# table 2^24 buckets x 8 slots at load 0.85 (114,085,069 keys); flow universe = first 100M keys;",
           "# bursts log-uniform in [1, 2048] ops: 0.9 n lookups (Zipf s=1.1 over the universe), 0.1 n inserts of",
           "# new flows, 0.05 n deletes of expired flows (stored keys outside the universe); "
           f"{rec['bursts_per_run']:,} bursts per run;",
           f"# admission budget {rec['budget_ops']} ops per kind; loop grid {rec['grid_blocks']} blocks x 512 threads;",
           "# every lookup, insert status and delete result of every run checked against the ground truth",
           "# command (repository root): python3 bench.py --serve 50000",
           "# a round's updates are spread over every wavefront (lane 0 of each, then lane 1, ...); an insert",
           "#   whose primary is full searches one- and two-step displacements with all candidates' loads at once;",
           "#   lookups run 4, 2 or 1 per lane per pass in registers (the loop keeps two wavefronts per SIMD);",
           "#   grid barriers: relaxed arrivals after a wait, one system-scope release per block per round",
           "# latency = host-observed completion - arrival; us/round = the loop's own clock per phase (insert:",
           "#   inserts, or inserts and deletes side by side in rounds with few updates; delete: deletes after)",
           f"{'offered':>10} {'Glookups/s':>11} {'p50_us':>9} {'p99_us':>9} {'rounds':>7} {'bursts/rnd':>10} "
           f"{'lookup':>7} {'insert':>7} {'delete':>7} {'bound.':>6}"]
    for r in rec["runs"]:
        off = "peak" if r["offered"] == "closed loop (peak)" else f"{int(round(r['offered'] * 100))}%"
        u = r["us_per_round"]
        out.append(f"{off:>10} {r['glookups']:>11.3f} {r['p50_us']:>9.1f} {r['p99_us']:>9.1f} "
                   f"{r['rounds']:>7} {r['bursts_per_round']:>10.0f} {u['lookup']:>7.1f} "
                   f"{u['insert']:>7.1f} {u['delete']:>7.1f} {u['boundary']:>6.1f}")
    out.append("# the peak run submits all bursts at once (closed loop): its latency is queueing behind the budget")
    pc = rec.get("plain_calls")
    if pc:
        out.append(f"# the same kind of stream ({pc['bursts']} bursts) through the plain batch calls, one "
                   "burst at a time (lookup, insert and delete batch, then a wait on their stream), checked:")
        out.append(f"{'plain-calls':>10} {pc['glookups']:>11.4f} {pc['p50_us']:>9.1f} {pc['p99_us']:>9.1f}")
    if trace_dir:
        rows = [r for r in csv.DictReader(open(os.path.join(trace_dir, "serve_trace", "serve_kernel_stats.csv")))
                if "serve_loop" in r["Name"]]
        for r in rows:
            out.append(f"# kernel trace (rocprofv3 --kernel-trace --stats --output-format csv -d "
                       f"{trace_dir}/serve_trace -o serve -- python3 bench.py --serve 20000):")
            out.append(f"#   serve_loop: {r['Calls']} launch(es), {float(r['TotalDurationNs']) / 1e9:.3f} s "
                       "resident (the loop stays on the device through all runs and idles between them;")
            out.append("#   its per-phase times are the loop's own clocks above)")
    if counter_dir:
        out += serve_counter_lines(counter_dir)
    with open(os.path.join(ROOT, "profiles", "serve_b24_load0.85_zipf1.1.txt"), "w") as fh:
        fh.write("\n".join(out) + "\n")
    print("\n".join(out))


def main():
    args = parse()
    if args.summarize_serve:
        summarize_serve(args.summarize_serve, args.summarize_serve_trace,
                        args.summarize_serve_counters)
        return
    if args.summarize_latency:
        summarize_latency(args.summarize_latency)
        return
    if args.summarize_serve_timers:
        summarize_serve_timers(args.summarize_serve_timers)
        return
    if args.summarize_many_tables:
        summarize_many_tables(args.summarize_many_tables)
        return
    if args.summarize_insert_workload:
        summarize_insert_workload(args.summarize_insert_workload)
        return
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles)
        return
    if args.summarize_plan_profiles:
        summarize_plan_profiles(args.summarize_plan_profiles)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the table is "
                                   "sharded one-per-GPU by design but no multi-GPU path is "
                                   "built", "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_1712_09624_amd import ckpp
    ckpp.load()
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_calib:
        copy_calibration(dev)
        return
    if args.latency:
        print(json.dumps({"latency_ns": latency_probe(dev)}), flush=True)
        return
    if args.burst_latency:
        # the default run's key stream (its table's keys at load 0.9)
        keys = W.distinct_five_tuples(W.keys_at_load(args.log2_buckets, args.load), 1)
        print(json.dumps({"burst_latency": burst_latency(dev, keys, args.log2_buckets)}),
              flush=True)
        return
    if args.serve:
        print(json.dumps({"serve": serve_bench(dev, args.serve, B=args.serve_log2_buckets,
                                                load=args.serve_load, timers=args.serve_timers,
                                                blocks_per_cu=args.serve_blocks_per_cu)}),
              flush=True)
        return
    if args.many_tables:
        shape = tuple(int(x) for x in args.plan_shape.split(",")) if args.plan_shape else None
        print(json.dumps({"many_tables": many_table_bench(dev, args.many_tables, shape=shape)}),
              flush=True)
        return
    if args.insert_workload:
        print(json.dumps({"insert_workload": insert_workload(dev)}), flush=True)
        return
    if args.sweep:
        peak = probe_rand_peak(dev)["128_coop"]["reads_per_s"]
        print(json.dumps({"sweep": sweep(dev, args.lookups, peak), "random_line_peak_per_s": peak}),
              flush=True)
        return

    B, load, n = args.log2_buckets, args.load, args.lookups
    t, keys, vals, build_s = build_table(B, load, 1, dev)
    cfg = t.get_lookup_launch()
    if args.lanes or args.per_lane or args.block or args.blocks_per_cu is not None:
        t.set_lookup_launch(args.lanes or cfg["lanes_per_lookup"],
                            args.per_lane or cfg["lookups_per_lane"],
                            args.block or cfg["block"],
                            cfg["blocks_per_cu"] if args.blocks_per_cu is None else args.blocks_per_cu)
    launch = t.get_lookup_launch()
    stats = t.stats()
    lines = expected_lines(stats)
    log(f"table: live {stats['live']} f_sec {stats['f_sec']:.4f} "
        f"fpr {stats['expected_fpr']:.5f} moved0 {stats['moved_zero_fraction']:.3f}")

    log(f"generating {n} positive and {n} negative lookups")
    pos, _, pos_idx = W.lookup_mix(keys, n, 0.0, 2)
    neg = W.five_tuples(n, 3, stream=W.STREAM_NEGATIVE)
    churn = W.distinct_five_tuples(args.churn, 4, stream=W.STREAM_FRESH)
    dpos, dneg = to_dev(pos, dev), to_dev(neg, dev)
    dchurn = to_dev(churn, dev)
    dchurn_v = to_dev(W.insertion_values(args.churn, 1 << 40).view(np.int64), dev)
    if args.tune:
        from paper_1712_09624_amd import tune
        tuned = {}
        for mode in ("both", "cuckoopp"):
            res = tune.tune(t, [dpos, dneg], mode)
            tuned[mode] = [{"ms_total": r[0], "ms_pos": r[2][0], "ms_neg": r[2][1], **r[1]}
                           for r in res]
            for r in res:
                log(f"tune {mode}: {r[1]} pos {r[2][0]:.3f} ms neg {r[2][1]:.3f} ms")
        print(json.dumps({"tune": tuned}), flush=True)
        launch = t.get_lookup_launch()
    f_pos = torch.empty(n, dtype=torch.uint8, device=dev)
    v_pos = torch.empty(n, dtype=torch.int64, device=dev)
    f_neg = torch.empty(n, dtype=torch.uint8, device=dev)
    v_neg = torch.empty(n, dtype=torch.int64, device=dev)
    st_churn = torch.empty(args.churn, dtype=torch.uint8, device=dev)
    nf_churn = torch.zeros(1, dtype=torch.int64, device=dev)
    d_churn = torch.empty(args.churn, dtype=torch.uint8, device=dev)
    s = torch.cuda.current_stream(dev)

    ev = {k: [] for k in ("ins", "pos", "neg", "del")}

    def step(record):
        marks = [torch.cuda.Event(enable_timing=True) for _ in range(5)] if record else None
        if record:
            marks[0].record(s)
        t.insert(dchurn, dchurn_v, status=st_churn, nfailed=nf_churn)
        if record:
            marks[1].record(s)
        t.lookup(dpos, "cuckoopp", found=f_pos, values=v_pos)
        if record:
            marks[2].record(s)
        t.lookup(dneg, "cuckoopp", found=f_neg, values=v_neg)
        if record:
            marks[3].record(s)
        t.delete(dchurn, found=d_churn)
        if record:
            marks[4].record(s)
            for i, k in enumerate(("ins", "pos", "neg", "del")):
                ev[k].append((marks[i], marks[i + 1]))

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    # exactness spot check of the warm-up results (the tests check it fully)
    chk = np.arange(0, n, max(1, n // 65536))
    fp = f_pos.cpu().numpy()
    vp = v_pos.cpu().numpy().view(np.uint64)
    if not (fp[chk].all() and np.array_equal(vp[chk], vals[pos_idx[chk]])):
        raise RuntimeError("positive lookups returned a wrong answer")
    if f_neg.cpu().numpy()[chk].any() or int(nf_churn.item()):
        raise RuntimeError("negative lookup hit, or churn insert failed")

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms = {k: float(np.mean([a.elapsed_time(b) for a, b in v])) for k, v in ev.items()}
    if not bool(d_churn.all().item()) or int(nf_churn.item()):
        raise RuntimeError("churn keys were not all inserted and deleted")
    ms_per_step = elapsed * 1e3 / args.steps
    value = 2.0 * n / (ms_per_step * 1e-3) / 1e9

    # roofline of the dominant kernel (the Cuckoo++ lookup: two launches per
    # step), on the method's algorithmic bytes: 64-byte lines per lookup
    # (algorithmic_lines_64) plus the 25 streamed bytes, per launch, over the
    # mean launch duration measured with events on the kernels' stream
    alg = algorithmic_lines_64(stats)
    bytes_pos = n * (ALG_LINE * alg["cuckoopp_pos"] + STREAM_BYTES)
    bytes_neg = n * (ALG_LINE * alg["cuckoopp_neg"] + STREAM_BYTES)
    avg_ms = (ms["pos"] + ms["neg"]) / 2
    achieved = (bytes_pos + bytes_neg) / 2 / (avg_ms * 1e-3) / 1e9
    # the same launches counted in the device layout's 128-byte lines (the
    # unit a random miss fills on this GPU; see lines_per_lookup)
    dev_bytes = n * (LINE * (lines["cuckoopp_pos"] + lines["cuckoopp_neg"]) + 2 * STREAM_BYTES) / 2
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "kernel": f"{ckpp.lookup_kernel_name(launch)}<waves={launch['block'] // 64}, Cuckoo++>",
                "algorithmic_bytes_per_launch": (bytes_pos + bytes_neg) / 2,
                "algorithmic_lines_64B": {"pos": alg["cuckoopp_pos"], "neg": alg["cuckoopp_neg"]},
                "avg_launch_ms": avg_ms,
                "device_layout_bytes_per_launch": dev_bytes,
                "frac_128B_granule": dev_bytes / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    tf = os.path.join(ROOT, "profiles", "lookup_traffic.json")
    if os.path.exists(tf):
        with open(tf) as fh:
            tr = json.load(fh)
        if tr.get("source_digest") == lookup_source_digest() and tr.get("launch") == launch:
            roofline["traffic"] = tr["hbm_bytes_per_launch"]
            roofline["traffic_over_algorithmic"] = (tr["hbm_bytes_per_launch"]
                                                    / roofline["algorithmic_bytes_per_launch"])

    stats["f_high"] = stats["high_slots"] / max(1, stats["live"])
    out = {
        "metric": METRIC, "value": value, "unit": "Glookups/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"Cuckoo++ table 2^{B} buckets x 8 slots, load {load}; step = "
                               f"insert {args.churn} + lookup {n} positive + lookup {n} "
                               f"negative + delete {args.churn}",
                   "log2_buckets": B, "load": load, "lookups_per_launch": n,
                   "churn_batch": args.churn, "key_bytes": 16, "value_bytes": 8,
                   "launch": launch, "parallelism": "single GPU"},
        "roofline": roofline,
        "ms": ms,
        "lookups": {
            "cuckoopp_pos_glookups": n / (ms["pos"] * 1e-3) / 1e9,
            "cuckoopp_neg_glookups": n / (ms["neg"] * 1e-3) / 1e9,
            "lines_per_lookup": lines,
            "algorithmic_lines_64B": alg,
        },
        "table": {"live": stats["live"], "f_sec": stats["f_sec"], "f_high": stats["f_high"],
                  "expected_fpr": stats["expected_fpr"],
                  "moved_zero_fraction": stats["moved_zero_fraction"],
                  "build_s": build_s},
    }
    if not args.core_only:
        lk = out["lookups"]
        for mode in ("both", "optimistic"):
            for name, d, fo, vo in (("pos", dpos, f_pos, v_pos), ("neg", dneg, f_neg, v_neg)):
                tms = timed(lambda: t.lookup(d, mode, found=fo, values=vo), 5, dev)
                lk[f"{'plain' if mode == 'both' else mode}_{name}_glookups"] = n / (tms * 1e-3) / 1e9
        for name in ("pos", "neg"):
            lk[f"cuckoopp_over_plain_{name}"] = (lk[f"cuckoopp_{name}_glookups"]
                                                 / lk[f"plain_{name}_glookups"])
        # the plain lookup at its own fastest form (four lanes per lookup: both
        # buckets' lines in flight at once, in registers), so the comparison
        # does not rest on a shape tuned for Cuckoo++
        t.set_lookup_launch(4, 1, 256, 0)
        for name, d, fo, vo in (("pos", dpos, f_pos, v_pos), ("neg", dneg, f_neg, v_neg)):
            tms = timed(lambda: t.lookup(d, "both", found=fo, values=vo), 5, dev)
            rate = n / (tms * 1e-3) / 1e9
            lk[f"plain_four_lanes_{name}_glookups"] = rate
            best = max(rate, lk[f"plain_{name}_glookups"])
            lk[f"cuckoopp_over_best_plain_{name}"] = lk[f"cuckoopp_{name}_glookups"] / best
        t.set_lookup_launch(**launch)
        t.close()
        log("burst latency")
        out["burst_latency"] = burst_latency(dev, keys, B)
        log("tables with timers")
        out["timers"] = timers_leg(dev, B, load, n, dpos, dneg, pos_idx, lk)
        del dpos, dneg, f_pos, v_pos, f_neg, v_neg
        torch.cuda.empty_cache()
        peak = probe_rand_peak(dev)
        out["random_read_peak"] = peak
        p128 = peak["128_coop"]["reads_per_s"]
        out["random_line_peak_per_s"] = p128
        for k in ("cuckoopp_pos", "cuckoopp_neg", "plain_pos", "plain_neg", "optimistic_pos",
                  "optimistic_neg"):
            lk[f"{k}_frac_random_line_peak"] = lk[f"{k}_glookups"] * 1e9 * lines[k] / p128
        roofline["frac_random_line_peak_pos"] = lk["cuckoopp_pos_frac_random_line_peak"]
        roofline["frac_random_line_peak_neg"] = lk["cuckoopp_neg_frac_random_line_peak"]
        out["cache_resident_table"] = cache_resident_table(dev, n, 20)
        out["mall_resident_table"] = cache_resident_table(dev, n, 19)
        if not args.no_cpu_baseline:
            log("timing the oracle on the host")
            out["cpu_baseline"] = cpu_baseline(keys, pos, neg, B, load)
    else:
        t.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
