// ckpp_api.hip -- the C ABI: argument checks, device memory, dispatch.

#include <algorithm>
#include <atomic>
#include <new>
#include <stdint.h>
#include <string.h>
#include <thread>
#include <vector>

#include "ckpp_internal.h"

namespace {

using ckpp::DeviceGuard;
using ckpp::dev_status;

using ckpp::kMaxLog2Buckets;
constexpr uint32_t kMaxKicksLimit = 4096;
constexpr uint32_t kMaxPathLanes = 65536;
constexpr uint32_t kAccWords = 128;   // device accumulator words
constexpr uint32_t kAccStats = 7 + CKPP_MOVED_BINS;
constexpr uint32_t kAccRetry = 127;   // retry-bound counter (never cleared)

bool aligned(const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

uint64_t nbuckets(const ckpp_table *t) { return 1ull << t->log2_buckets; }
uint64_t table_bytes(const ckpp_table *t) { return 256ull << t->log2_buckets; }
uint64_t image_bucket_bytes(const ckpp_table *t) { return 64ull << t->log2_buckets; }
uint64_t image_kv_bytes(const ckpp_table *t) { return 256ull << t->log2_buckets; }

// Byte offsets of slot s's key and value within a 256-byte device bucket
// (the layout documented in ckpp_device.h).
uint32_t dev_key_offset(uint32_t s) { return s < 4 ? 32 + 16 * s : 128 + 16 * (s - 4); }
uint32_t dev_value_offset(uint32_t s) { return s < 4 ? 96 + 8 * s : 192 + 8 * (s - 4); }
constexpr uint32_t kDevOther = 224;

// Runs f(lo, hi) over [0, n) split across host threads.
template <class F>
void parallel_range(uint64_t n, F f) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < (1u << 16)) nt = 1;
  std::vector<std::thread> th;
  const uint64_t chunk = (n + nt - 1) / nt;
  for (unsigned i = 0; i < nt; ++i) {
    const uint64_t lo = i * chunk, hi = std::min(n, lo + chunk);
    if (lo < hi) th.emplace_back(f, lo, hi);
  }
  for (auto &x : th) x.join();
}

constexpr uint64_t kValueBits48 = (1ull << 48) - 1ull;

// What an image must satisfy before the library copies it to the device:
// every lock word zero, sec a subset of busy, and for every occupied slot an
// other bucket inside the table (inserts and the scan follow other[] into
// other buckets, so a wild index would send them outside the table's
// memory); on a table with timers, every occupied slot's value below 2^48
// and its reserved word a 16-bit time (the device layout's limit).  The rest
// of the invariants (each entry in one of its two buckets, exact moved
// counters, no filter false negative) are the caller's to keep: lookups on
// an image that breaks them are unspecified but stay inside the table.
bool image_valid(const uint8_t *hb, const uint8_t *hk, uint64_t nb, bool timed) {
  std::atomic<bool> ok{true};
  parallel_range(nb, [=, &ok](uint64_t lo, uint64_t hi) {
    for (uint64_t b = lo; b < hi && ok.load(std::memory_order_relaxed); ++b) {
      const uint8_t *src = hb + 64 * b;
      const uint8_t busy = src[26], sec = src[27];
      uint32_t lock;
      memcpy(&lock, src + 28, 4);
      if (lock != 0u || (sec & ~busy) != 0) {
        ok.store(false);
        break;
      }
      for (uint32_t s = 0; s < 8; ++s) {
        if (!((busy >> s) & 1u)) continue;
        uint32_t other;
        memcpy(&other, src + 32 + 4 * s, 4);
        bool good = other < nb;
        if (timed) {
          const uint8_t *r = hk + 32 * (8 * b + s);
          uint64_t v, pad;
          memcpy(&v, r + 16, 8);
          memcpy(&pad, r + 24, 8);
          good = good && (v >> 48) == 0 && (pad >> 16) == 0;
        }
        if (!good) {
          ok.store(false);
          break;
        }
      }
    }
  });
  return ok.load();
}

// image (64-byte buckets + 32-byte records) -> device layout.  With timers
// the device value word is value | expiration time << 48 (the image keeps
// the time in the record's reserved word); image_valid has checked that the
// occupied slots' values and times fit (a free slot's record, never read,
// keeps only those bits).
void image_to_device(const uint8_t *hb, const uint8_t *hk, uint8_t *dev, uint64_t nb,
                     bool timed) {
  parallel_range(nb, [=](uint64_t lo, uint64_t hi) {
    for (uint64_t b = lo; b < hi; ++b) {
      uint8_t *d = dev + 256 * b;
      const uint8_t *src = hb + 64 * b;
      memcpy(d, src, 32);               // tags, filter, masks, lock
      memcpy(d + kDevOther, src + 32, 32);  // other[8]
      for (uint32_t s = 0; s < 8; ++s) {
        const uint8_t *r = hk + 32 * (8 * b + s);
        memcpy(d + dev_key_offset(s), r, 16);
        uint64_t v, pad;
        memcpy(&v, r + 16, 8);
        memcpy(&pad, r + 24, 8);
        if (timed) v = (v & kValueBits48) | ((pad & 0xffffull) << 48);
        memcpy(d + dev_value_offset(s), &v, 8);
      }
    }
  });
}

// device layout -> image (the records' reserved 8 bytes are written as 0,
// or as the expiration time on a table with timers)
void device_to_image(const uint8_t *dev, uint8_t *hb, uint8_t *hk, uint64_t nb, bool timed) {
  parallel_range(nb, [=](uint64_t lo, uint64_t hi) {
    for (uint64_t b = lo; b < hi; ++b) {
      const uint8_t *d = dev + 256 * b;
      if (hb) {
        memcpy(hb + 64 * b, d, 32);
        memcpy(hb + 64 * b + 32, d + kDevOther, 32);
      }
      if (hk) {
        for (uint32_t s = 0; s < 8; ++s) {
          uint8_t *r = hk + 32 * (8 * b + s);
          memcpy(r, d + dev_key_offset(s), 16);
          uint64_t v;
          memcpy(&v, d + dev_value_offset(s), 8);
          const uint64_t pad = timed ? (v >> 48) : 0ull;
          if (timed) v &= kValueBits48;
          memcpy(r + 16, &v, 8);
          memcpy(r + 24, &pad, 8);
        }
      }
    }
  });
}

bool timed(const ckpp_table *t) { return (t->flags & CKPP_TIMERS) != 0; }

// A refresh time must keep the entry alive at `now` (Sec. 4.2: expiration
// times lie within 1024 units after the current time).

}  // namespace

extern "C" {

const char *ckpp_strerror(int code) {
  switch (code) {
    case CKPP_OK: return "ok";
    case CKPP_EINVAL: return "invalid argument";
    case CKPP_ENOMEM: return "out of device memory";
    case CKPP_EDEVICE: return "HIP runtime error";
    default: return "unknown status";
  }
}

int ckpp_create(ckpp_table **out, uint32_t log2_buckets, uint64_t hash_seed, uint32_t max_kicks,
                uint32_t flags, int device) {
  if (!out) return CKPP_EINVAL;
  *out = nullptr;
  if (log2_buckets < 1 || log2_buckets > kMaxLog2Buckets) return CKPP_EINVAL;
  if (max_kicks > kMaxKicksLimit) return CKPP_EINVAL;
  if (flags & ~(CKPP_PLAIN | CKPP_TIMERS)) return CKPP_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess) return CKPP_EDEVICE;
  if (device < 0 || device >= ndev) return CKPP_EINVAL;
  DeviceGuard g(device);
  if (!g.ok()) return CKPP_EDEVICE;

  ckpp_table *t = new (std::nothrow) ckpp_table();
  if (!t) return CKPP_ENOMEM;
  memset(t, 0, sizeof(*t));
  t->log2_buckets = log2_buckets;
  t->max_kicks = max_kicks;
  t->flags = flags;
  t->device = device;
  t->seed = hash_seed;
  t->retry_limit = ckpp::kMaxRetryLimit;
  t->lookup_launch.lanes_per_lookup = 8;
  t->lookup_launch.lookups_per_lane = 2;
  t->lookup_launch.block = 128;
  t->lookup_launch.blocks_per_cu = 0;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete t;
    return CKPP_EDEVICE;
  }
  t->num_cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
  // lanes of the persistent insert/delete grid: enough to keep every CU busy
  // on large tables, fewer on small ones (they would only contend)
  uint64_t lanes = 8ull << log2_buckets;
  if (lanes < 256) lanes = 256;
  if (lanes > kMaxPathLanes) lanes = kMaxPathLanes;
  t->path_lanes = (uint32_t)lanes;
  // the table's own path scratch: as many lanes as a launch may use while
  // it stays within a small share of the table's memory, at least 4096
  {
    const uint64_t lane_bytes = 4ull * (max_kicks ? max_kicks : 1u);
    uint64_t own = table_bytes(t) / ckpp::kOwnPathShare / lane_bytes;
    if (own > lanes) own = lanes;
    if (own < ckpp::kOwnPathLanesMin) own = ckpp::kOwnPathLanesMin;
    t->own_path_lanes = (uint32_t)own;
  }

  int rc = CKPP_OK;
  if (hipMalloc(&t->d_table, table_bytes(t)) != hipSuccess ||
      hipMalloc(&t->d_stats, kAccWords * sizeof(uint64_t)) != hipSuccess) {
    rc = CKPP_ENOMEM;
  } else if (hipMemset(t->d_table, 0, table_bytes(t)) != hipSuccess ||
             hipMemset(t->d_stats, 0, kAccWords * sizeof(uint64_t)) != hipSuccess ||
             hipDeviceSynchronize() != hipSuccess) {
    rc = CKPP_EDEVICE;
  }
  if (rc != CKPP_OK) {
    (void)hipGetLastError();
    if (t->d_table) (void)hipFree(t->d_table);
    if (t->d_stats) (void)hipFree(t->d_stats);
    delete t;
    return rc;
  }
  *out = t;
  return CKPP_OK;
}

int ckpp_destroy(ckpp_table *t) {
  if (!t) return CKPP_OK;
  DeviceGuard g(t->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(t->d_table);
  (void)hipFree(t->d_stats);
  if (t->d_own_paths) (void)hipFree(t->d_own_paths);
  delete t;
  return CKPP_OK;
}

int ckpp_clear(ckpp_table *t, void *stream) {
  if (!t) return CKPP_EINVAL;
  DeviceGuard g(t->device);
  if (!g.ok()) return CKPP_EDEVICE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return dev_status(ckpp::launch_fill_zero(t->d_table, table_bytes(t), s));
}

namespace {

int insert_common(ckpp_table *t, const void *d_keys, const uint64_t *d_values,
                  const uint16_t *d_expiry, const ckpp::TimerArgs *tm, uint64_t n,
                  uint8_t *d_status, uint64_t *d_nfailed, void *stream) {
  if (n == 0) return CKPP_OK;
  if (!d_keys || !d_values || !aligned(d_keys, 16) || !aligned(d_values, 8)) return CKPP_EINVAL;
  if (tm && (!d_expiry || !aligned(d_expiry, 2))) return CKPP_EINVAL;
  if (d_nfailed && !aligned(d_nfailed, 8)) return CKPP_EINVAL;
  DeviceGuard g(t->device);
  if (!g.ok()) return CKPP_EDEVICE;
  return dev_status(ckpp::launch_insert(t, d_keys, d_values, d_expiry, tm, n, d_status, d_nfailed,
                                        reinterpret_cast<hipStream_t>(stream)));
}

int lookup_common(ckpp_table *t, const void *d_keys, uint64_t n, uint32_t mode,
                  const ckpp::TimerArgs *tm, uint8_t *d_found, uint64_t *d_values, void *stream) {
  if (mode > CKPP_LOOKUP_OPTIMISTIC) return CKPP_EINVAL;
  if (n == 0) return CKPP_OK;
  if (!d_keys || !d_found || !d_values) return CKPP_EINVAL;
  if (!aligned(d_keys, 16) || !aligned(d_values, 8)) return CKPP_EINVAL;
  // a plain table keeps no filter: its default lookup reads both buckets
  if (mode == CKPP_LOOKUP_DEFAULT && (t->flags & CKPP_PLAIN)) mode = CKPP_LOOKUP_BOTH;
  DeviceGuard g(t->device);
  if (!g.ok()) return CKPP_EDEVICE;
  return dev_status(ckpp::launch_lookup(t, d_keys, n, mode, tm, d_found, d_values,
                                        reinterpret_cast<hipStream_t>(stream)));
}

int delete_common(ckpp_table *t, const void *d_keys, uint64_t n, const ckpp::TimerArgs *tm,
                  uint8_t *d_found, void *stream) {
  if (n == 0) return CKPP_OK;
  if (!d_keys || !aligned(d_keys, 16)) return CKPP_EINVAL;
  DeviceGuard g(t->device);
  if (!g.ok()) return CKPP_EDEVICE;
  return dev_status(
      ckpp::launch_delete(t, d_keys, n, tm, d_found, reinterpret_cast<hipStream_t>(stream)));
}

}  // namespace

int ckpp_insert_batch(ckpp_table *t, const void *d_keys, const uint64_t *d_values, uint64_t n,
                      uint8_t *d_status, uint64_t *d_nfailed, void *stream) {
  if (!t || timed(t)) return CKPP_EINVAL;
  return insert_common(t, d_keys, d_values, nullptr, nullptr, n, d_status, d_nfailed, stream);
}

int ckpp_insert_batch_noalloc(ckpp_table *t, const void *d_keys, const uint64_t *d_values,
                              uint64_t n, uint8_t *d_status, uint64_t *d_nfailed, void *stream) {
  if (!t || timed(t)) return CKPP_EINVAL;
  if (n == 0) return CKPP_OK;
  if (!d_keys || !d_values || !aligned(d_keys, 16) || !aligned(d_values, 8)) return CKPP_EINVAL;
  if (d_nfailed && !aligned(d_nfailed, 8)) return CKPP_EINVAL;
  DeviceGuard g(t->device);
  if (!g.ok()) return CKPP_EDEVICE;
  return ckpp::insert_noalloc(t, d_keys, d_values, n, d_status, d_nfailed,
                              reinterpret_cast<hipStream_t>(stream));
}

int ckpp_lookup_batch(ckpp_table *t, const void *d_keys, uint64_t n, uint32_t mode,
                      uint8_t *d_found, uint64_t *d_values, void *stream) {
  if (!t || timed(t)) return CKPP_EINVAL;
  return lookup_common(t, d_keys, n, mode, nullptr, d_found, d_values, stream);
}

int ckpp_delete_batch(ckpp_table *t, const void *d_keys, uint64_t n, uint8_t *d_found,
                      void *stream) {
  if (!t || timed(t)) return CKPP_EINVAL;
  return delete_common(t, d_keys, n, nullptr, d_found, stream);
}

int ckpp_insert_batch_at(ckpp_table *t, const void *d_keys, const uint64_t *d_values,
                         const uint16_t *d_expiry, uint64_t n, uint16_t now, uint8_t *d_status,
                         uint64_t *d_nfailed, void *stream) {
  if (!t || !timed(t)) return CKPP_EINVAL;
  const ckpp::TimerArgs tm{now, 0u, 0u};
  return insert_common(t, d_keys, d_values, d_expiry, &tm, n, d_status, d_nfailed, stream);
}

int ckpp_lookup_batch_at(ckpp_table *t, const void *d_keys, uint64_t n, uint32_t mode,
                         uint16_t now, uint32_t refresh, uint16_t expiry, uint8_t *d_found,
                         uint64_t *d_values, void *stream) {
  if (!t || !timed(t) || refresh > 1u) return CKPP_EINVAL;
  if (refresh && !ckpp::in_window(expiry, now)) return CKPP_EINVAL;
  const ckpp::TimerArgs tm{now, refresh, expiry};
  return lookup_common(t, d_keys, n, mode, &tm, d_found, d_values, stream);
}

int ckpp_delete_batch_at(ckpp_table *t, const void *d_keys, uint64_t n, uint16_t now,
                         uint8_t *d_found, void *stream) {
  if (!t || !timed(t)) return CKPP_EINVAL;
  const ckpp::TimerArgs tm{now, 0u, 0u};
  return delete_common(t, d_keys, n, &tm, d_found, stream);
}

int ckpp_expire_scan(ckpp_table *t, uint16_t now, uint64_t *d_removed, void *stream) {
  if (!t || !timed(t)) return CKPP_EINVAL;
  if (d_removed && !aligned(d_removed, 8)) return CKPP_EINVAL;
  DeviceGuard g(t->device);
  if (!g.ok()) return CKPP_EDEVICE;
  return dev_status(
      ckpp::launch_expire_scan(t, now, d_removed, reinterpret_cast<hipStream_t>(stream)));
}

int ckpp_export(const ckpp_table *t, void *h_buckets, void *h_kv, void *stream) {
  if (!t) return CKPP_EINVAL;
  if (!h_buckets && !h_kv) return CKPP_OK;
  DeviceGuard g(t->device);
  if (!g.ok()) return CKPP_EDEVICE;
  uint8_t *stage = new (std::nothrow) uint8_t[table_bytes(t)];
  if (!stage) return CKPP_ENOMEM;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(stage, t->d_table, table_bytes(t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess)
    device_to_image(stage, static_cast<uint8_t *>(h_buckets), static_cast<uint8_t *>(h_kv),
                    nbuckets(t), timed(t));
  delete[] stage;
  return dev_status(e);
}

int ckpp_check_image(uint32_t log2_buckets, uint32_t flags, const void *h_buckets,
                     const void *h_kv) {
  if (!h_buckets || !h_kv) return CKPP_EINVAL;
  if (log2_buckets < 1 || log2_buckets > kMaxLog2Buckets) return CKPP_EINVAL;
  if (flags & ~(CKPP_PLAIN | CKPP_TIMERS)) return CKPP_EINVAL;
  return image_valid(static_cast<const uint8_t *>(h_buckets), static_cast<const uint8_t *>(h_kv),
                     1ull << log2_buckets, (flags & CKPP_TIMERS) != 0)
             ? CKPP_OK
             : CKPP_EINVAL;
}

int ckpp_import(ckpp_table *t, const void *h_buckets, const void *h_kv, void *stream) {
  if (!t || !h_buckets || !h_kv) return CKPP_EINVAL;
  if (!image_valid(static_cast<const uint8_t *>(h_buckets), static_cast<const uint8_t *>(h_kv),
                   nbuckets(t), timed(t)))
    return CKPP_EINVAL;
  DeviceGuard g(t->device);
  if (!g.ok()) return CKPP_EDEVICE;
  uint8_t *stage = new (std::nothrow) uint8_t[table_bytes(t)];
  if (!stage) return CKPP_ENOMEM;
  image_to_device(static_cast<const uint8_t *>(h_buckets), static_cast<const uint8_t *>(h_kv),
                  stage, nbuckets(t), timed(t));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(t->d_table, stage, table_bytes(t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  delete[] stage;
  return dev_status(e);
}

int ckpp_stats(const ckpp_table *t, ckpp_stats_t *h_out, void *stream) {
  if (!t || !h_out) return CKPP_EINVAL;
  DeviceGuard g(t->device);
  if (!g.ok()) return CKPP_EDEVICE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  uint64_t acc[kAccWords];
  hipError_t e = ckpp::launch_fill_zero(t->d_stats, 16 * ((kAccStats * 8 + 15) / 16), s);
  if (e == hipSuccess) e = ckpp::launch_stats(t, t->d_stats, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(acc, t->d_stats, sizeof(acc), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return CKPP_EDEVICE;
  memset(h_out, 0, sizeof(*h_out));
  h_out->nbuckets = 1ull << t->log2_buckets;
  h_out->live = acc[0];
  h_out->in_secondary = acc[1];
  h_out->bloom_pc_sum = acc[2];
  h_out->bloom_pc2_sum = acc[3];
  h_out->locked = acc[4];
  h_out->high_slots = acc[5];
  h_out->high_slots_secondary = acc[6];
  h_out->retry_exhausted = acc[kAccRetry];
  for (int i = 0; i < CKPP_MOVED_BINS; ++i) h_out->moved_hist[i] = acc[7 + i];
  return CKPP_OK;
}

int ckpp_hash_batch(const ckpp_table *t, const void *d_keys, uint64_t n, uint64_t *d_hash,
                    void *stream) {
  if (!t) return CKPP_EINVAL;
  if (n == 0) return CKPP_OK;
  if (!d_keys || !d_hash || !aligned(d_keys, 16) || !aligned(d_hash, 8)) return CKPP_EINVAL;
  DeviceGuard g(t->device);
  if (!g.ok()) return CKPP_EDEVICE;
  return dev_status(ckpp::launch_hash(t, d_keys, n, d_hash, reinterpret_cast<hipStream_t>(stream)));
}

int ckpp_info(const ckpp_table *t, ckpp_info_t *out) {
  if (!t || !out) return CKPP_EINVAL;
  out->log2_buckets = t->log2_buckets;
  out->max_kicks = t->max_kicks;
  out->flags = t->flags;
  out->device = t->device;
  out->hash_seed = t->seed;
  out->image_bucket_bytes = image_bucket_bytes(t);
  out->image_kv_bytes = image_kv_bytes(t);
  out->device_bytes = table_bytes(t);
  out->d_table = t->d_table;
  return CKPP_OK;
}

int ckpp_set_lookup_launch(ckpp_table *t, const ckpp_launch_t *cfg) {
  if (!t || !cfg) return CKPP_EINVAL;
  const uint32_t lanes = cfg->lanes_per_lookup, per = cfg->lookups_per_lane;
  if (lanes != 1 && lanes != 4 && lanes != 8) return CKPP_EINVAL;
  if (per != 1 && per != 2 && !(per == 4 && lanes == 1)) return CKPP_EINVAL;
  if (cfg->block != 64 && cfg->block != 128 && cfg->block != 256) return CKPP_EINVAL;
  if (cfg->blocks_per_cu > 4096) return CKPP_EINVAL;
  t->lookup_launch = *cfg;
  t->launch_set = true;
  return CKPP_OK;
}

int ckpp_get_lookup_launch(const ckpp_table *t, ckpp_launch_t *cfg) {
  if (!t || !cfg) return CKPP_EINVAL;
  *cfg = t->lookup_launch;
  return CKPP_OK;
}

int ckpp_set_retry_limit(ckpp_table *t, uint32_t limit) {
  if (!t || limit < 1u || limit > ckpp::kMaxRetryLimit) return CKPP_EINVAL;
  t->retry_limit = limit;
  return CKPP_OK;
}

int ckpp_get_retry_limit(const ckpp_table *t, uint32_t *limit) {
  if (!t || !limit) return CKPP_EINVAL;
  *limit = t->retry_limit;
  return CKPP_OK;
}

int ckpp_probe_random_reads(const void *d_buf, uint64_t bytes, uint32_t granule, uint64_t nreads,
                            uint32_t per_lane, uint32_t cooperative, uint32_t block, uint32_t grid,
                            uint64_t seed, uint64_t *d_sink, void *stream) {
  if (!d_buf || !d_sink) return CKPP_EINVAL;
  if (granule != 16 && granule != 32 && granule != 64 && granule != 128) return CKPP_EINVAL;
  if (!aligned(d_buf, granule) || bytes < granule || bytes % granule) return CKPP_EINVAL;
  if (per_lane != 1 && per_lane != 2 && per_lane != 4 && per_lane != 8) return CKPP_EINVAL;
  if (cooperative > 1) return CKPP_EINVAL;
  if (block != 64 && block != 128 && block != 256) return CKPP_EINVAL;
  if (grid == 0 || !aligned(d_sink, 8)) return CKPP_EINVAL;
  if (nreads == 0) return CKPP_OK;
  return dev_status(ckpp::launch_probe(d_buf, bytes, granule, nreads, per_lane, cooperative, block,
                                       grid, seed, d_sink, reinterpret_cast<hipStream_t>(stream)));
}

int ckpp_probe_latency(void *d_buf, uint64_t bytes, uint32_t kind, uint32_t steps, uint64_t seed,
                       uint64_t *d_out, void *stream) {
  if (!d_buf || !d_out || !aligned(d_buf, 256) || !aligned(d_out, 8)) return CKPP_EINVAL;
  if (bytes < 256 || bytes % 256 || kind > 6 || steps == 0) return CKPP_EINVAL;
  return dev_status(ckpp::launch_latency(d_buf, bytes, kind, steps, seed, d_out,
                                         reinterpret_cast<hipStream_t>(stream)));
}

}  // extern "C"
