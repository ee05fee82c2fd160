// ckpp_internal.h -- host-side table object and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ckpp.h"

struct ckpp_table {
  uint32_t log2_buckets;
  uint32_t max_kicks;
  uint32_t flags;
  int device;
  uint64_t seed;
  uint8_t *d_table;     // 256 * 2^B bytes: bucket b at 256 * b (ckpp_device.h)
  uint32_t path_lanes;  // lanes of the persistent insert grid
  uint32_t *d_own_paths;    // the table's own cuckoo-path scratch (own_path_lanes
                            // lanes), allocated on the first batch that fits it
  uint32_t own_path_lanes;
  uint64_t *d_stats;    // device accumulator of ckpp_stats_t
  uint32_t retry_limit; // attempts per key on contended locks (ckpp_set_retry_limit)
  ckpp_launch_t lookup_launch;
  bool launch_set;      // a caller set lookup_launch (else small batches take their own shape)
  int num_cus;
};

namespace ckpp {

// Insert batches take their cuckoo-path scratch (max_kicks words per
// launched lane) from a buffer of the table's own, kept for its lifetime,
// when it fits: the stream-ordered pool's allocate/free pair costs tens of
// microseconds of host time per batch, during which the device idles.  The
// buffer holds at least kOwnPathLanesMin lanes, and more up to the launch's
// maximum while it stays within 1/kOwnPathShare of the table's own memory;
// larger batches use the pool.
constexpr uint32_t kOwnPathLanesMin = 4096;
constexpr uint64_t kOwnPathShare = 32;

// One work item of a plan: lookups [start, start + count) of the
// concatenated key batch, all of one table, with that table's parameters
// (so a wave needs a single descriptor load per item).
struct PlanItem {
  const uint4 *tab;  // the table's buckets
  uint64_t seed;     // its hash seed
  uint64_t start;
  uint32_t count;
  uint32_t log2b;    // log2 of its bucket count
  uint32_t mode;     // kMode* of its lookups
  uint32_t table;    // index of the table in the plan
};

// Largest table: 2^29 buckets (128 GiB, 2^32 slots); bucket indices fit in
// 29 bits.
constexpr uint32_t kMaxLog2Buckets = 29;

// Attempts an insert or delete makes on contended bucket locks before it
// gives up with CKPP_RETRY: the default and largest retry limit.
constexpr uint32_t kMaxRetryLimit = 1u << 20;

constexpr uint32_t kModeCuckoopp = 0;
constexpr uint32_t kModeBoth = 1;
constexpr uint32_t kModeOptimistic = 2;
// PlanItem::mode: the lookup mode in the low byte, and this flag on a table
// with timers.
constexpr uint32_t kPlanModeMask = 0xffu;
constexpr uint32_t kPlanItemTimed = 0x100u;

// Blocks of a launch over n items, per_block items per block: at most
// blocks_per_cu per compute unit (0: no cap) and at most 2^31 - 1.
inline uint64_t capped_grid(uint64_t n, uint64_t per_block, uint32_t blocks_per_cu, int num_cus) {
  uint64_t grid = (n + per_block - 1) / per_block;
  if (blocks_per_cu) {
    const uint64_t cap = (uint64_t)blocks_per_cu * (uint64_t)num_cus;
    if (grid > cap) grid = cap;
  }
  return grid > 0x7fffffffull ? 0x7fffffffull : grid;
}

// A refreshing lookup's new expiration time lies in [now, now + 1023] mod
// 2^16, so the entry it writes is alive at `now` (Sec. 4.2).
inline bool in_window(uint32_t expiry, uint32_t now) { return ((expiry - now) & 0xffffu) < 1024u; }

// Timers of a batch on a table with timers (Sec. 4.2): the current time;
// for lookups, whether a hit sets the entry's expiration time to `expiry`.
struct TimerArgs {
  uint32_t now;
  uint32_t refresh;
  uint32_t expiry;
};

// timers: null on a table without timers.
hipError_t launch_lookup(const ckpp_table *t, const void *d_keys, uint64_t n, uint32_t mode,
                         const TimerArgs *timers, uint8_t *d_found, uint64_t *d_values,
                         hipStream_t s);
// One launch of the plan's persistent lookup kernel over its items.
// d_ctr: two u32 counters (next item, finished waves), zero before the
// launch and zero again after it.  two_buffers: some table uses the
// pessimistic mode.  timers: the launch's time, for the items flagged
// kPlanItemTimed (null: no item is).
hipError_t launch_plan(const PlanItem *d_items, uint32_t nitems, uint32_t *d_ctr, bool two_buffers,
                       const TimerArgs *timers, const ckpp_plan_launch_t &L, int num_cus,
                       const void *d_keys, uint8_t *d_found, uint64_t *d_values, hipStream_t s);
// d_expiry and timers: null on a table without timers.
hipError_t launch_insert(const ckpp_table *t, const void *d_keys, const uint64_t *d_values,
                         const uint16_t *d_expiry, const TimerArgs *timers, uint64_t n,
                         uint8_t *d_status, uint64_t *d_nfailed, hipStream_t s);
hipError_t launch_delete(const ckpp_table *t, const void *d_keys, uint64_t n,
                         const TimerArgs *timers, uint8_t *d_found, hipStream_t s);
// The insert without any allocation (ckpp_insert_batch_noalloc): returns a
// CKPP_* status.
int insert_noalloc(const ckpp_table *t, const void *d_keys, const uint64_t *d_values, uint64_t n,
                   uint8_t *d_status, uint64_t *d_nfailed, hipStream_t s);
// Removes every entry expired at `now` (one pass over the table).
hipError_t launch_expire_scan(const ckpp_table *t, uint32_t now, uint64_t *d_removed,
                              hipStream_t s);
hipError_t launch_stats(const ckpp_table *t, uint64_t *d_acc, hipStream_t s);
hipError_t launch_hash(const ckpp_table *t, const void *d_keys, uint64_t n, uint64_t *d_hash,
                       hipStream_t s);
hipError_t launch_fill_zero(void *d, uint64_t bytes, hipStream_t s);
// The dependent-access latency probe (ckpp_probe_latency).
hipError_t launch_latency(void *d_buf, uint64_t bytes, uint32_t kind, uint32_t steps,
                          uint64_t seed, uint64_t *d_out, hipStream_t s);
hipError_t launch_probe(const void *d_buf, uint64_t bytes, uint32_t granule, uint64_t nreads,
                        uint32_t per_lane, uint32_t cooperative, uint32_t block, uint32_t grid,
                        uint64_t seed, uint64_t *d_sink, hipStream_t s);

// Makes a device current for the duration of a call.
class DeviceGuard {
 public:
  explicit DeviceGuard(int dev) : prev_(-1), ok_(true) {
    if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
    if (prev_ != dev) ok_ = hipSetDevice(dev) == hipSuccess;
    else prev_ = -1;
  }
  ~DeviceGuard() {
    if (prev_ >= 0) (void)hipSetDevice(prev_);
  }
  bool ok() const { return ok_; }

 private:
  int prev_;
  bool ok_;
};

inline int dev_status(hipError_t e) {
  if (e == hipSuccess) return CKPP_OK;
  return e == hipErrorOutOfMemory ? CKPP_ENOMEM : CKPP_EDEVICE;
}

}  // namespace ckpp
