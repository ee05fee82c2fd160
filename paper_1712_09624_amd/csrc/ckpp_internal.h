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
  uint64_t *d_stats;    // device accumulator of ckpp_stats_t
  ckpp_launch_t lookup_launch;
  int num_cus;
};

namespace ckpp {

constexpr uint32_t kModeCuckoopp = 0;
constexpr uint32_t kModeBoth = 1;
constexpr uint32_t kModeOptimistic = 2;

hipError_t launch_lookup(const ckpp_table *t, const void *d_keys, uint64_t n, uint32_t mode,
                         uint8_t *d_found, uint64_t *d_values, hipStream_t s);
hipError_t launch_insert(const ckpp_table *t, const void *d_keys, const uint64_t *d_values,
                         uint64_t n, uint8_t *d_status, uint64_t *d_nfailed, hipStream_t s);
hipError_t launch_delete(const ckpp_table *t, const void *d_keys, uint64_t n, uint8_t *d_found,
                         hipStream_t s);
hipError_t launch_stats(const ckpp_table *t, uint64_t *d_acc, hipStream_t s);
hipError_t launch_hash(const ckpp_table *t, const void *d_keys, uint64_t n, uint64_t *d_hash,
                       hipStream_t s);
hipError_t launch_fill_zero(void *d, uint64_t bytes, hipStream_t s);
hipError_t launch_probe(const void *d_buf, uint64_t bytes, uint32_t granule, uint64_t nreads,
                        uint32_t per_lane, uint32_t cooperative, uint32_t block, uint32_t grid,
                        uint64_t seed, uint64_t *d_sink, hipStream_t s);

}  // namespace ckpp
