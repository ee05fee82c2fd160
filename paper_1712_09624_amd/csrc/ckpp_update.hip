// ckpp_update.hip -- batched insert and delete kernels (gfx950): one lane
// per key at a time on a persistent grid; the per-key state machines are in
// ckpp_update_dev.h.

#include "ckpp_update_dev.h"

namespace ckpp {
namespace {

// TIMED: the table has timers; expiry[i] is key i's expiration time and
// `now` the current time (Sec. 4.2).
template <bool TIMED>
__global__ void __launch_bounds__(256)
    insert_kernel(uint8_t *bk, const uint4 *__restrict__ keys,
                  const uint64_t *__restrict__ vals, const uint16_t *__restrict__ expiry,
                  uint32_t now, uint64_t n, uint32_t log2b, uint64_t seed,
                  uint32_t max_kicks, uint32_t plain_flag, uint32_t *paths,
                  uint8_t *__restrict__ status, unsigned long long *nfailed,
                  unsigned long long *nspin) {
  const bool plain = plain_flag != 0u;
  const uint64_t lane = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t nlanes = (uint64_t)gridDim.x * blockDim.x;
  uint32_t *path = paths + lane * (uint64_t)(max_kicks ? max_kicks : 1u);
  for (uint64_t i = lane; i < n; i += nlanes) {
    const InsertOutcome o = insert_one<TIMED>(bk, keys[i], vals[i], log2b, seed, max_kicks, plain,
                                              path, TIMED ? expiry[i] : 0u, now);
    if (status) status[i] = (uint8_t)o.status;
    if (o.status == CKPP_FAILED && nfailed) atomicAdd(nfailed, 1ull);
    if (o.spun && nspin) atomicAdd(nspin, 1ull);
  }
}

template <bool TIMED>
__global__ void __launch_bounds__(256)
    delete_kernel(uint8_t *bk, const uint4 *__restrict__ keys, uint64_t n, uint32_t now,
                  uint32_t log2b, uint64_t seed, uint32_t plain_flag,
                  uint8_t *__restrict__ found, unsigned long long *nspin) {
  const bool plain = plain_flag != 0u;
  const uint64_t lane = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t nlanes = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = lane; i < n; i += nlanes) {
    bool spun = false;
    const int r = delete_one<TIMED>(bk, keys[i], log2b, seed, plain, &spun, now);
    if (spun && nspin) atomicAdd(nspin, 1ull);
    if (found) found[i] = (uint8_t)r;
  }
}

// Anti-revival scan (Sec. 4.2), first kernel: every bucket removes its
// expired entries.  The table is read as a stream: 16 neighbouring lanes
// read one bucket's 256 bytes, one 16-byte quarter each (a wavefront reads
// four consecutive buckets per instruction, 1 KiB, fully coalesced).  Lane
// 1 of the group holds the metadata word, lanes 6, 7, 12 and 13 the value
// words (two slots each, the expiration time in the high 16 bits), lanes 14
// and 15 the other buckets of the slots; the group shares them through
// cross-lane reads.  Only the group's lane 0 changes the bucket's busy and
// sec bits (an atomic AND); the moved counter of the primary bucket of a
// removed entry that sat in its secondary drops by one through an atomic
// subtraction on that bucket's meta word (the counter is its low 16 bits
// and is at least 1 while the entry is counted there), done by the lane
// that holds the entry's other bucket, so no lock is needed.  The filters
// of counters that reach zero are emptied by the second kernel.
__global__ void __launch_bounds__(256)
    expire_slots_kernel(uint8_t *bk, uint64_t nb, uint32_t now, uint32_t plain_flag,
                        unsigned long long *removed) {
  const bool plain = plain_flag != 0u;
  const uint32_t lane = threadIdx.x & 63u, r = lane & 15u, g0 = lane & 48u;
  const uint64_t groups = (uint64_t)gridDim.x * (blockDim.x / 16u);
  uint64_t count = 0;
  for (uint64_t b = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / 16u; b < nb;
       b += groups) {
    const uint4 q = reinterpret_cast<const uint4 *>(bucket_ptr(bk, (uint32_t)b))[r];
    const uint32_t meta = (uint32_t)__shfl((int)q.z, (int)(g0 + 1u));
    // expired bits of this lane's two value words (lanes 6, 7, 12, 13)
    uint32_t mine = 0u;
    const uint32_t s0 = r == 6u ? 0u : r == 7u ? 2u : r == 12u ? 4u : 6u;
    if (r == 6u || r == 7u || r == 12u || r == 13u) {
      if ((((q.y >> 16) - now) & 0xffffu) >= kMaxDelay) mine |= 1u << s0;
      if ((((q.w >> 16) - now) & 0xffffu) >= kMaxDelay) mine |= 2u << s0;
    }
    const uint32_t exp = meta_busy(meta) &
                         ((uint32_t)__shfl((int)mine, (int)(g0 + 6u)) |
                          (uint32_t)__shfl((int)mine, (int)(g0 + 7u)) |
                          (uint32_t)__shfl((int)mine, (int)(g0 + 12u)) |
                          (uint32_t)__shfl((int)mine, (int)(g0 + 13u)));
    if (!exp) continue;
    if (r == 0u) {
      __hip_atomic_fetch_and(meta_ptr(bk, (uint32_t)b).p, ~((exp << 16) | (exp << 24)),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      count += (uint64_t)__builtin_popcount(exp);
    }
    if (!plain && (r == 14u || r == 15u)) {
      const uint32_t base = r == 14u ? 0u : 4u;
      const uint32_t oth[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (uint32_t k = 0; k < 4; ++k) {
        const uint32_t y = oth[k];
        if (((exp & meta_sec(meta)) >> (base + k)) & 1u && y < nb)  // y < nb: always, on a
                                                                   // table that keeps its invariants
          __hip_atomic_fetch_sub(meta_ptr(bk, y).p, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
  if (count && removed) atomicAdd(removed, (unsigned long long)count);
}

// Second kernel: a bucket whose moved counter is zero has an empty filter
// (Sec. 4.1: the filter is reset when its counter returns to zero).
__global__ void __launch_bounds__(256) expire_filters_kernel(uint8_t *bk, uint64_t nb) {
  for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb;
       b += (uint64_t)gridDim.x * blockDim.x) {
    if (meta_moved(*meta_ptr(bk, (uint32_t)b)) == 0u && *bloom_ptr(bk, (uint32_t)b) != 0ull)
      *bloom_ptr(bk, (uint32_t)b) = 0ull;
  }
}

}  // namespace

hipError_t launch_insert(const ckpp_table *t, const void *d_keys, const uint64_t *d_values,
                         const uint16_t *d_expiry, const TimerArgs *timers, uint64_t n,
                         uint8_t *d_status, uint64_t *d_nfailed, hipStream_t s) {
  const uint64_t lanes = n < t->path_lanes ? n : t->path_lanes;
  const uint32_t block = 256;
  const uint32_t grid = (uint32_t)((lanes + block - 1) / block);
  // cuckoo-path scratch of this batch, one path of max_kicks entries per
  // launched lane: the table's own buffer when it is large enough, else
  // stream-ordered from the device's pool
  const uint64_t per_lane = (uint64_t)(t->max_kicks ? t->max_kicks : 1u);
  const uint64_t words = (uint64_t)grid * block * per_lane;
  uint32_t *paths = nullptr;
  const bool own = (uint64_t)grid * block <= t->own_path_lanes;
  hipError_t e = hipSuccess;
  if (own) {
    ckpp_table *tm = const_cast<ckpp_table *>(t);
    if (!tm->d_own_paths)
      e = hipMalloc(reinterpret_cast<void **>(&tm->d_own_paths),
                    (uint64_t)t->own_path_lanes * per_lane * sizeof(uint32_t));
    paths = tm->d_own_paths;
  } else {
    e = hipMallocAsync(reinterpret_cast<void **>(&paths), words * sizeof(uint32_t), s);
  }
  if (e != hipSuccess) return e;
  unsigned long long *nspin = reinterpret_cast<unsigned long long *>(t->d_stats) + 127;
  const uint32_t plain = (t->flags & CKPP_PLAIN) ? 1u : 0u;
  unsigned long long *nfailed = reinterpret_cast<unsigned long long *>(d_nfailed);
  const uint4 *keys = reinterpret_cast<const uint4 *>(d_keys);
  if (timers)
    hipLaunchKernelGGL(insert_kernel<true>, dim3(grid), dim3(block), 0, s, t->d_table, keys,
                       d_values, d_expiry, timers->now, n, t->log2_buckets, t->seed, t->max_kicks,
                       plain, paths, d_status, nfailed, nspin);
  else
    hipLaunchKernelGGL(insert_kernel<false>, dim3(grid), dim3(block), 0, s, t->d_table, keys,
                       d_values, nullptr, 0u, n, t->log2_buckets, t->seed, t->max_kicks, plain,
                       paths, d_status, nfailed, nspin);
  e = hipGetLastError();
  if (own) return e;
  const hipError_t f = hipFreeAsync(paths, s);
  return e != hipSuccess ? e : f;
}

hipError_t launch_delete(const ckpp_table *t, const void *d_keys, uint64_t n,
                         const TimerArgs *timers, uint8_t *d_found, hipStream_t s) {
  const uint64_t lanes = n < t->path_lanes ? n : t->path_lanes;
  const uint32_t block = 256;
  const uint32_t grid = (uint32_t)((lanes + block - 1) / block);
  unsigned long long *nspin = reinterpret_cast<unsigned long long *>(t->d_stats) + 127;
  const uint32_t plain = (t->flags & CKPP_PLAIN) ? 1u : 0u;
  const uint4 *keys = reinterpret_cast<const uint4 *>(d_keys);
  if (timers)
    hipLaunchKernelGGL(delete_kernel<true>, dim3(grid), dim3(block), 0, s, t->d_table, keys, n,
                       timers->now, t->log2_buckets, t->seed, plain, d_found, nspin);
  else
    hipLaunchKernelGGL(delete_kernel<false>, dim3(grid), dim3(block), 0, s, t->d_table, keys, n,
                       0u, t->log2_buckets, t->seed, plain, d_found, nspin);
  return hipGetLastError();
}

hipError_t launch_expire_scan(const ckpp_table *t, uint32_t now, uint64_t *d_removed,
                              hipStream_t s) {
  const uint64_t nb = 1ull << t->log2_buckets;
  const uint32_t block = 256;
  // 16 lanes per bucket; a persistent grid of 16 blocks per compute unit
  uint64_t grid = (16u * nb + block - 1) / block;
  const uint64_t cap = 16ull * (uint64_t)t->num_cus;
  if (grid > cap) grid = cap;
  hipLaunchKernelGGL(expire_slots_kernel, dim3((uint32_t)grid), dim3(block), 0, s, t->d_table, nb,
                     now, (t->flags & CKPP_PLAIN) ? 1u : 0u,
                     reinterpret_cast<unsigned long long *>(d_removed));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(expire_filters_kernel, dim3((uint32_t)grid), dim3(block), 0, s, t->d_table,
                     nb);
  return hipGetLastError();
}

}  // namespace ckpp
