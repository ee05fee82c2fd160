// ckpp_update.hip -- batched insert and delete kernels (gfx950): one lane
// per key at a time on a persistent grid; the per-key state machines are in
// ckpp_update_dev.h.

#include <mutex>

#include "ckpp_update_dev.h"

namespace ckpp {
namespace {

// Cuckoo-path scratch of ckpp_insert_batch_noalloc: a fixed array in each
// device's memory, held for the life of the process.  Host code never uses
// its name as an address: the device address comes from
// hipGetSymbolAddress, once per device (scratch_on).
constexpr uint64_t kScratchBytes = 8ull << 20;
// Batches of at most this many keys run one key per wavefront (its lane 0):
// a wavefront runs its lanes' updates in lockstep, so a few keys side by
// side in one wavefront take several times as long as one key alone
// (measured on MI355X: an insert 2.7 us alone, 9.1 us for 8 lanes of one
// wavefront).
constexpr uint64_t kSpreadKeys = 1024;

// The key slots of a launch: its lanes, or with `spread` its wavefronts
// (lane 0 of each; false for the other lanes, which have nothing to do).
__device__ __forceinline__ bool worker_of(bool spread, uint64_t &worker, uint64_t &nworkers) {
  const uint64_t lane = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t nlanes = (uint64_t)gridDim.x * blockDim.x;
  if (!spread) {
    worker = lane;
    nworkers = nlanes;
    return true;
  }
  worker = lane >> 6;
  nworkers = nlanes >> 6;
  return (threadIdx.x & 63u) == 0u;
}
static __device__ __align__(256) uint32_t scratch[kScratchBytes / sizeof(uint32_t)];

// TIMED: the table has timers; expiry[i] is key i's expiration time and
// `now` the current time (Sec. 4.2).
template <bool TIMED>
__global__ void __launch_bounds__(256)
    insert_kernel(uint8_t *bk, const uint4 *__restrict__ keys,
                  const uint64_t *__restrict__ vals, const uint16_t *__restrict__ expiry,
                  uint32_t now, uint64_t n, uint32_t log2b, uint64_t seed,
                  uint32_t max_kicks, uint32_t plain_flag, uint32_t spin_limit, uint32_t *paths,
                  uint8_t *__restrict__ status, unsigned long long *nfailed,
                  unsigned long long *nspin, uint32_t spread) {
  const bool plain = plain_flag != 0u;
  uint64_t worker, nworkers;
  if (!worker_of(spread != 0u, worker, nworkers)) return;
  uint32_t *path = paths + worker * (uint64_t)(max_kicks ? max_kicks : 1u);
  for (uint64_t i = worker; i < n; i += nworkers) {
    const InsertOutcome o = insert_one<TIMED>(bk, keys[i], vals[i], log2b, seed, max_kicks, plain,
                                              path, spin_limit, TIMED ? expiry[i] : 0u, now);
    if (status) status[i] = (uint8_t)o.status;
    if (o.status == CKPP_FAILED && nfailed) atomicAdd(nfailed, 1ull);
    if (o.spun && nspin) atomicAdd(nspin, 1ull);
  }
}

template <bool TIMED>
__global__ void __launch_bounds__(256)
    delete_kernel(uint8_t *bk, const uint4 *__restrict__ keys, uint64_t n, uint32_t now,
                  uint32_t log2b, uint64_t seed, uint32_t plain_flag, uint32_t spin_limit,
                  uint8_t *__restrict__ found, unsigned long long *nspin, uint32_t spread) {
  const bool plain = plain_flag != 0u;
  uint64_t worker, nworkers;
  if (!worker_of(spread != 0u, worker, nworkers)) return;
  for (uint64_t i = worker; i < n; i += nworkers) {
    bool spun = false;
    const int r = delete_one<TIMED>(bk, keys[i], log2b, seed, plain, spin_limit, &spun, now);
    if (spun && nspin) atomicAdd(nspin, 1ull);
    if (found) found[i] = (uint8_t)r;
  }
}

// Anti-revival scan (Sec. 4.2): every bucket removes its expired entries,
// with the counter and filter maintenance of a delete (expire_slots_pass:
// the table is read as a stream, 16 lanes per bucket, a wavefront reading
// four consecutive buckets, 1 KiB, per instruction).
__global__ void __launch_bounds__(256)
    expire_slots_kernel(uint8_t *bk, uint64_t nb, uint32_t now, uint32_t plain_flag,
                        unsigned long long *removed) {
  const uint64_t count =
      expire_slots_pass(bk, nb, now, plain_flag != 0u, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x,
                        (uint64_t)gridDim.x * blockDim.x);
  if (count && removed) atomicAdd(removed, (unsigned long long)count);
}

}  // namespace

hipError_t launch_insert(const ckpp_table *t, const void *d_keys, const uint64_t *d_values,
                         const uint16_t *d_expiry, const TimerArgs *timers, uint64_t n,
                         uint8_t *d_status, uint64_t *d_nfailed, hipStream_t s) {
  const bool spread = n <= kSpreadKeys;
  const uint64_t lanes = spread ? 64u * n : n < t->path_lanes ? n : t->path_lanes;
  const uint32_t block = 256;
  const uint32_t grid = (uint32_t)((lanes + block - 1) / block);
  // cuckoo-path scratch of this batch, one path of max_kicks entries per
  // key slot (a lane, or a wavefront when spread): the table's own buffer
  // when it is large enough, else stream-ordered from the device's pool
  const uint64_t per_lane = (uint64_t)(t->max_kicks ? t->max_kicks : 1u);
  const uint64_t slots = (uint64_t)grid * (spread ? block / 64u : block);
  const uint64_t words = slots * per_lane;
  uint32_t *paths = nullptr;
  const bool own = slots <= t->own_path_lanes;
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
                       plain, t->retry_limit, paths, d_status, nfailed, nspin, spread ? 1u : 0u);
  else
    hipLaunchKernelGGL(insert_kernel<false>, dim3(grid), dim3(block), 0, s, t->d_table, keys,
                       d_values, nullptr, 0u, n, t->log2_buckets, t->seed, t->max_kicks, plain,
                       t->retry_limit, paths, d_status, nfailed, nspin, spread ? 1u : 0u);
  e = hipGetLastError();
  if (own) return e;
  const hipError_t f = hipFreeAsync(paths, s);
  return e != hipSuccess ? e : f;
}

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
uint32_t *g_scratch_ptr[kMaxScratchDevices];

// Device address of `scratch` on the current device `dev`, looked up once
// per device with that device current; null if the lookup fails.
uint32_t *scratch_on(int dev) {
  if (dev < 0 || dev >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[dev] = static_cast<uint32_t *>(p);
  }
  return g_scratch_ptr[dev];
}

}  // namespace

// The insert of launch_insert with its path scratch in `scratch`: at most
// as many lanes as fit kScratchBytes (whole blocks of 256), no allocation.
int insert_noalloc(const ckpp_table *t, const void *d_keys, const uint64_t *d_values, uint64_t n,
                   uint8_t *d_status, uint64_t *d_nfailed, hipStream_t s) {
  const uint64_t per_lane = (uint64_t)(t->max_kicks ? t->max_kicks : 1u);
  const uint32_t block = 256;
  const uint64_t fit = kScratchBytes / (per_lane * sizeof(uint32_t)) / block * block;
  if (fit == 0) return CKPP_EINVAL;  // a path longer than the whole array
  uint32_t *paths = scratch_on(t->device);
  if (!paths) return CKPP_EDEVICE;
  uint64_t lanes = n < t->path_lanes ? n : t->path_lanes;
  if (lanes > fit) lanes = fit;
  const uint32_t grid = (uint32_t)((lanes + block - 1) / block);
  unsigned long long *nspin = reinterpret_cast<unsigned long long *>(t->d_stats) + 127;
  const uint32_t plain = (t->flags & CKPP_PLAIN) ? 1u : 0u;
  hipLaunchKernelGGL(insert_kernel<false>, dim3(grid), dim3(block), 0, s, t->d_table,
                     reinterpret_cast<const uint4 *>(d_keys), d_values, nullptr, 0u, n,
                     t->log2_buckets, t->seed, t->max_kicks, plain, t->retry_limit, paths,
                     d_status, reinterpret_cast<unsigned long long *>(d_nfailed), nspin, 0u);
  return dev_status(hipGetLastError());
}

hipError_t launch_delete(const ckpp_table *t, const void *d_keys, uint64_t n,
                         const TimerArgs *timers, uint8_t *d_found, hipStream_t s) {
  const bool spread = n <= kSpreadKeys;
  const uint64_t lanes = spread ? 64u * n : n < t->path_lanes ? n : t->path_lanes;
  const uint32_t block = 256;
  const uint32_t grid = (uint32_t)((lanes + block - 1) / block);
  unsigned long long *nspin = reinterpret_cast<unsigned long long *>(t->d_stats) + 127;
  const uint32_t plain = (t->flags & CKPP_PLAIN) ? 1u : 0u;
  const uint4 *keys = reinterpret_cast<const uint4 *>(d_keys);
  if (timers)
    hipLaunchKernelGGL(delete_kernel<true>, dim3(grid), dim3(block), 0, s, t->d_table, keys, n,
                       timers->now, t->log2_buckets, t->seed, plain, t->retry_limit, d_found, nspin,
                       spread ? 1u : 0u);
  else
    hipLaunchKernelGGL(delete_kernel<false>, dim3(grid), dim3(block), 0, s, t->d_table, keys, n,
                       0u, t->log2_buckets, t->seed, plain, t->retry_limit, d_found, nspin,
                       spread ? 1u : 0u);
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
  return hipGetLastError();
}

}  // namespace ckpp
