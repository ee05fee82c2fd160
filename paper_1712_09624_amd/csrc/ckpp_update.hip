// ckpp_update.hip -- batched insert and delete kernels (gfx950): one lane
// per key at a time on a persistent grid; the per-key state machines are in
// ckpp_update_dev.h.

#include "ckpp_update_dev.h"

namespace ckpp {
namespace {

__global__ void __launch_bounds__(256)
    insert_kernel(uint8_t *bk, const uint4 *__restrict__ keys,
                  const uint64_t *__restrict__ vals, uint64_t n, uint32_t log2b, uint64_t seed,
                  uint32_t max_kicks, uint32_t plain_flag, uint32_t *paths,
                  uint8_t *__restrict__ status, unsigned long long *nfailed,
                  unsigned long long *nspin) {
  const bool plain = plain_flag != 0u;
  const uint64_t lane = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t nlanes = (uint64_t)gridDim.x * blockDim.x;
  uint32_t *path = paths + lane * (uint64_t)(max_kicks ? max_kicks : 1u);
  for (uint64_t i = lane; i < n; i += nlanes) {
    const InsertOutcome o = insert_one(bk, keys[i], vals[i], log2b, seed, max_kicks, plain, path);
    if (status) status[i] = (uint8_t)o.status;
    if (o.status == CKPP_FAILED && nfailed) atomicAdd(nfailed, 1ull);
    if (o.spun && nspin) atomicAdd(nspin, 1ull);
  }
}

__global__ void __launch_bounds__(256)
    delete_kernel(uint8_t *bk, const uint4 *__restrict__ keys, uint64_t n,
                  uint32_t log2b, uint64_t seed, uint32_t plain_flag,
                  uint8_t *__restrict__ found, unsigned long long *nspin) {
  const bool plain = plain_flag != 0u;
  const uint64_t lane = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t nlanes = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = lane; i < n; i += nlanes) {
    bool spun = false;
    const int r = delete_one(bk, keys[i], log2b, seed, plain, &spun);
    if (spun && nspin) atomicAdd(nspin, 1ull);
    if (found) found[i] = (uint8_t)r;
  }
}

}  // namespace

hipError_t launch_insert(const ckpp_table *t, const void *d_keys, const uint64_t *d_values,
                         uint64_t n, uint8_t *d_status, uint64_t *d_nfailed, hipStream_t s) {
  const uint64_t lanes = n < t->path_lanes ? n : t->path_lanes;
  const uint32_t block = 256;
  const uint32_t grid = (uint32_t)((lanes + block - 1) / block);
  // cuckoo-path scratch of this batch, stream-ordered from the device's pool:
  // one path of max_kicks entries per launched lane
  const uint64_t words = (uint64_t)grid * block * (uint64_t)(t->max_kicks ? t->max_kicks : 1u);
  uint32_t *paths = nullptr;
  hipError_t e = hipMallocAsync(reinterpret_cast<void **>(&paths), words * sizeof(uint32_t), s);
  if (e != hipSuccess) return e;
  unsigned long long *nspin = reinterpret_cast<unsigned long long *>(t->d_stats) + 127;
  hipLaunchKernelGGL(insert_kernel, dim3(grid), dim3(block), 0, s, t->d_table,
                     reinterpret_cast<const uint4 *>(d_keys), d_values, n, t->log2_buckets,
                     t->seed, t->max_kicks, (t->flags & CKPP_PLAIN) ? 1u : 0u, paths,
                     d_status, reinterpret_cast<unsigned long long *>(d_nfailed), nspin);
  e = hipGetLastError();
  const hipError_t f = hipFreeAsync(paths, s);
  return e != hipSuccess ? e : f;
}

hipError_t launch_delete(const ckpp_table *t, const void *d_keys, uint64_t n, uint8_t *d_found,
                         hipStream_t s) {
  const uint64_t lanes = n < t->path_lanes ? n : t->path_lanes;
  const uint32_t block = 256;
  const uint32_t grid = (uint32_t)((lanes + block - 1) / block);
  unsigned long long *nspin = reinterpret_cast<unsigned long long *>(t->d_stats) + 127;
  hipLaunchKernelGGL(delete_kernel, dim3(grid), dim3(block), 0, s, t->d_table,
                     reinterpret_cast<const uint4 *>(d_keys), n, t->log2_buckets, t->seed,
                     (t->flags & CKPP_PLAIN) ? 1u : 0u, d_found, nspin);
  return hipGetLastError();
}

}  // namespace ckpp
