// ckpp_aux.hip -- statistics, hashing, zero-fill, the random-read probe and
// the dependent-access latency probe.

#include "ckpp_device.h"
#include "ckpp_internal.h"

namespace ckpp {
namespace {

// Accumulator layout (u64 words) shared with the host side:
//   0 live, 1 in_secondary, 2 bloom_pc_sum, 3 bloom_pc2_sum, 4 locked,
//   5 busy slots 4..7, 6 secondary entries in slots 4..7,
//   7 .. 7+CKPP_MOVED_BINS-1 moved histogram.
constexpr uint32_t kHistBase = 7;
constexpr uint32_t kSums = 7;

__global__ void __launch_bounds__(256)
    stats_kernel(const uint4 *__restrict__ bk, uint64_t nbuckets, unsigned long long *acc) {
  __shared__ unsigned int hist[CKPP_MOVED_BINS];
  __shared__ unsigned long long part[kSums];
  for (uint32_t i = threadIdx.x; i < CKPP_MOVED_BINS; i += blockDim.x) hist[i] = 0u;
  if (threadIdx.x < kSums) part[threadIdx.x] = 0ull;
  __syncthreads();
  unsigned long long live = 0, insec = 0, pc = 0, pc2 = 0, locked = 0, hi = 0, hisec = 0;
  for (uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nbuckets;
       b += (uint64_t)gridDim.x * blockDim.x) {
    const uint4 q1 = bk[b * kQuartersPerBucket + 1];
    const uint32_t meta = q1.z;
    live += (unsigned long long)__builtin_popcount(meta_busy(meta));
    insec += (unsigned long long)__builtin_popcount(meta_sec(meta));
    const unsigned long long c =
        (unsigned long long)(__builtin_popcount(q1.x) + __builtin_popcount(q1.y));
    pc += c;
    pc2 += c * c;
    locked += q1.w != 0u ? 1ull : 0ull;
    hi += (unsigned long long)__builtin_popcount(meta_busy(meta) & 0xf0u);
    hisec += (unsigned long long)__builtin_popcount(meta_sec(meta) & 0xf0u);
    const uint32_t m = meta_moved(meta);
    atomicAdd(&hist[m < CKPP_MOVED_BINS - 1 ? m : CKPP_MOVED_BINS - 1], 1u);
  }
  atomicAdd(&part[0], live);
  atomicAdd(&part[1], insec);
  atomicAdd(&part[2], pc);
  atomicAdd(&part[3], pc2);
  atomicAdd(&part[4], locked);
  atomicAdd(&part[5], hi);
  atomicAdd(&part[6], hisec);
  __syncthreads();
  if (threadIdx.x < kSums) atomicAdd(&acc[threadIdx.x], part[threadIdx.x]);
  for (uint32_t i = threadIdx.x; i < CKPP_MOVED_BINS; i += blockDim.x)
    if (hist[i]) atomicAdd(&acc[kHistBase + i], (unsigned long long)hist[i]);
}

__global__ void __launch_bounds__(256)
    hash_kernel(const uint4 *__restrict__ keys, uint64_t n, uint64_t seed,
                uint64_t *__restrict__ out) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = key_hash(keys[i], seed);
}

__global__ void __launch_bounds__(256) fill_zero_kernel(uint4 *d, uint64_t n16) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
       i += (uint64_t)gridDim.x * blockDim.x)
    d[i] = make_uint4(0u, 0u, 0u, 0u);
}

// Random-read probe: read i of the launch reads the granule at index
// mix64(seed + i) * units >> 64 (uniform over the buffer).  Lane form: each
// lane reads whole granules (Q 16-byte loads each), PL granules in flight.
// Cooperative form: Q neighbouring lanes read one granule together, one
// 16-byte piece each, so a granule is a single coalesced request.
template <int Q, int PL, bool COOP>
__global__ void __launch_bounds__(256)
    probe_kernel(const uint4 *__restrict__ buf, uint64_t units, uint64_t nreads, uint64_t seed,
                 unsigned long long *__restrict__ sink) {
  const uint64_t lane = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t nl = (uint64_t)gridDim.x * blockDim.x;
  constexpr int QL = COOP ? 1 : Q;  // loads per granule per lane
  const uint64_t group = COOP ? lane / Q : lane;
  const uint64_t ngroups = COOP ? nl / Q : nl;
  const uint32_t part = COOP ? (uint32_t)(threadIdx.x % Q) : 0u;
  uint32_t acc = 0u;
  for (uint64_t r0 = group * PL; r0 < nreads; r0 += ngroups * PL) {
    uint4 v[PL][QL];
#pragma unroll
    for (int j = 0; j < PL; ++j) {
      const uint64_t i = r0 + j;
      if (i < nreads) {
        const uint64_t u = __umul64hi(mix64(seed + i), units);
#pragma unroll
        for (int q = 0; q < QL; ++q) v[j][q] = buf[u * Q + part + q];
      } else {
#pragma unroll
        for (int q = 0; q < QL; ++q) v[j][q] = make_uint4(0u, 0u, 0u, 0u);
      }
    }
#pragma unroll
    for (int j = 0; j < PL; ++j)
#pragma unroll
      for (int q = 0; q < QL; ++q) acc ^= v[j][q].x ^ v[j][q].y ^ v[j][q].z ^ v[j][q].w;
  }
  sink[lane] = acc;
}

template <int Q, bool COOP>
hipError_t probe_q(const void *d_buf, uint64_t units, uint64_t nreads, uint32_t per_lane,
                   uint32_t block, uint32_t grid, uint64_t seed, uint64_t *d_sink,
                   hipStream_t s) {
  const uint4 *b = reinterpret_cast<const uint4 *>(d_buf);
  unsigned long long *k = reinterpret_cast<unsigned long long *>(d_sink);
  switch (per_lane) {
    case 1: hipLaunchKernelGGL((probe_kernel<Q, 1, COOP>), dim3(grid), dim3(block), 0, s, b, units, nreads, seed, k); break;
    case 2: hipLaunchKernelGGL((probe_kernel<Q, 2, COOP>), dim3(grid), dim3(block), 0, s, b, units, nreads, seed, k); break;
    case 4: hipLaunchKernelGGL((probe_kernel<Q, 4, COOP>), dim3(grid), dim3(block), 0, s, b, units, nreads, seed, k); break;
    default: hipLaunchKernelGGL((probe_kernel<Q, 8, COOP>), dim3(grid), dim3(block), 0, s, b, units, nreads, seed, k); break;
  }
  return hipGetLastError();
}

template <bool COOP>
hipError_t probe_g(const void *d_buf, uint64_t bytes, uint32_t granule, uint64_t nreads,
                   uint32_t per_lane, uint32_t block, uint32_t grid, uint64_t seed,
                   uint64_t *d_sink, hipStream_t s) {
  const uint64_t units = bytes / granule;
  if (granule == 16) return probe_q<1, COOP>(d_buf, units, nreads, per_lane, block, grid, seed, d_sink, s);
  if (granule == 32) return probe_q<2, COOP>(d_buf, units, nreads, per_lane, block, grid, seed, d_sink, s);
  if (granule == 64) return probe_q<4, COOP>(d_buf, units, nreads, per_lane, block, grid, seed, d_sink, s);
  return probe_q<8, COOP>(d_buf, units, nreads, per_lane, block, grid, seed, d_sink, s);
}

// Latency probe: one lane follows a chain of `steps` dependent accesses,
// one request per step.
// Step k reads (kind 0: a plain load; 1: a relaxed agent-scope atomic load,
// the accesses of a critical section; 2: a relaxed agent-scope
// compare-and-swap that expects 1 and writes 1, the lock's operation,
// which never changes a word holding anything else and leaves a 1 as it
// is; 3: an atomic load, then the same value stored back with an atomic
// store and a wait until the store is complete, the end of a critical
// section; 4: two compare-and-swaps issued together, on lines half the
// buffer apart, a lock pair's first attempt) the 16-byte-aligned word of 128-byte line
// mix64(seed + k + value of step k - 1) mod lines, so every access waits
// for the one before it.  The buffer's contents are not changed.
// out[0] = elapsed real-time counter ticks (100 MHz), out[1] = a fold of the
// values read.
constexpr uint32_t kLatencyBatch = 32;  // loads per step of kinds 5 and 6

template <int KIND>
__global__ void __launch_bounds__(64)
    latency_kernel(uint64_t *buf, uint64_t lines, uint32_t steps, uint64_t seed, uint64_t *out) {
  if (threadIdx.x != 0) return;  // one lane: one request per step
  uint64_t v = 0, fold = 0;
  const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
  for (uint32_t k = 0; k < steps; ++k) {
    const uint64_t line = __umul64hi(mix64(seed + k + v), lines);
    uint64_t *w = buf + line * 16u;
    if (KIND == 0) {
      v = *reinterpret_cast<volatile uint64_t *>(w);
    } else if (KIND == 1) {
      v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if (KIND == 2) {
      uint64_t e = 1u;
      __hip_atomic_compare_exchange_strong(w, &e, 1ull, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
      v = e;
    } else if (KIND == 3) {
      v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(w, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __builtin_amdgcn_s_waitcnt(0);
    } else if (KIND >= 5) {
      // kLatencyBatch independent loads of different lines, all issued
      // before the first is waited for: plain loads (5) and relaxed
      // agent-scope atomic loads (6) through a global-memory pointer, and
      // atomic loads through a generic pointer (7: the compiler then emits
      // flat loads, which also count against the LDS counter)
      uint64_t got[kLatencyBatch];
#pragma unroll
      for (uint32_t j = 0; j < kLatencyBatch; ++j) {
        const uint64_t lj = __umul64hi(mix64(seed + (uint64_t)k * kLatencyBatch + j + v), lines);
        uint64_t *wj = buf + lj * 16u;
        __attribute__((address_space(1))) uint64_t *gj =
            (__attribute__((address_space(1))) uint64_t *)wj;
        if (KIND == 5) got[j] = *gj;
        else if (KIND == 6) got[j] = __hip_atomic_load(gj, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else got[j] = __hip_atomic_load(wj, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      v = 0;
#pragma unroll
      for (uint32_t j = 0; j < kLatencyBatch; ++j) v ^= got[j];
    } else {
      // a line half the buffer away (a lock pair's buckets are far apart)
      const uint64_t far = line + lines / 2u;
      uint64_t *w2 = buf + (far < lines ? far : far - lines) * 16u;
      uint64_t e = 1u, e2 = 1u;
      __hip_atomic_compare_exchange_strong(w, &e, 1ull, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_compare_exchange_strong(w2, &e2, 1ull, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
      v = e ^ e2;
    }
    fold ^= v;
  }
  out[0] = __builtin_amdgcn_s_memrealtime() - t0;
  out[1] = fold;
}

}  // namespace

hipError_t launch_latency(void *d_buf, uint64_t bytes, uint32_t kind, uint32_t steps,
                          uint64_t seed, uint64_t *d_out, hipStream_t s) {
  uint64_t *b = static_cast<uint64_t *>(d_buf);
  const uint64_t lines = bytes / 128u;
  switch (kind) {
    case 0: hipLaunchKernelGGL(latency_kernel<0>, dim3(1), dim3(64), 0, s, b, lines, steps, seed, d_out); break;
    case 1: hipLaunchKernelGGL(latency_kernel<1>, dim3(1), dim3(64), 0, s, b, lines, steps, seed, d_out); break;
    case 2: hipLaunchKernelGGL(latency_kernel<2>, dim3(1), dim3(64), 0, s, b, lines, steps, seed, d_out); break;
    case 3: hipLaunchKernelGGL(latency_kernel<3>, dim3(1), dim3(64), 0, s, b, lines, steps, seed, d_out); break;
    case 4: hipLaunchKernelGGL(latency_kernel<4>, dim3(1), dim3(64), 0, s, b, lines, steps, seed, d_out); break;
    case 5: hipLaunchKernelGGL(latency_kernel<5>, dim3(1), dim3(64), 0, s, b, lines, steps, seed, d_out); break;
    case 6: hipLaunchKernelGGL(latency_kernel<6>, dim3(1), dim3(64), 0, s, b, lines, steps, seed, d_out); break;
    default: hipLaunchKernelGGL(latency_kernel<7>, dim3(1), dim3(64), 0, s, b, lines, steps, seed, d_out); break;
  }
  return hipGetLastError();
}

hipError_t launch_stats(const ckpp_table *t, uint64_t *d_acc, hipStream_t s) {
  const uint64_t nb = 1ull << t->log2_buckets;
  uint64_t grid = (nb + 255) / 256;
  const uint64_t cap = (uint64_t)t->num_cus * 8;
  if (grid > cap) grid = cap;
  hipLaunchKernelGGL(stats_kernel, dim3((uint32_t)grid), dim3(256), 0, s,
                     reinterpret_cast<const uint4 *>(t->d_table), nb,
                     reinterpret_cast<unsigned long long *>(d_acc));
  return hipGetLastError();
}

hipError_t launch_hash(const ckpp_table *t, const void *d_keys, uint64_t n, uint64_t *d_hash,
                       hipStream_t s) {
  uint64_t grid = (n + 255) / 256;
  if (grid > 65536) grid = 65536;
  hipLaunchKernelGGL(hash_kernel, dim3((uint32_t)grid), dim3(256), 0, s,
                     reinterpret_cast<const uint4 *>(d_keys), n, t->seed, d_hash);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void *d, uint64_t bytes, hipStream_t s) {
  const uint64_t n16 = bytes / 16;
  uint64_t grid = (n16 + 255) / 256;
  if (grid > 65536) grid = 65536;
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((uint32_t)grid), dim3(256), 0, s,
                     reinterpret_cast<uint4 *>(d), n16);
  return hipGetLastError();
}

hipError_t launch_probe(const void *d_buf, uint64_t bytes, uint32_t granule, uint64_t nreads,
                        uint32_t per_lane, uint32_t cooperative, uint32_t block, uint32_t grid,
                        uint64_t seed, uint64_t *d_sink, hipStream_t s) {
  if (cooperative)
    return probe_g<true>(d_buf, bytes, granule, nreads, per_lane, block, grid, seed, d_sink, s);
  return probe_g<false>(d_buf, bytes, granule, nreads, per_lane, block, grid, seed, d_sink, s);
}

}  // namespace ckpp
