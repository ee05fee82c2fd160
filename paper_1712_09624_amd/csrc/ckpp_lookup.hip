// ckpp_lookup.hip -- batched lookup kernel (gfx950).
//
// One lookup (Sec. 2 lookup procedure, Sec. 4.1 pruning):
//   hash the key -> primary bucket p, alternate a, tag, two bloom bits;
//   read p; a slot holds the key iff it is busy and its full 16-byte key
//   equals the searched key (its tag is only a hint that selects which
//   record to fetch); if not found, Cuckoo++ reads a only when both bloom
//   bits are set in p's filter, the pessimistic mode reads a together with
//   p, the optimistic mode reads a whenever the key was not in p;
//   write found (u8) and the value (u64, 0 on a miss).
//
// GPU form: a group of 8 neighbouring lanes owns a lookup.  Lane r of the
// group reads 16-byte quarter r of the bucket's first 128-byte line, so the
// whole line -- tags, filter, masks, and the keys and values of slots 0..3
// -- arrives in ONE memory request (a random 128-byte read costs the same
// request as a 64-byte one on MI355X).  The group combines per-lane verdicts
// with three cross-lane exchanges: lane 0 the tag matches, lane 1 the busy
// mask and the filter verdict, lanes 2..5 the full-key equality of slots
// 0..3.  Only if a busy slot 4..7 carries the key's tag is the second line
// (keys and values of slots 4..7) read.  Each group keeps K lookups in
// flight; keys stream in and results stream out with non-temporal accesses.

#include "ckpp_device.h"
#include "ckpp_internal.h"

namespace ckpp {
namespace {

// Group word of a bucket's first line:
//   bits 0..7   tag equality of slots 0..7       (lane 0)
//   bits 8..15  busy mask                        (lane 1)
//   bit  16     both bloom bits set              (lane 1)
//   bits 24..27 key equality of slots 0..3       (lanes 2..5)
__device__ __forceinline__ uint32_t line0_word(uint32_t r, uint4 q, const KeyFields &f,
                                               uint4 key) {
  if (r == 0u) return tag_eq_mask(q, f.tag);
  if (r == 1u) return (meta_busy(q.z) << 8) | (bloom_pass(q, f.bloom_bits) ? 0x10000u : 0u);
  if (r < 6u) return key_eq(q, key) ? (1u << (22u + r)) : 0u;
  return 0u;
}

// Group word of a bucket's second line: bits 4..7 key equality of slots
// 4..7 (lanes 0..3).
__device__ __forceinline__ uint32_t line1_word(uint32_t r, uint4 q, uint4 key) {
  return (r < 4u && key_eq(q, key)) ? (1u << (4u + r)) : 0u;
}

// OR of w over the 8 lanes of the group.
__device__ __forceinline__ uint32_t group_or(uint32_t w) {
  w |= (uint32_t)__shfl_xor((int)w, 1);
  w |= (uint32_t)__shfl_xor((int)w, 2);
  w |= (uint32_t)__shfl_xor((int)w, 4);
  return w;
}

// The 64-bit value of slot s (slot parity selects the half) from the
// quarter that holds it.
__device__ __forceinline__ uint64_t quarter_value(uint4 q, uint32_t s) {
  return (s & 1u) ? ((uint64_t)q.z | ((uint64_t)q.w << 32))
                  : ((uint64_t)q.x | ((uint64_t)q.y << 32));
}

// Search state of one lookup, identical in the 8 lanes of its group except
// `val`, which is meaningful in lane `owner` only.
struct Probe {
  bool hit;
  uint32_t owner;
  uint64_t val;
};

// Analyses the first line of a bucket (quarter q of this lane): a hit in
// slots 0..3 resolves here; returns the group word (busy mask, tag
// matches, filter verdict).
__device__ __forceinline__ uint32_t analyse_line0(uint32_t r, uint4 q, const KeyFields &f,
                                                  uint4 key, Probe &pr) {
  const uint32_t w = group_or(line0_word(r, q, f, key));
  const uint32_t m = (w >> 8) & (w >> 24) & 0xfu;  // busy and equal, slots 0..3
  if (m) {
    const uint32_t s = (uint32_t)__builtin_ctz(m);
    pr.hit = true;
    pr.owner = 6u + (s >> 1);
    pr.val = quarter_value(q, s);
  }
  return w;
}

// After the second line of a bucket (quarter q) arrived: a hit in 4..7.
__device__ __forceinline__ void analyse_line1(uint32_t r, uint4 q, uint32_t w0, uint4 key,
                                              Probe &pr) {
  const uint32_t w = group_or(line1_word(r, q, key));
  const uint32_t m = (w0 >> 8) & w & 0xf0u;
  if (m) {
    const uint32_t s = (uint32_t)__builtin_ctz(m);
    pr.hit = true;
    pr.owner = 4u + ((s - 4u) >> 1);
    pr.val = quarter_value(q, s);
  }
}

// Whether the second line must be read: no hit yet and a busy slot 4..7
// carries the key's tag.
__device__ __forceinline__ bool needs_line1(uint32_t w0, const Probe &pr) {
  return !pr.hit && (((w0 >> 8) & w0 & 0xf0u) != 0u);
}

template <int K, uint32_t MODE>
__global__ void __launch_bounds__(256)
    lookup_group8(const uint4 *__restrict__ tab, const uint4 *__restrict__ keys, uint64_t n,
                  uint32_t log2b, uint64_t seed, uint8_t *__restrict__ found,
                  uint64_t *__restrict__ vals) {
  const uint32_t r = threadIdx.x & 7u;
  const uint32_t groups = blockDim.x >> 3;
  const uint32_t gid = threadIdx.x >> 3;
  const uint64_t tile_sz = (uint64_t)groups * K;
  for (uint64_t tile = (uint64_t)blockIdx.x * tile_sz; tile < n;
       tile += (uint64_t)gridDim.x * tile_sz) {
    uint4 key[K];
    bool ok[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const uint64_t i = tile + (uint64_t)j * groups + gid;
      ok[j] = i < n;
      key[j] = ok[j] ? load_stream(keys + i) : make_uint4(0u, 0u, 0u, 0u);
    }
    KeyFields f[K];
    uint4 qp[K], qa[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      f[j] = key_fields(key_hash(key[j], seed), log2b);
      qp[j] = qa[j] = make_uint4(0u, 0u, 0u, 0u);
    }
    // first lines: one 128-byte request per lookup (two for pessimistic)
#pragma unroll
    for (int j = 0; j < K; ++j) {
      if (ok[j]) {
        qp[j] = tab[(uint64_t)f[j].p * kQuartersPerBucket + r];
        if (MODE == kModeBoth) qa[j] = tab[(uint64_t)f[j].a * kQuartersPerBucket + r];
      }
    }
    Probe pr[K];
    uint32_t wp[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      pr[j].hit = false;
      pr[j].owner = 0u;
      pr[j].val = 0ull;
      wp[j] = ok[j] ? analyse_line0(r, qp[j], f[j], key[j], pr[j]) : 0u;
    }
    // second line of the primary bucket, only on a tag match in slots 4..7
    bool need[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      need[j] = ok[j] && needs_line1(wp[j], pr[j]);
      if (need[j]) qp[j] = tab[(uint64_t)f[j].p * kQuartersPerBucket + 8u + r];
    }
#pragma unroll
    for (int j = 0; j < K; ++j)
      if (need[j]) analyse_line1(r, qp[j], wp[j], key[j], pr[j]);
    // secondary bucket
#pragma unroll
    for (int j = 0; j < K; ++j) {
      need[j] = ok[j] && !pr[j].hit && (MODE != kModeCuckoopp || ((wp[j] >> 16) & 1u));
      if (MODE != kModeBoth && need[j]) qa[j] = tab[(uint64_t)f[j].a * kQuartersPerBucket + r];
    }
    uint32_t wa[K];
#pragma unroll
    for (int j = 0; j < K; ++j)
      wa[j] = need[j] ? analyse_line0(r, qa[j], f[j], key[j], pr[j]) : 0u;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      need[j] = need[j] && needs_line1(wa[j], pr[j]);
      if (need[j]) qa[j] = tab[(uint64_t)f[j].a * kQuartersPerBucket + 8u + r];
    }
#pragma unroll
    for (int j = 0; j < K; ++j)
      if (need[j]) analyse_line1(r, qa[j], wa[j], key[j], pr[j]);
    // results: lane 0 writes the found flag; the value is written by the
    // lane that holds it (lane 0 writes 0 on a miss)
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const uint64_t i = tile + (uint64_t)j * groups + gid;
      if (ok[j]) {
        if (r == 0u) __builtin_nontemporal_store((uint8_t)(pr[j].hit ? 1 : 0), found + i);
        if (pr[j].hit ? (r == pr[j].owner) : (r == 0u))
          __builtin_nontemporal_store(pr[j].hit ? pr[j].val : 0ull, vals + i);
      }
    }
  }
}

template <int K, uint32_t MODE>
hipError_t launch_shape(const ckpp_table *t, const uint4 *keys, uint64_t n, uint8_t *found,
                        uint64_t *vals, hipStream_t s) {
  const ckpp_launch_t &L = t->lookup_launch;
  const uint32_t block = L.block;
  const uint64_t per_block = (uint64_t)(block / 8u) * K;
  uint64_t grid = (n + per_block - 1) / per_block;
  if (L.blocks_per_cu) {
    const uint64_t cap = (uint64_t)L.blocks_per_cu * (uint64_t)t->num_cus;
    if (grid > cap) grid = cap;
  }
  if (grid > 0x7fffffffull) grid = 0x7fffffffull;
  hipLaunchKernelGGL((lookup_group8<K, MODE>), dim3((uint32_t)grid), dim3(block), 0, s,
                     reinterpret_cast<const uint4 *>(t->d_table), keys, n, t->log2_buckets,
                     t->seed, found, vals);
  return hipGetLastError();
}

template <uint32_t MODE>
hipError_t launch_mode(const ckpp_table *t, const uint4 *keys, uint64_t n, uint8_t *found,
                       uint64_t *vals, hipStream_t s) {
  switch (t->lookup_launch.lookups_per_lane) {
    case 1: return launch_shape<1, MODE>(t, keys, n, found, vals, s);
    case 2: return launch_shape<2, MODE>(t, keys, n, found, vals, s);
    default: return launch_shape<4, MODE>(t, keys, n, found, vals, s);
  }
}

}  // namespace

hipError_t launch_lookup(const ckpp_table *t, const void *d_keys, uint64_t n, uint32_t mode,
                         uint8_t *d_found, uint64_t *d_values, hipStream_t s) {
  const uint4 *keys = reinterpret_cast<const uint4 *>(d_keys);
  if (mode == kModeBoth) return launch_mode<kModeBoth>(t, keys, n, d_found, d_values, s);
  if (mode == kModeOptimistic)
    return launch_mode<kModeOptimistic>(t, keys, n, d_found, d_values, s);
  return launch_mode<kModeCuckoopp>(t, keys, n, d_found, d_values, s);
}

}  // namespace ckpp
