// ckpp_lookup.hip -- batched lookup kernels (gfx950).
//
// One pass of a lookup (Sec. 2 lookup procedure, Sec. 4.1 pruning):
//   hash the key -> primary bucket p, alternate a, tag, two bloom bits;
//   fetch the first 32 bytes of bucket p (tags, filter, masks);
//   candidates = busy slots whose tag equals the key's tag;
//   for each candidate (ascending slot): fetch its 32-byte record and compare
//   all 16 key bytes; stop at the first equal key;
//   if not found: Cuckoo++ fetches bucket a only if both bloom bits are set
//   in p's filter; the pessimistic mode fetched a together with p; the
//   optimistic mode fetches a whenever the key was not in p;
//   write found (u8) and the value (u64, 0 on a miss).
//
// GPU form: a lane (or a pair of lanes) owns a lookup; each lane keeps K
// lookups in flight, issuing all K bucket fetches before consuming any, then
// all K first-candidate record fetches, so that a wave holds K x 64 random
// line reads in flight.  Keys are streamed in and results streamed out with
// non-temporal accesses so they do not evict table lines from the caches.

#include "ckpp_device.h"
#include "ckpp_internal.h"

namespace ckpp {
namespace {

template <int K>
__device__ __forceinline__ void probe_records(const uint4 *__restrict__ kv, const uint32_t (&b)[K],
                                              uint32_t (&cand)[K], const uint4 (&key)[K],
                                              bool (&hit)[K], uint64_t (&val)[K]) {
  const uint2 *kv2 = reinterpret_cast<const uint2 *>(kv);
  uint4 rk[K];
  uint2 rv[K];
  bool had[K];
  // first candidate of every lookup: the K record fetches go out together
#pragma unroll
  for (int j = 0; j < K; ++j) {
    had[j] = (cand[j] != 0u) && !hit[j];
    if (had[j]) {
      const uint32_t s = (uint32_t)__builtin_ctz(cand[j]);
      cand[j] &= cand[j] - 1u;
      const uint64_t r = (uint64_t)b[j] * kSlots + s;
      rk[j] = kv[r * kQuartersPerRecord];
      rv[j] = kv2[r * 4 + 2];
    }
  }
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if (had[j] && key_eq(rk[j], key[j])) {
      hit[j] = true;
      val[j] = (uint64_t)rv[j].x | ((uint64_t)rv[j].y << 32);
    }
  }
  // further candidates: tag matches of other keys (about 2^-16 per slot)
#pragma unroll
  for (int j = 0; j < K; ++j) {
    while (!hit[j] && cand[j] != 0u) {
      const uint32_t s = (uint32_t)__builtin_ctz(cand[j]);
      cand[j] &= cand[j] - 1u;
      const uint64_t r = (uint64_t)b[j] * kSlots + s;
      const uint4 k2 = kv[r * kQuartersPerRecord];
      const uint2 v2 = kv2[r * 4 + 2];
      if (key_eq(k2, key[j])) {
        hit[j] = true;
        val[j] = (uint64_t)v2.x | ((uint64_t)v2.y << 32);
      }
    }
  }
}

// One lane per lookup, K lookups per lane.  bk: bucket array as uint4
// quarters; kv: record array as uint4 halves.
template <int K, uint32_t MODE>
__global__ void __launch_bounds__(256)
    lookup_lane(const uint4 *__restrict__ bk, const uint4 *__restrict__ kv,
                const uint4 *__restrict__ keys, uint64_t n, uint32_t log2b, uint64_t seed,
                uint8_t *__restrict__ found, uint64_t *__restrict__ vals) {
  const uint64_t tile_sz = (uint64_t)blockDim.x * K;
  for (uint64_t tile = (uint64_t)blockIdx.x * tile_sz; tile < n;
       tile += (uint64_t)gridDim.x * tile_sz) {
    uint4 key[K];
    bool ok[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const uint64_t i = tile + (uint64_t)j * blockDim.x + threadIdx.x;
      ok[j] = i < n;
      key[j] = ok[j] ? load_stream(keys + i) : make_uint4(0u, 0u, 0u, 0u);
    }
    KeyFields f[K];
    uint32_t bp[K], ba[K];
    uint4 h0[K], h1[K], g0[K], g1[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      f[j] = key_fields(key_hash(key[j], seed), log2b);
      bp[j] = f[j].p;
      ba[j] = f[j].a;
      h0[j] = h1[j] = g0[j] = g1[j] = make_uint4(0u, 0u, 0u, 0u);
    }
    // primary bucket heads (and, pessimistic mode, the secondary ones too)
#pragma unroll
    for (int j = 0; j < K; ++j) {
      if (ok[j]) {
        h0[j] = bk[(uint64_t)bp[j] * kQuartersPerBucket];
        h1[j] = bk[(uint64_t)bp[j] * kQuartersPerBucket + 1];
        if (MODE == kModeBoth) {
          g0[j] = bk[(uint64_t)ba[j] * kQuartersPerBucket];
          g1[j] = bk[(uint64_t)ba[j] * kQuartersPerBucket + 1];
        }
      }
    }
    uint32_t cand[K];
    bool hit[K];
    uint64_t val[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      cand[j] = ok[j] ? (tag_eq_mask(h0[j], f[j].tag) & meta_busy(h1[j].z)) : 0u;
      hit[j] = false;
      val[j] = 0;
    }
    probe_records<K>(kv, bp, cand, key, hit, val);
    bool need[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      need[j] = ok[j] && !hit[j] &&
                (MODE != kModeCuckoopp || bloom_pass(h1[j], f[j].bloom_bits));
    }
    if (MODE != kModeBoth) {
#pragma unroll
      for (int j = 0; j < K; ++j) {
        if (need[j]) {
          g0[j] = bk[(uint64_t)ba[j] * kQuartersPerBucket];
          g1[j] = bk[(uint64_t)ba[j] * kQuartersPerBucket + 1];
        }
      }
    }
#pragma unroll
    for (int j = 0; j < K; ++j)
      cand[j] = need[j] ? (tag_eq_mask(g0[j], f[j].tag) & meta_busy(g1[j].z)) : 0u;
    probe_records<K>(kv, ba, cand, key, hit, val);
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const uint64_t i = tile + (uint64_t)j * blockDim.x + threadIdx.x;
      if (ok[j]) {
        __builtin_nontemporal_store((uint8_t)(hit[j] ? 1 : 0), found + i);
        __builtin_nontemporal_store(val[j], vals + i);
      }
    }
  }
}

// Two neighbouring lanes per lookup: the even lane fetches the bucket's tag
// quarter and the odd lane its filter/mask quarter, one 32-byte coalesced
// request per bucket; the tag match is completed across the pair, and the
// pair fetches a candidate record as key (even) + value (odd).
template <int K, uint32_t MODE>
__global__ void __launch_bounds__(256)
    lookup_pair(const uint4 *__restrict__ bk, const uint4 *__restrict__ kv,
                const uint4 *__restrict__ keys, uint64_t n, uint32_t log2b, uint64_t seed,
                uint8_t *__restrict__ found, uint64_t *__restrict__ vals) {
  const uint32_t half = threadIdx.x & 1u;  // 0: tags/key side, 1: filter/value side
  const uint32_t pairs = blockDim.x >> 1;
  const uint32_t pid = threadIdx.x >> 1;
  const uint64_t tile_sz = (uint64_t)pairs * K;
  for (uint64_t tile = (uint64_t)blockIdx.x * tile_sz; tile < n;
       tile += (uint64_t)gridDim.x * tile_sz) {
    uint4 key[K];
    bool ok[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const uint64_t i = tile + (uint64_t)j * pairs + pid;
      ok[j] = i < n;
      key[j] = ok[j] ? load_stream(keys + i) : make_uint4(0u, 0u, 0u, 0u);
    }
    KeyFields f[K];
    uint4 q[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      f[j] = key_fields(key_hash(key[j], seed), log2b);
      q[j] = make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int j = 0; j < K; ++j)
      if (ok[j]) q[j] = bk[(uint64_t)f[j].p * kQuartersPerBucket + half];
    uint4 qs[K];
    if (MODE == kModeBoth) {
#pragma unroll
      for (int j = 0; j < K; ++j) {
        qs[j] = make_uint4(0u, 0u, 0u, 0u);
        if (ok[j]) qs[j] = bk[(uint64_t)f[j].a * kQuartersPerBucket + half];
      }
    }
    bool hit[K], need[K];
    uint64_t val[K];
    uint32_t cand[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
      // even lane contributes the tag-equality mask, odd lane the busy mask
      // and the filter verdict (bit 8)
      const uint32_t mine = half == 0u
                                ? tag_eq_mask(q[j], f[j].tag)
                                : (meta_busy(q[j].z) | (bloom_pass(q[j], f[j].bloom_bits) ? 0x100u : 0u));
      const uint32_t theirs = (uint32_t)__shfl_xor((int)mine, 1);
      const uint32_t odd = half ? mine : theirs;
      cand[j] = ok[j] ? (mine & theirs & 0xffu) : 0u;
      need[j] = (odd & 0x100u) != 0u;
      hit[j] = false;
      val[j] = 0;
    }
    // records: the pair reads key (even) and value (odd) of the candidate
    for (int side = 0; side < 2; ++side) {
      if (side == 1) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
          need[j] = ok[j] && !hit[j] && (MODE != kModeCuckoopp || need[j]);
          if (MODE == kModeBoth) {
            q[j] = qs[j];
          } else if (need[j]) {
            q[j] = bk[(uint64_t)f[j].a * kQuartersPerBucket + half];
          }
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const uint32_t mine = half == 0u ? tag_eq_mask(q[j], f[j].tag) : meta_busy(q[j].z);
          const uint32_t theirs = (uint32_t)__shfl_xor((int)mine, 1);
          cand[j] = need[j] ? (mine & theirs & 0xffu) : 0u;
        }
      }
      bool any = true;
      while (any) {
        any = false;
        uint4 r[K];
        bool had[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
          had[j] = cand[j] != 0u && !hit[j];
          if (had[j]) {
            const uint32_t s = (uint32_t)__builtin_ctz(cand[j]);
            cand[j] &= cand[j] - 1u;
            const uint64_t b = side ? f[j].a : f[j].p;
            r[j] = kv[(b * kSlots + s) * kQuartersPerRecord + half];
          }
        }
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const uint32_t eq = (had[j] && half == 0u && key_eq(r[j], key[j])) ? 1u : 0u;
          const uint32_t e2 = eq | (uint32_t)__shfl_xor((int)eq, 1);
          if (had[j] && e2) {
            hit[j] = true;
            if (half) val[j] = (uint64_t)r[j].x | ((uint64_t)r[j].y << 32);
          }
          if (!hit[j] && cand[j] != 0u) any = true;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
      const uint64_t i = tile + (uint64_t)j * pairs + pid;
      if (ok[j]) {
        if (half == 0u)
          __builtin_nontemporal_store((uint8_t)(hit[j] ? 1 : 0), found + i);
        else
          __builtin_nontemporal_store(val[j], vals + i);
      }
    }
  }
}

template <int K, uint32_t MODE>
hipError_t launch_shape(const ckpp_table *t, uint32_t lanes, const uint4 *keys, uint64_t n,
                        uint8_t *found, uint64_t *vals, hipStream_t s) {
  const ckpp_launch_t &L = t->lookup_launch;
  const uint32_t block = L.block;
  const uint64_t per_block = (uint64_t)(block / lanes) * K;
  uint64_t grid = (n + per_block - 1) / per_block;
  if (L.blocks_per_cu) {
    const uint64_t cap = (uint64_t)L.blocks_per_cu * (uint64_t)t->num_cus;
    if (grid > cap) grid = cap;
  }
  if (grid > 0x7fffffffull) grid = 0x7fffffffull;
  const uint4 *bk = reinterpret_cast<const uint4 *>(t->d_buckets);
  const uint4 *kv = reinterpret_cast<const uint4 *>(t->d_kv);
  if (lanes == 1)
    hipLaunchKernelGGL((lookup_lane<K, MODE>), dim3((uint32_t)grid), dim3(block), 0, s, bk, kv,
                       keys, n, t->log2_buckets, t->seed, found, vals);
  else
    hipLaunchKernelGGL((lookup_pair<K, MODE>), dim3((uint32_t)grid), dim3(block), 0, s, bk, kv,
                       keys, n, t->log2_buckets, t->seed, found, vals);
  return hipGetLastError();
}

template <uint32_t MODE>
hipError_t launch_mode(const ckpp_table *t, const uint4 *keys, uint64_t n, uint8_t *found,
                       uint64_t *vals, hipStream_t s) {
  const uint32_t lanes = t->lookup_launch.lanes_per_lookup;
  switch (t->lookup_launch.lookups_per_lane) {
    case 1: return launch_shape<1, MODE>(t, lanes, keys, n, found, vals, s);
    case 2: return launch_shape<2, MODE>(t, lanes, keys, n, found, vals, s);
    default: return launch_shape<4, MODE>(t, lanes, keys, n, found, vals, s);
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
