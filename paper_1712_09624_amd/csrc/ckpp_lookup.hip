// ckpp_lookup.hip -- batched lookup kernel (gfx950).
//
// One lookup (Sec. 2 lookup procedure, Sec. 4.1 pruning):
//   hash the key -> primary bucket p, alternate a, tag, two bloom bits;
//   read p; a slot holds the key iff it is busy and its full 16-byte key
//   equals the searched key (its tag is only a hint that selects which keys
//   to compare); if not found, Cuckoo++ reads a only when both bloom bits
//   are set in p's filter, the pessimistic mode reads a together with p, the
//   optimistic mode reads a whenever the key was not in p;
//   write found (u8) and the value (u64, 0 on a miss).
//
// GPU form.  On MI355X every random read that misses the L2 costs one
// 128-byte line request, a later second access to the same line costs
// another, and the request rate -- not the byte rate -- bounds random reads.
// So a bucket line is read exactly once, in one instruction, by 8 lanes (16
// bytes each), straight into LDS (global_load_lds_dwordx4: the data in
// flight occupies no registers, so a wave keeps 64 line requests in flight
// at once).  Each lane owns one lookup: it hashes its key once, hands its
// bucket index to the fetching group (ds_bpermute), and after the lines
// have landed it analyses its own line from LDS: tags and busy mask, then
// the full keys of the candidate slots and the value.  The first line of a
// bucket holds the metadata and slots 0..3, so most lookups need one
// request; the second line (slots 4..7) and the secondary bucket are
// fetched, in the same cooperative way, only for the lookups of the wave
// that need them, and skipped when none does.  Keys for the next tile are
// loaded while the current tile is processed; keys stream in and results
// stream out with non-temporal accesses.

#include "ckpp_device.h"
#include "ckpp_internal.h"

namespace ckpp {
namespace {

constexpr uint32_t kNoFetch = 0xffffffffu;  // bucket indices are < 2^24

// Lines of one wave: 64 lines x 8 quarters; lookup j's line at [8j, 8j+8).
constexpr uint32_t kWaveQuarters = 64 * 8;

// Cooperative fetch of one 128-byte line (half `half` of the bucket) for
// every lookup of the wave whose `bucket` is not kNoFetch: in round k the
// lanes 8g..8g+7 read the line of lookup 8k+g, lane r its quarter r, and
// the line lands at lines[8(8k+g) .. 8(8k+g)+8).
__device__ __forceinline__ void fetch_lines(uint4 *lines, const uint4 *tab, uint32_t bucket,
                                            uint32_t half, uint32_t g, uint32_t r) {
#pragma unroll
  for (uint32_t k = 0; k < 8; ++k) {
    const uint32_t b = (uint32_t)__builtin_amdgcn_ds_bpermute((int)((8u * k + g) << 2), (int)bucket);
    if (b != kNoFetch) {
      const uint4 *src = tab + (uint64_t)b * kQuartersPerBucket + 8u * half + r;
      __builtin_amdgcn_global_load_lds(
          (const void __attribute__((address_space(1))) *)src,
          (void __attribute__((address_space(3))) *)(lines + 64u * k), 16, 0, 0);
    }
  }
}

// Waits until the lines requested by this wave have landed in LDS (the
// loads' counter drains once the data is written there); the compiler may
// not move LDS reads above this point.
__device__ __forceinline__ void lines_landed() {
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ uint64_t quarter_value(uint4 q, uint32_t s) {
  return (s & 1u) ? ((uint64_t)q.z | ((uint64_t)q.w << 32))
                  : ((uint64_t)q.x | ((uint64_t)q.y << 32));
}

// Compares the key with the candidate slots `cand` (ascending) of a first
// line (mine[0..7]); on a hit sets hit/val.
__device__ __forceinline__ void match_line0(const uint4 *mine, uint32_t cand, uint4 key, bool &hit,
                                            uint64_t &val) {
  while (cand != 0u && !hit) {
    const uint32_t s = (uint32_t)__builtin_ctz(cand);
    cand &= cand - 1u;
    if (key_eq(mine[2u + s], key)) {
      hit = true;
      val = quarter_value(mine[6u + (s >> 1)], s);
    }
  }
}

// Same for slots 4..7 on a second line (mine[0..7]).
__device__ __forceinline__ void match_line1(const uint4 *mine, uint32_t cand, uint4 key, bool &hit,
                                            uint64_t &val) {
  while (cand != 0u && !hit) {
    const uint32_t s = (uint32_t)__builtin_ctz(cand);
    cand &= cand - 1u;
    if (key_eq(mine[s - 4u], key)) {
      hit = true;
      val = quarter_value(mine[4u + ((s - 4u) >> 1)], s);
    }
  }
}

template <uint32_t WAVES, uint32_t MODE>
__global__ void __launch_bounds__(64 * WAVES)
    lookup_lds(const uint4 *__restrict__ tab, const uint4 *__restrict__ keys, uint64_t n,
               uint32_t log2b, uint64_t seed, uint8_t *__restrict__ found,
               uint64_t *__restrict__ vals) {
  constexpr uint32_t NB = MODE == kModeBoth ? 2 : 1;  // line buffers per wave
  __shared__ uint4 s_lines[WAVES * NB * kWaveQuarters];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t g = lane >> 3, r = lane & 7u;
  uint4 *lines = s_lines + (threadIdx.x >> 6) * NB * kWaveQuarters;
  uint4 *lines_a = lines + (NB - 1) * kWaveQuarters;  // pessimistic: secondary lines
  const uint4 *mine = lines + 8u * lane;
  const uint4 *mine_a = lines_a + 8u * lane;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint4 key = i < n ? load_stream(keys + i) : make_uint4(0u, 0u, 0u, 0u);
  // the wave stays together: its loop condition is the wave's first lookup
  for (; i - lane < n; i += stride) {
    const bool ok = i < n;
    const uint64_t h = key_hash(key, seed);
    const KeyFields f = key_fields(h, log2b);
    // first line of the primary (and, pessimistic mode, the secondary)
    fetch_lines(lines, tab, ok ? f.p : kNoFetch, 0u, g, r);
    if (MODE == kModeBoth) fetch_lines(lines_a, tab, ok ? f.a : kNoFetch, 0u, g, r);
    const uint64_t inext = i + stride;
    const uint4 knext = inext < n ? load_stream(keys + inext) : make_uint4(0u, 0u, 0u, 0u);
    lines_landed();
    bool hit = false;
    uint64_t val = 0;
    const uint4 t0 = mine[0], t1 = mine[1];
    const uint32_t cand = ok ? (tag_eq_mask(t0, f.tag) & meta_busy(t1.z)) : 0u;
    const bool pass = MODE != kModeCuckoopp || bloom_pass(t1, f.bloom_bits);
    match_line0(mine, cand & 0xfu, key, hit, val);
    // second line of the primary, for keys whose tag sits in slots 4..7
    bool need = !hit && (cand & 0xf0u);
    if (__builtin_amdgcn_ballot_w64(need)) {
      fetch_lines(lines, tab, need ? f.p : kNoFetch, 1u, g, r);
      lines_landed();
      if (need) match_line1(mine, cand & 0xf0u, key, hit, val);
    }
    // secondary bucket
    need = ok && !hit && pass;
    if (__builtin_amdgcn_ballot_w64(need)) {
      if (MODE != kModeBoth) {
        fetch_lines(lines, tab, need ? f.a : kNoFetch, 0u, g, r);
        lines_landed();
      }
      uint32_t cand2 = 0u;
      if (need) {
        const uint4 u0 = mine_a[0], u1 = mine_a[1];
        cand2 = tag_eq_mask(u0, f.tag) & meta_busy(u1.z);
        match_line0(mine_a, cand2 & 0xfu, key, hit, val);
      }
      need = need && !hit && (cand2 & 0xf0u);
      if (__builtin_amdgcn_ballot_w64(need)) {
        fetch_lines(lines_a, tab, need ? f.a : kNoFetch, 1u, g, r);
        lines_landed();
        if (need) match_line1(mine_a, cand2 & 0xf0u, key, hit, val);
      }
    }
    if (ok) {
      __builtin_nontemporal_store((uint8_t)(hit ? 1 : 0), found + i);
      __builtin_nontemporal_store(hit ? val : 0ull, vals + i);
    }
    key = knext;
  }
}

// Register-landing counterpart of fetch_lines: the same rounds, but the
// quarter arrives in q[k] of the fetching lane; park_lines() later writes
// the quarters to LDS in exactly the layout fetch_lines produces.
__device__ __forceinline__ void fetch_lines_reg(uint4 (&q)[8], const uint4 *tab, uint32_t bucket,
                                                uint32_t half, uint32_t g, uint32_t r) {
#pragma unroll
  for (uint32_t k = 0; k < 8; ++k) {
    const uint32_t b = (uint32_t)__builtin_amdgcn_ds_bpermute((int)((8u * k + g) << 2), (int)bucket);
    q[k] = make_uint4(0u, 0u, 0u, 0u);
    if (b != kNoFetch) q[k] = tab[(uint64_t)b * kQuartersPerBucket + 8u * half + r];
  }
}

__device__ __forceinline__ void park_lines(uint4 *lines, const uint4 (&q)[8], uint32_t lane) {
#pragma unroll
  for (uint32_t k = 0; k < 8; ++k) lines[64u * k + lane] = q[k];
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Lookup state of one lookup owned by a lane.
struct Look {
  uint4 key;
  KeyFields f;
  bool ok, hit, pass;
  uint32_t cand;
  uint64_t val;
};

__device__ __forceinline__ void first_line(const uint4 *mine, Look &L, uint32_t mode) {
  const uint4 t0 = mine[0], t1 = mine[1];
  L.cand = L.ok ? (tag_eq_mask(t0, L.f.tag) & meta_busy(t1.z)) : 0u;
  L.pass = mode != kModeCuckoopp || bloom_pass(t1, L.f.bloom_bits);
  match_line0(mine, L.cand & 0xfu, L.key, L.hit, L.val);
}

// Two lookups per lane (lookups tile + lane and tile + 64 + lane): for each
// phase the lines of the first 64 land in LDS directly, those of the other
// 64 in registers, which are parked in LDS once the first 64 have been
// analysed -- twice the line requests in flight for the same LDS.
template <uint32_t WAVES, uint32_t MODE>
__global__ void __launch_bounds__(64 * WAVES)
    lookup_dual(const uint4 *__restrict__ tab, const uint4 *__restrict__ keys, uint64_t n,
                uint32_t log2b, uint64_t seed, uint8_t *__restrict__ found,
                uint64_t *__restrict__ vals) {
  static_assert(MODE != kModeBoth, "the pessimistic mode uses lookup_lds");
  __shared__ uint4 s_lines[WAVES * kWaveQuarters];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t g = lane >> 3, r = lane & 7u;
  uint4 *lines = s_lines + (threadIdx.x >> 6) * kWaveQuarters;
  const uint4 *mine = lines + 8u * lane;
  const uint64_t wave0 = ((uint64_t)blockIdx.x * WAVES + (threadIdx.x >> 6)) * 128u;
  const uint64_t stride = (uint64_t)gridDim.x * WAVES * 128u;
  uint4 ka = wave0 + lane < n ? load_stream(keys + wave0 + lane) : make_uint4(0u, 0u, 0u, 0u);
  uint4 kb = wave0 + 64u + lane < n ? load_stream(keys + wave0 + 64u + lane)
                                    : make_uint4(0u, 0u, 0u, 0u);
  for (uint64_t w0 = wave0; w0 < n; w0 += stride) {
    Look A, Bq;
    A.key = ka;
    Bq.key = kb;
    A.ok = w0 + lane < n;
    Bq.ok = w0 + 64u + lane < n;
    A.f = key_fields(key_hash(A.key, seed), log2b);
    Bq.f = key_fields(key_hash(Bq.key, seed), log2b);
    A.hit = Bq.hit = false;
    A.val = Bq.val = 0ull;
    uint4 q[8];
    // phase 1: primary first lines
    fetch_lines(lines, tab, A.ok ? A.f.p : kNoFetch, 0u, g, r);
    fetch_lines_reg(q, tab, Bq.ok ? Bq.f.p : kNoFetch, 0u, g, r);
    const uint64_t nx = w0 + stride;
    ka = nx + lane < n ? load_stream(keys + nx + lane) : make_uint4(0u, 0u, 0u, 0u);
    kb = nx + 64u + lane < n ? load_stream(keys + nx + 64u + lane) : make_uint4(0u, 0u, 0u, 0u);
    lines_landed();
    first_line(mine, A, MODE);
    park_lines(lines, q, lane);
    first_line(mine, Bq, MODE);
    // phase 2: primary second lines
    bool na = !A.hit && (A.cand & 0xf0u), nb = !Bq.hit && (Bq.cand & 0xf0u);
    if (__builtin_amdgcn_ballot_w64(na || nb)) {
      fetch_lines(lines, tab, na ? A.f.p : kNoFetch, 1u, g, r);
      fetch_lines_reg(q, tab, nb ? Bq.f.p : kNoFetch, 1u, g, r);
      lines_landed();
      if (na) match_line1(mine, A.cand & 0xf0u, A.key, A.hit, A.val);
      park_lines(lines, q, lane);
      if (nb) match_line1(mine, Bq.cand & 0xf0u, Bq.key, Bq.hit, Bq.val);
    }
    // phase 3: secondary first lines
    na = A.ok && !A.hit && A.pass;
    nb = Bq.ok && !Bq.hit && Bq.pass;
    if (__builtin_amdgcn_ballot_w64(na || nb)) {
      fetch_lines(lines, tab, na ? A.f.a : kNoFetch, 0u, g, r);
      fetch_lines_reg(q, tab, nb ? Bq.f.a : kNoFetch, 0u, g, r);
      lines_landed();
      uint32_t ca = 0u, cb = 0u;
      if (na) {
        ca = tag_eq_mask(mine[0], A.f.tag) & meta_busy(mine[1].z);
        match_line0(mine, ca & 0xfu, A.key, A.hit, A.val);
      }
      park_lines(lines, q, lane);
      if (nb) {
        cb = tag_eq_mask(mine[0], Bq.f.tag) & meta_busy(mine[1].z);
        match_line0(mine, cb & 0xfu, Bq.key, Bq.hit, Bq.val);
      }
      // phase 4: secondary second lines
      na = na && !A.hit && (ca & 0xf0u);
      nb = nb && !Bq.hit && (cb & 0xf0u);
      if (__builtin_amdgcn_ballot_w64(na || nb)) {
        fetch_lines(lines, tab, na ? A.f.a : kNoFetch, 1u, g, r);
        fetch_lines_reg(q, tab, nb ? Bq.f.a : kNoFetch, 1u, g, r);
        lines_landed();
        if (na) match_line1(mine, ca & 0xf0u, A.key, A.hit, A.val);
        park_lines(lines, q, lane);
        if (nb) match_line1(mine, cb & 0xf0u, Bq.key, Bq.hit, Bq.val);
      }
    }
    if (A.ok) {
      __builtin_nontemporal_store((uint8_t)(A.hit ? 1 : 0), found + w0 + lane);
      __builtin_nontemporal_store(A.hit ? A.val : 0ull, vals + w0 + lane);
    }
    if (Bq.ok) {
      __builtin_nontemporal_store((uint8_t)(Bq.hit ? 1 : 0), found + w0 + 64u + lane);
      __builtin_nontemporal_store(Bq.hit ? Bq.val : 0ull, vals + w0 + 64u + lane);
    }
  }
}

template <uint32_t WAVES, uint32_t MODE>
hipError_t launch_dual(const ckpp_table *t, const uint4 *keys, uint64_t n, uint8_t *found,
                       uint64_t *vals, hipStream_t s) {
  const ckpp_launch_t &L = t->lookup_launch;
  const uint64_t per_block = 128ull * WAVES;
  uint64_t grid = (n + per_block - 1) / per_block;
  if (L.blocks_per_cu) {
    const uint64_t cap = (uint64_t)L.blocks_per_cu * (uint64_t)t->num_cus;
    if (grid > cap) grid = cap;
  }
  if (grid > 0x7fffffffull) grid = 0x7fffffffull;
  hipLaunchKernelGGL((lookup_dual<WAVES, MODE>), dim3((uint32_t)grid), dim3(64 * WAVES), 0, s,
                     reinterpret_cast<const uint4 *>(t->d_table), keys, n, t->log2_buckets,
                     t->seed, found, vals);
  return hipGetLastError();
}

template <uint32_t WAVES, uint32_t MODE>
hipError_t launch_shape(const ckpp_table *t, const uint4 *keys, uint64_t n, uint8_t *found,
                        uint64_t *vals, hipStream_t s) {
  if (MODE != kModeBoth && t->lookup_launch.lookups_per_lane == 2)
    return launch_dual<WAVES, (MODE == kModeBoth ? kModeCuckoopp : MODE)>(t, keys, n, found, vals, s);
  const ckpp_launch_t &L = t->lookup_launch;
  const uint64_t per_block = 64ull * WAVES;
  uint64_t grid = (n + per_block - 1) / per_block;
  if (L.blocks_per_cu) {
    const uint64_t cap = (uint64_t)L.blocks_per_cu * (uint64_t)t->num_cus;
    if (grid > cap) grid = cap;
  }
  if (grid > 0x7fffffffull) grid = 0x7fffffffull;
  hipLaunchKernelGGL((lookup_lds<WAVES, MODE>), dim3((uint32_t)grid), dim3(64 * WAVES), 0, s,
                     reinterpret_cast<const uint4 *>(t->d_table), keys, n, t->log2_buckets,
                     t->seed, found, vals);
  return hipGetLastError();
}

template <uint32_t MODE>
hipError_t launch_mode(const ckpp_table *t, const uint4 *keys, uint64_t n, uint8_t *found,
                       uint64_t *vals, hipStream_t s) {
  switch (t->lookup_launch.block) {
    case 64: return launch_shape<1, MODE>(t, keys, n, found, vals, s);
    case 128: return launch_shape<2, MODE>(t, keys, n, found, vals, s);
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
