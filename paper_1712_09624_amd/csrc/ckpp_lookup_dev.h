// ckpp_lookup_dev.h -- the lookup passes shared by every lookup kernel
// (one table, a plan of many tables, the serving loop).  See ckpp_lookup.hip
// for the lookup procedure and its GPU form.
#pragma once

#include "ckpp_device.h"
#include "ckpp_internal.h"

namespace ckpp {
namespace {

constexpr uint32_t kNoFetch = 0xffffffffu;  // bucket indices are < 2^29

// Lines of one wave: 64 lines x 8 quarters; lookup j's line at [8j, 8j+8).
constexpr uint32_t kWaveQuarters = 64 * 8;

// Cooperative fetch of one 128-byte line (half `half` of the bucket) for
// every lookup of the wave whose `bucket` is not kNoFetch: in round k the
// lanes 8g..8g+7 read the line of lookup 8k+g, and the line lands at
// lines[8(8k+g) .. 8(8k+g)+8), its quarters rotated (Mine): lane r reads
// quarter r ^ g, which lands at position r.  The eight lanes' requests still
// cover the whole line, one 128-byte request.  The buckets of the eight
// rounds are gathered first and waited for once: a wave that waits for each
// exchange before its load spends most of its time in those waits when it
// is alone on its SIMD.
__device__ __forceinline__ void fetch_lines(uint4 *lines, const uint4 *tab, uint32_t bucket,
                                            uint32_t half, uint32_t g, uint32_t r) {
  uint32_t b[8];
#pragma unroll
  for (uint32_t k = 0; k < 8; ++k)
    b[k] = (uint32_t)__builtin_amdgcn_ds_bpermute((int)((8u * k + g) << 2), (int)bucket);
#pragma unroll
  for (uint32_t k = 0; k < 8; ++k) {
    if (b[k] != kNoFetch) {
      const uint4 *src = tab + (uint64_t)b[k] * kQuartersPerBucket + 8u * half + (r ^ g);
      __builtin_amdgcn_global_load_lds(
          (const void __attribute__((address_space(1))) *)src,
          (void __attribute__((address_space(3))) *)(lines + 64u * k), 16, 0, 0);
    }
  }
}

// A lane's own line in the wave's LDS lines: quarter q of lookup j's line
// sits at 8j + (q ^ (j & 7)), so that when every lane reads the same
// quarter of its own line (the lines 128 bytes apart), eight neighbouring
// lanes hit eight different groups of LDS banks instead of one.
struct Mine {
  const uint4 *p;  // the line's first position
  uint32_t sw;     // j & 7
  __device__ __forceinline__ uint4 operator[](uint32_t q) const { return p[q ^ sw]; }
  __device__ __forceinline__ Mine operator+(uint32_t quarters) const { return Mine{p + quarters, sw}; }
};

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

// `now` of a table without timers in a timed pass (a plan's kernel serves
// tables of both kinds with the timed passes): every entry counts and the
// whole word is the value.
constexpr uint32_t kNoTime = 0x10000u;

// A slot answers the lookup iff its full key equals the searched key and,
// with timers, its entry is alive at `now` (Sec. 4.2: expired entries are
// not considered); on a hit sets hit, val (the stored word, time included:
// hit_value gives the answer) and slot.
template <bool TIMED>
__device__ __forceinline__ void take_word(uint64_t w, uint32_t s, uint32_t now, bool &hit,
                                          uint64_t &val, uint32_t &slot) {
  const bool timed = TIMED && now < kNoTime;
  if (!timed || word_alive(w, now)) {
    hit = true;
    val = w;
    slot = s;
  }
}

// The answer of a hit whose stored word is w: the word without its time on a
// table with timers, else the word.
template <bool TIMED>
__device__ __forceinline__ uint64_t hit_value(uint64_t w, uint32_t now) {
  return TIMED && now < kNoTime ? (w & kValueMask) : w;
}


// Compares the key with the candidate slots `cand` (ascending) of a first
// line (mine[0..7]).
template <bool TIMED>
__device__ __forceinline__ void match_line0(Mine mine, uint32_t cand, uint4 key,
                                            uint32_t now, bool &hit, uint64_t &val,
                                            uint32_t &slot) {
  while (cand != 0u && !hit) {
    const uint32_t s = (uint32_t)__builtin_ctz(cand);
    cand &= cand - 1u;
    if (key_eq(mine[2u + s], key))
      take_word<TIMED>(quarter_value(mine[6u + (s >> 1)], s), s, now, hit, val, slot);
  }
}

// Same for slots 4..7 on a second line (mine[0..7]).
template <bool TIMED>
__device__ __forceinline__ void match_line1(Mine mine, uint32_t cand, uint4 key,
                                            uint32_t now, bool &hit, uint64_t &val,
                                            uint32_t &slot) {
  while (cand != 0u && !hit) {
    const uint32_t s = (uint32_t)__builtin_ctz(cand);
    cand &= cand - 1u;
    if (key_eq(mine[s - 4u], key))
      take_word<TIMED>(quarter_value(mine[4u + ((s - 4u) >> 1)], s), s, now, hit, val, slot);
  }
}

// LDS line buffers of one wave and the lane's place in them: `lines` holds
// the wave's first (or only) buffer, lookup j's line at quarters 8j..8j+7;
// `lines_a` the secondary lines of the pessimistic mode, which fetches both
// buckets at once (the same buffer when the kernel keeps one per wave).
struct Wave {
  uint4 *lines, *lines_a;
  Mine mine, mine_a;
  uint32_t lane, g, r;
};

template <uint32_t NB>
__device__ __forceinline__ Wave wave_lines(uint4 *s_lines) {
  Wave w;
  w.lane = threadIdx.x & 63u;
  w.g = w.lane >> 3;
  w.r = w.lane & 7u;
  w.lines = s_lines + (threadIdx.x >> 6) * NB * kWaveQuarters;
  w.lines_a = w.lines + (NB - 1) * kWaveQuarters;
  w.mine = Mine{w.lines + 8u * w.lane, w.r};
  w.mine_a = Mine{w.lines_a + 8u * w.lane, w.r};
  return w;
}

// What a lookup needs of its table.  Timers (tables with timers only): the
// current time, and whether a hit sets the entry's expiration time to
// `expiry` (Sec. 4.2: a lookup may update it).
struct TableRef {
  const uint4 *tab;
  uint64_t seed;
  uint32_t log2b;
  uint32_t now = 0u;
  uint32_t refresh = 0u;
  uint32_t expiry = 0u;
};

// A renewing lookup (Sec. 4.2) that found the entry with stored word w
// writes its new expiration time only when the time differs: rewriting the
// same time would dirty the line for nothing (hot keys found again and
// again at one time).
__device__ __forceinline__ bool needs_refresh(const TableRef &T, uint64_t w) {
  return (uint32_t)(w >> kTimerShift) != T.expiry;
}

// Writes the new expiration time of the entry in slot s of bucket b: the
// high 16 bits of its value word, nothing else.  Lookups of the same batch
// may read the word meanwhile; they see the old or the new time, and both
// are alive at `now`, so their answers do not depend on the order.
// The store is a relaxed agent-scope atomic, performed where the accesses of
// every XCD meet (like the words written under a bucket lock), so an insert
// or delete running on another XCD after a grid barrier of the serving loop
// reads the new time without a write-back of this XCD's L2 cache.
__device__ __forceinline__ void refresh_entry(const TableRef &T, uint32_t b, uint32_t s) {
  const uint32_t off = s < 4u ? 96u + 8u * s : 192u + 8u * (s - 4u);
  uint8_t *base = reinterpret_cast<uint8_t *>(const_cast<uint4 *>(T.tab)) +
                  (uint64_t)b * kBucketBytes + off + kTimerShift / 8u;
  __hip_atomic_store(reinterpret_cast<uint16_t *>(base), (uint16_t)T.expiry, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint4 zero4() { return make_uint4(0u, 0u, 0u, 0u); }

// One pass of a wave over 64 lookups, one per lane (the lane's `key`, a
// real lookup iff `ok`), in mode MODE; the result goes to *found / *val.
// `pre` runs once the first lines are requested and before they are waited
// for: the caller loads its next keys there.  The pessimistic mode needs a
// wave with two line buffers; the other modes use the first one only.
template <uint32_t MODE, bool TIMED = false, class Pre>
__device__ __forceinline__ void lds_pass(const Wave &w, const TableRef &T, uint4 key, bool ok,
                                         uint8_t *found, uint64_t *val_out, Pre &&pre) {
  // the secondary's lines: the second buffer in the pessimistic mode (fetched
  // with the primary), else the first one again (fetched after it)
  uint4 *const lines_a = MODE == kModeBoth ? w.lines_a : w.lines;
  const Mine mine_a = MODE == kModeBoth ? w.mine_a : w.mine;
  const KeyFields f = key_fields(key_hash(key, T.seed), T.log2b);
  // first line of the primary (and, pessimistic mode, the secondary)
  fetch_lines(w.lines, T.tab, ok ? f.p : kNoFetch, 0u, w.g, w.r);
  if (MODE == kModeBoth) fetch_lines(lines_a, T.tab, ok ? f.a : kNoFetch, 0u, w.g, w.r);
  pre();
  lines_landed();
  bool hit = false;
  uint64_t val = 0;
  uint32_t slot = 0u;
  const uint4 t0 = w.mine[0], t1 = w.mine[1];
  const uint32_t cand = ok ? (tag_eq_mask(t0, f.tag) & meta_busy(t1.z)) : 0u;
  const bool pass = MODE != kModeCuckoopp || bloom_pass(t1, f.bloom_bits);
  match_line0<TIMED>(w.mine, cand & 0xfu, key, T.now, hit, val, slot);
  // second line of the primary, for keys whose tag sits in slots 4..7
  bool need = !hit && (cand & 0xf0u);
  if (__builtin_amdgcn_ballot_w64(need)) {
    fetch_lines(w.lines, T.tab, need ? f.p : kNoFetch, 1u, w.g, w.r);
    lines_landed();
    if (need) match_line1<TIMED>(w.mine, cand & 0xf0u, key, T.now, hit, val, slot);
  }
  const bool hit_primary = hit;
  // secondary bucket
  need = ok && !hit && pass;
  if (__builtin_amdgcn_ballot_w64(need)) {
    if (MODE != kModeBoth) {
      fetch_lines(w.lines, T.tab, need ? f.a : kNoFetch, 0u, w.g, w.r);
      lines_landed();
    }
    uint32_t cand2 = 0u;
    if (need) {
      const uint4 u0 = mine_a[0], u1 = mine_a[1];
      cand2 = tag_eq_mask(u0, f.tag) & meta_busy(u1.z);
      match_line0<TIMED>(mine_a, cand2 & 0xfu, key, T.now, hit, val, slot);
    }
    need = need && !hit && (cand2 & 0xf0u);
    if (__builtin_amdgcn_ballot_w64(need)) {
      fetch_lines(lines_a, T.tab, need ? f.a : kNoFetch, 1u, w.g, w.r);
      lines_landed();
      if (need) match_line1<TIMED>(mine_a, cand2 & 0xf0u, key, T.now, hit, val, slot);
    }
  }
  if (TIMED && T.refresh && ok && hit && needs_refresh(T, val))
    refresh_entry(T, hit_primary ? f.p : f.a, slot);
  if (ok) {
    __builtin_nontemporal_store((uint8_t)(hit ? 1 : 0), found);
    __builtin_nontemporal_store(hit ? hit_value<TIMED>(val, T.now) : 0ull, val_out);
  }
}

// Register-landing counterpart of fetch_lines: the same rounds, but the
// quarter arrives in q[k] of the fetching lane; park_lines() later writes
// the quarters to LDS in exactly the layout fetch_lines produces.
__device__ __forceinline__ void fetch_lines_reg(uint4 (&q)[8], const uint4 *tab, uint32_t bucket,
                                                uint32_t half, uint32_t g, uint32_t r) {
  uint32_t b[8];
#pragma unroll
  for (uint32_t k = 0; k < 8; ++k)
    b[k] = (uint32_t)__builtin_amdgcn_ds_bpermute((int)((8u * k + g) << 2), (int)bucket);
#pragma unroll
  for (uint32_t k = 0; k < 8; ++k) {
    q[k] = zero4();
    if (b[k] != kNoFetch) q[k] = tab[(uint64_t)b[k] * kQuartersPerBucket + 8u * half + (r ^ g)];
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
  bool ok, hit, pass, hit_primary;
  uint32_t cand, slot;
  uint64_t val;
};

template <bool TIMED>
__device__ __forceinline__ void first_line(Mine mine, Look &L, uint32_t mode,
                                           uint32_t now) {
  const uint4 t0 = mine[0], t1 = mine[1];
  L.cand = L.ok ? (tag_eq_mask(t0, L.f.tag) & meta_busy(t1.z)) : 0u;
  L.pass = mode != kModeCuckoopp || bloom_pass(t1, L.f.bloom_bits);
  match_line0<TIMED>(mine, L.cand & 0xfu, L.key, now, L.hit, L.val, L.slot);
}

// One pass of a wave over 128 lookups, two per lane (A and B): for each
// phase the lines of the A lookups land in LDS directly, those of the B
// lookups in registers, which are parked in LDS once the A lookups have been
// analysed -- twice the line requests in flight for the same LDS.  `pre` as
// in lds_pass.  Not for the pessimistic mode.
template <uint32_t MODE, bool TIMED = false, class Pre>
__device__ __forceinline__ void dual_pass(const Wave &w, const TableRef &T, uint4 ka, bool oka,
                                          uint4 kb, bool okb, uint8_t *fa, uint64_t *va,
                                          uint8_t *fb, uint64_t *vb, Pre &&pre) {
  static_assert(MODE != kModeBoth, "the pessimistic mode runs in lds_pass");
  const uint32_t lane = w.lane, g = w.g, r = w.r;
  uint4 *lines = w.lines;
  const Mine mine = w.mine;
  Look A, Bq;
  A.key = ka;
  Bq.key = kb;
  A.ok = oka;
  Bq.ok = okb;
  A.f = key_fields(key_hash(A.key, T.seed), T.log2b);
  Bq.f = key_fields(key_hash(Bq.key, T.seed), T.log2b);
  A.hit = Bq.hit = false;
  A.val = Bq.val = 0ull;
  A.slot = Bq.slot = 0u;
  const uint32_t now = T.now;
  uint4 q[8];
  // phase 1: primary first lines
  fetch_lines(lines, T.tab, A.ok ? A.f.p : kNoFetch, 0u, g, r);
  fetch_lines_reg(q, T.tab, Bq.ok ? Bq.f.p : kNoFetch, 0u, g, r);
  pre();
  lines_landed();
  first_line<TIMED>(mine, A, MODE, now);
  park_lines(lines, q, lane);
  first_line<TIMED>(mine, Bq, MODE, now);
  // phase 2: primary second lines
  bool na = !A.hit && (A.cand & 0xf0u), nb = !Bq.hit && (Bq.cand & 0xf0u);
  if (__builtin_amdgcn_ballot_w64(na || nb)) {
    fetch_lines(lines, T.tab, na ? A.f.p : kNoFetch, 1u, g, r);
    fetch_lines_reg(q, T.tab, nb ? Bq.f.p : kNoFetch, 1u, g, r);
    lines_landed();
    if (na) match_line1<TIMED>(mine, A.cand & 0xf0u, A.key, now, A.hit, A.val, A.slot);
    park_lines(lines, q, lane);
    if (nb) match_line1<TIMED>(mine, Bq.cand & 0xf0u, Bq.key, now, Bq.hit, Bq.val, Bq.slot);
  }
  A.hit_primary = A.hit;
  Bq.hit_primary = Bq.hit;
  // phase 3: secondary first lines
  na = A.ok && !A.hit && A.pass;
  nb = Bq.ok && !Bq.hit && Bq.pass;
  if (__builtin_amdgcn_ballot_w64(na || nb)) {
    fetch_lines(lines, T.tab, na ? A.f.a : kNoFetch, 0u, g, r);
    fetch_lines_reg(q, T.tab, nb ? Bq.f.a : kNoFetch, 0u, g, r);
    lines_landed();
    uint32_t ca = 0u, cb = 0u;
    if (na) {
      ca = tag_eq_mask(mine[0], A.f.tag) & meta_busy(mine[1].z);
      match_line0<TIMED>(mine, ca & 0xfu, A.key, now, A.hit, A.val, A.slot);
    }
    park_lines(lines, q, lane);
    if (nb) {
      cb = tag_eq_mask(mine[0], Bq.f.tag) & meta_busy(mine[1].z);
      match_line0<TIMED>(mine, cb & 0xfu, Bq.key, now, Bq.hit, Bq.val, Bq.slot);
    }
    // phase 4: secondary second lines
    na = na && !A.hit && (ca & 0xf0u);
    nb = nb && !Bq.hit && (cb & 0xf0u);
    if (__builtin_amdgcn_ballot_w64(na || nb)) {
      fetch_lines(lines, T.tab, na ? A.f.a : kNoFetch, 1u, g, r);
      fetch_lines_reg(q, T.tab, nb ? Bq.f.a : kNoFetch, 1u, g, r);
      lines_landed();
      if (na) match_line1<TIMED>(mine, ca & 0xf0u, A.key, now, A.hit, A.val, A.slot);
      park_lines(lines, q, lane);
      if (nb) match_line1<TIMED>(mine, cb & 0xf0u, Bq.key, now, Bq.hit, Bq.val, Bq.slot);
    }
  }
  if (TIMED && T.refresh) {
    if (A.ok && A.hit && needs_refresh(T, A.val))
      refresh_entry(T, A.hit_primary ? A.f.p : A.f.a, A.slot);
    if (Bq.ok && Bq.hit && needs_refresh(T, Bq.val))
      refresh_entry(T, Bq.hit_primary ? Bq.f.p : Bq.f.a, Bq.slot);
  }
  if (A.ok) {
    __builtin_nontemporal_store((uint8_t)(A.hit ? 1 : 0), fa);
    __builtin_nontemporal_store(A.hit ? hit_value<TIMED>(A.val, T.now) : 0ull, va);
  }
  if (Bq.ok) {
    __builtin_nontemporal_store((uint8_t)(Bq.hit ? 1 : 0), fb);
    __builtin_nontemporal_store(Bq.hit ? hit_value<TIMED>(Bq.val, T.now) : 0ull, vb);
  }
}

// ---- One lane per lookup, lines in registers -----------------------------
// Each lane fetches the 32-byte head of its own bucket (tags, filter, masks:
// two 16-byte loads of the first line, one memory request) into registers,
// and only for tag matches the candidate's key and value word (the same
// line for slots 0..3, the second for 4..7).  A negative lookup keeps 8
// registers per lookup in flight and no LDS, so a lane can own PER lookups
// and a compute unit keeps far more lines in flight than with lines landing
// in LDS; a positive lookup reads its line twice (head, then key), which
// costs a second request when the line has left the L2 in between.

template <uint32_t PER>
struct RegLooks {
  uint4 key[PER];
  KeyFields f[PER];
  uint4 h0[PER], h1[PER];  // head of the bucket being probed
  uint32_t cand[PER], slot[PER];
  bool ok[PER], hit[PER], pass[PER], hit_primary[PER];
  uint64_t val[PER];
};

__device__ __forceinline__ const uint8_t *bucket_bytes(const uint4 *tab, uint32_t b) {
  return reinterpret_cast<const uint8_t *>(tab) + (uint64_t)b * kBucketBytes;
}

// Probes the candidates of every lookup (ascending slot order), one
// candidate per lookup per round trip, until each has a hit or none left.
template <bool TIMED, uint32_t PER>
__device__ __forceinline__ void reg_match(const uint4 *tab, RegLooks<PER> &L, const uint32_t *b,
                                          uint32_t now) {
  for (;;) {
    uint4 k[PER];
    uint64_t w[PER];
    uint32_t s[PER];
    bool any = false;
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) {
      s[j] = kSlots;
      if (L.cand[j] != 0u && !L.hit[j]) {
        s[j] = (uint32_t)__builtin_ctz(L.cand[j]);
        L.cand[j] &= L.cand[j] - 1u;
        const uint8_t *base = bucket_bytes(tab, b[j]);
        const uint32_t ko = s[j] < 4u ? 32u + 16u * s[j] : 128u + 16u * (s[j] - 4u);
        const uint32_t vo = s[j] < 4u ? 96u + 8u * s[j] : 192u + 8u * (s[j] - 4u);
        k[j] = *reinterpret_cast<const uint4 *>(base + ko);
        w[j] = *reinterpret_cast<const uint64_t *>(base + vo);
        any = true;
      }
    }
    if (!any) break;
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j)
      if (s[j] < kSlots && key_eq(k[j], L.key[j]))
        take_word<TIMED>(w[j], s[j], now, L.hit[j], L.val[j], L.slot[j]);
  }
}

// One pass of a wave over 64 * PER lookups, PER per lane (the lane's
// key[j], a real lookup iff ok[j]); lookup j's answer goes to *found[j] /
// *vals[j].  `pre` runs once the first heads are requested.  SYS: the
// answers are written through to memory (system-scope stores), visible to
// the host once the wave has waited for its stores.
template <uint32_t MODE, bool TIMED, uint32_t PER, bool SYS = false, class Pre>
__device__ __forceinline__ void reg_pass_to(const TableRef &T, const uint4 (&key)[PER],
                                            const bool (&ok)[PER], uint8_t *const (&found)[PER],
                                            uint64_t *const (&vals)[PER], Pre &&pre) {
  RegLooks<PER> L;
  uint32_t b[PER];
  uint4 g0[PER], g1[PER];  // pessimistic mode: head of the secondary, fetched with the primary
#pragma unroll
  for (uint32_t j = 0; j < PER; ++j) {
    L.key[j] = key[j];
    L.ok[j] = ok[j];
    L.hit[j] = false;
    L.val[j] = 0ull;
    L.slot[j] = 0u;
    L.f[j] = key_fields(key_hash(key[j], T.seed), T.log2b);
    L.h0[j] = L.h1[j] = g0[j] = g1[j] = zero4();
    if (ok[j]) {
      const uint4 *q = T.tab + (uint64_t)L.f[j].p * kQuartersPerBucket;
      L.h0[j] = q[0];
      L.h1[j] = q[1];
      if (MODE == kModeBoth) {
        const uint4 *r = T.tab + (uint64_t)L.f[j].a * kQuartersPerBucket;
        g0[j] = r[0];
        g1[j] = r[1];
      }
    }
  }
  pre();
  // A lookup with no tag candidate in its primary cannot hit there: if it
  // needs the secondary (the filter passes, or the mode always looks), the
  // secondary's head is requested now, in the round trip of the other
  // lookups' primary keys and values, instead of one round trip later.
  // The requests are the same; only their order changes.
  bool early[PER];
#pragma unroll
  for (uint32_t j = 0; j < PER; ++j) {
    L.cand[j] = L.ok[j] ? (tag_eq_mask(L.h0[j], L.f[j].tag) & meta_busy(L.h1[j].z)) : 0u;
    L.pass[j] = MODE != kModeCuckoopp || bloom_pass(L.h1[j], L.f[j].bloom_bits);
    b[j] = L.f[j].p;
    early[j] = MODE != kModeBoth && L.ok[j] && L.cand[j] == 0u && L.pass[j];
    if (early[j]) {
      const uint4 *q = T.tab + (uint64_t)L.f[j].a * kQuartersPerBucket;
      g0[j] = q[0];
      g1[j] = q[1];
    }
  }
  reg_match<TIMED, PER>(T.tab, L, b, T.now);
  bool need_any = false;
#pragma unroll
  for (uint32_t j = 0; j < PER; ++j) {
    L.hit_primary[j] = L.hit[j];
    const bool need = L.ok[j] && !L.hit[j] && L.pass[j];
    L.cand[j] = 0u;
    b[j] = L.f[j].a;
    if (need) {
      if (MODE != kModeBoth && !early[j]) {
        const uint4 *q = T.tab + (uint64_t)L.f[j].a * kQuartersPerBucket;
        g0[j] = q[0];
        g1[j] = q[1];
      }
      need_any = true;
    }
    L.pass[j] = need;
  }
  if (need_any) {
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j)
      if (L.pass[j]) L.cand[j] = tag_eq_mask(g0[j], L.f[j].tag) & meta_busy(g1[j].z);
    reg_match<TIMED, PER>(T.tab, L, b, T.now);
  }
#pragma unroll
  for (uint32_t j = 0; j < PER; ++j) {
    if (!L.ok[j]) continue;
    if (TIMED && T.refresh && L.hit[j] && needs_refresh(T, L.val[j]))
      refresh_entry(T, L.hit_primary[j] ? L.f[j].p : L.f[j].a, L.slot[j]);
    const uint8_t fj = L.hit[j] ? 1 : 0;
    const uint64_t vj = L.hit[j] ? hit_value<TIMED>(L.val[j], T.now) : 0ull;
    if (SYS) {
      __hip_atomic_store(found[j], fj, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(vals[j], vj, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    } else {
      __builtin_nontemporal_store(fj, found[j]);
      __builtin_nontemporal_store(vj, vals[j]);
    }
  }
}

// reg_pass_to over a tile: lookup j of lane l is lookup 64 j + l of the
// tile, its results at found[64 j] / vals[64 j] (the caller offsets both by
// the lane).
template <uint32_t MODE, bool TIMED, uint32_t PER, class Pre>
__device__ __forceinline__ void reg_pass(const TableRef &T, const uint4 (&key)[PER],
                                         const bool (&ok)[PER], uint8_t *found, uint64_t *vals,
                                         Pre &&pre) {
  uint8_t *fo[PER];
  uint64_t *vo[PER];
#pragma unroll
  for (uint32_t j = 0; j < PER; ++j) {
    fo[j] = found + 64u * j;
    vo[j] = vals + 64u * j;
  }
  reg_pass_to<MODE, TIMED, PER>(T, key, ok, fo, vo, pre);
}

// ---- Four lanes per lookup, lines in registers ----------------------------
// A quad of lanes (4q .. 4q+3) owns four lookups, one per lane, and reads
// each of their lines together: lane j of the quad loads the line's j-th
// 32-byte chunk (two 16-byte loads; the quad's loads of one line make one
// memory request).  The chunks of a first line are the header (tags, filter,
// masks) | keys of slots 0,1 | keys of slots 2,3 | value words of slots
// 0..3; of a second line keys 4,5 | keys 6,7 | value words 4..7 | other[]
// (not read).  A line is analysed where it lies: the header lane finds the
// tag candidates and the filter test, the key lanes compare full keys, the
// value lane picks the value; quad_perm DPP moves carry the lookup's key
// and fields to the quad and the answer back to the lookup's lane.  No LDS;
// 8 registers per line in flight per lane.

template <uint32_t R>
struct QuadR {
  static constexpr uint32_t value = R;
};

// Runs f(QuadR<R>{}) for R = 0..3 (R a constant inside f, as DPP needs).
template <class F>
__device__ __forceinline__ void each_of_quad(F &&f) {
  f(QuadR<0>{});
  f(QuadR<1>{});
  f(QuadR<2>{});
  f(QuadR<3>{});
}

// Value of v in lane R of the caller's quad.  Every lane of the wave must be
// active (DPP reads the other lane's register).
template <uint32_t R>
__device__ __forceinline__ uint32_t quad_get(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, (int)(R * 0x55u), 0xf, 0xf, false);
}

template <uint32_t R>
__device__ __forceinline__ uint4 quad_get4(uint4 v) {
  return make_uint4(quad_get<R>(v.x), quad_get<R>(v.y), quad_get<R>(v.z), quad_get<R>(v.w));
}

// OR of v over the caller's quad.
__device__ __forceinline__ uint32_t quad_or(uint32_t v) {
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xb1, 0xf, 0xf, false);  // lanes 1,0,3,2
  v |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4e, 0xf, 0xf, false);  // lanes 2,3,0,1
  return v;
}

// Line `H` of the bucket of each of the quad's lookups whose lane passes a
// bucket other than kNoFetch: c[R] receives this lane's chunk of lookup R's
// line (zero when not fetched).
template <uint32_t H>
__device__ __forceinline__ void quad_fetch(uint4 (&c)[4][2], const uint4 *tab, uint32_t bucket,
                                           uint32_t j) {
  each_of_quad([&](auto rc) {
    constexpr uint32_t R = decltype(rc)::value;
    const uint32_t b = quad_get<R>(bucket);
    c[R][0] = c[R][1] = zero4();
    if (b != kNoFetch && (H == 0u || j < 3u)) {
      const uint4 *src = tab + (uint64_t)b * kQuartersPerBucket + 8u * H + 2u * j;
      c[R][0] = src[0];
      c[R][1] = src[1];
    }
  });
}

// Answer of one line for one lookup, the same in every lane of the quad.
struct QuadAnswer {
  uint32_t cand;  // first line: tag candidates (tag match and busy)
  bool pass;      // first line: the filter holds both of the key's bits
  bool hit;
  uint32_t slot;
  uint64_t val;
};

// The value lane's part: the first slot of m (ascending) whose entry is
// alive picks its value word from the lane's two quarters (four words of
// consecutive slots from `first`); the answer is broadcast from lane VL.
template <bool TIMED, uint32_t VL>
__device__ __forceinline__ void quad_pick(const uint4 (&c)[2], uint32_t j, uint32_t m,
                                          uint32_t first, uint32_t now, QuadAnswer &A) {
  uint32_t res = 0u, lo = 0u, hi = 0u;
  if (j == VL) {
    uint64_t w[4];
    w[0] = (uint64_t)c[0].x | ((uint64_t)c[0].y << 32);
    w[1] = (uint64_t)c[0].z | ((uint64_t)c[0].w << 32);
    w[2] = (uint64_t)c[1].x | ((uint64_t)c[1].y << 32);
    w[3] = (uint64_t)c[1].z | ((uint64_t)c[1].w << 32);
    const bool timed = TIMED && now < kNoTime;
    uint32_t live = m;
    if (timed) {
#pragma unroll
      for (uint32_t s = 0; s < 4u; ++s)
        if (!word_alive(w[s], now)) live &= ~(1u << (first + s));
    }
    if (live != 0u) {
      const uint32_t s = (uint32_t)__builtin_ctz(live), i = s - first;
      // the stored word, time included (hit_value gives the answer)
      const uint64_t v = (i & 2u) ? ((i & 1u) ? w[3] : w[2]) : ((i & 1u) ? w[1] : w[0]);
      res = 1u | (s << 1);
      lo = (uint32_t)v;
      hi = (uint32_t)(v >> 32);
    }
  }
  res = quad_get<VL>(res);
  lo = quad_get<VL>(lo);
  hi = quad_get<VL>(hi);
  A.hit = (res & 1u) != 0u;
  A.slot = res >> 1;
  A.val = (uint64_t)lo | ((uint64_t)hi << 32);
}

// First line of a bucket for the quad's lookup whose key is k and whose tag
// and filter bits are packed in pk (tag | bit index 1 << 16 | bit index 2
// << 22): slots 0..3.
template <bool TIMED>
__device__ __forceinline__ QuadAnswer quad_first(const uint4 (&c)[2], uint32_t j, uint4 k,
                                                 uint32_t pk, uint32_t now) {
  uint32_t x = 0u;
  if (j == 0u) {
    const uint32_t cand = tag_eq_mask(c[0], pk & 0xffffu) & meta_busy(c[1].z);
    const uint64_t bits = (1ull << ((pk >> 16) & 63u)) | (1ull << ((pk >> 22) & 63u));
    x = (cand << 8) | (bloom_pass(c[1], bits) ? 0x10000u : 0u);
  } else if (j < 3u) {
    x = ((key_eq(c[0], k) ? 1u : 0u) | (key_eq(c[1], k) ? 2u : 0u)) << (2u * (j - 1u));
  }
  x = quad_or(x);
  QuadAnswer A;
  A.cand = (x >> 8) & 0xffu;
  A.pass = (x & 0x10000u) != 0u;
  quad_pick<TIMED, 3>(c, j, x & (x >> 8) & 0xfu, 0u, now, A);
  return A;
}

// Second line of a bucket: slots 4..7 among the candidates cm.
template <bool TIMED>
__device__ __forceinline__ QuadAnswer quad_second(const uint4 (&c)[2], uint32_t j, uint4 k,
                                                  uint32_t cm, uint32_t now) {
  uint32_t x = 0u;
  if (j < 2u) x = ((key_eq(c[0], k) ? 1u : 0u) | (key_eq(c[1], k) ? 2u : 0u)) << (4u + 2u * j);
  x = quad_or(x);
  QuadAnswer A;
  A.cand = 0u;
  A.pass = false;
  quad_pick<TIMED, 2>(c, j, x & cm & 0xf0u, 4u, now, A);
  return A;
}

// One pass of a wave over 64 * PER lookups (PER 1 or 2), four lanes per
// line: lookup j of lane l is lookup 64 j + l of the tile, its results at
// found[64 j] / vals[64 j] (the caller offsets both by the lane); the
// phases and answers are those of lds_pass.  `pre` runs once the first
// lines are requested.
template <uint32_t MODE, bool TIMED, uint32_t PER, class Pre>
__device__ __forceinline__ void quad_pass(const TableRef &T, const uint4 (&key)[PER],
                                          const bool (&ok)[PER], uint8_t *found, uint64_t *vals,
                                          Pre &&pre) {
  const uint32_t j = threadIdx.x & 3u;
  KeyFields f[PER];
  uint32_t pk[PER];  // tag | filter bit index 1 << 16 | index 2 << 22
  uint4 c[PER][4][2], d[PER][4][2];  // chunks of the primary's and the secondary's lines
#pragma unroll
  for (uint32_t p = 0; p < PER; ++p) {
    f[p] = key_fields(key_hash(key[p], T.seed), T.log2b);
    pk[p] = f[p].tag | (f[p].bidx << 16);
    quad_fetch<0>(c[p], T.tab, ok[p] ? f[p].p : kNoFetch, j);
    if (MODE == kModeBoth) quad_fetch<0>(d[p], T.tab, ok[p] ? f[p].a : kNoFetch, j);
  }
  pre();
  // the quad's keys and packed fields are fetched from their lanes where
  // used (a DPP move each) rather than held: registers are line slots
  bool hit[PER], pass[PER], hit_primary[PER], need[PER];
  uint64_t val[PER];
  uint32_t slot[PER], cand[PER];
  auto take = [&](uint32_t p, const QuadAnswer &A) {
    hit[p] = true;
    val[p] = A.val;
    slot[p] = A.slot;
  };
  bool any = false;
#pragma unroll
  for (uint32_t p = 0; p < PER; ++p) {
    hit[p] = pass[p] = false;
    val[p] = 0ull;
    slot[p] = cand[p] = 0u;
    each_of_quad([&](auto rc) {
      constexpr uint32_t R = decltype(rc)::value;
      const QuadAnswer A =
          quad_first<TIMED>(c[p][R], j, quad_get4<R>(key[p]), quad_get<R>(pk[p]), T.now);
      if (j == R && ok[p]) {
        cand[p] = A.cand;
        pass[p] = MODE != kModeCuckoopp || A.pass;
        if (A.hit) take(p, A);
      }
    });
    // second line of the primary, for keys whose tag sits in slots 4..7
    need[p] = !hit[p] && (cand[p] & 0xf0u);
    any = any || need[p];
  }
  if (__builtin_amdgcn_ballot_w64(any)) {
#pragma unroll
    for (uint32_t p = 0; p < PER; ++p)
      quad_fetch<1>(c[p], T.tab, need[p] ? f[p].p : kNoFetch, j);
#pragma unroll
    for (uint32_t p = 0; p < PER; ++p) {
      const uint32_t cm = need[p] ? cand[p] : 0u;
      each_of_quad([&](auto rc) {
        constexpr uint32_t R = decltype(rc)::value;
        const QuadAnswer A =
            quad_second<TIMED>(c[p][R], j, quad_get4<R>(key[p]), quad_get<R>(cm), T.now);
        if (j == R && need[p] && A.hit) take(p, A);
      });
    }
  }
  // secondary bucket
  any = false;
#pragma unroll
  for (uint32_t p = 0; p < PER; ++p) {
    hit_primary[p] = hit[p];
    need[p] = ok[p] && !hit[p] && pass[p];
    any = any || need[p];
  }
  if (__builtin_amdgcn_ballot_w64(any)) {
    if (MODE != kModeBoth) {
#pragma unroll
      for (uint32_t p = 0; p < PER; ++p)
        quad_fetch<0>(d[p], T.tab, need[p] ? f[p].a : kNoFetch, j);
    }
    any = false;
#pragma unroll
    for (uint32_t p = 0; p < PER; ++p) {
      uint32_t cand2 = 0u;
      each_of_quad([&](auto rc) {
        constexpr uint32_t R = decltype(rc)::value;
        const QuadAnswer A =
            quad_first<TIMED>(d[p][R], j, quad_get4<R>(key[p]), quad_get<R>(pk[p]), T.now);
        if (j == R && need[p]) {
          cand2 = A.cand;
          if (A.hit) take(p, A);
        }
      });
      cand[p] = cand2;
      need[p] = need[p] && !hit[p] && (cand2 & 0xf0u);
      any = any || need[p];
    }
    if (__builtin_amdgcn_ballot_w64(any)) {
#pragma unroll
      for (uint32_t p = 0; p < PER; ++p)
        quad_fetch<1>(d[p], T.tab, need[p] ? f[p].a : kNoFetch, j);
#pragma unroll
      for (uint32_t p = 0; p < PER; ++p) {
        const uint32_t cm = need[p] ? cand[p] : 0u;
        each_of_quad([&](auto rc) {
          constexpr uint32_t R = decltype(rc)::value;
          const QuadAnswer A =
              quad_second<TIMED>(d[p][R], j, quad_get4<R>(key[p]), quad_get<R>(cm), T.now);
          if (j == R && need[p] && A.hit) take(p, A);
        });
      }
    }
  }
#pragma unroll
  for (uint32_t p = 0; p < PER; ++p) {
    if (!ok[p]) continue;
    if (TIMED && T.refresh && hit[p] && needs_refresh(T, val[p]))
      refresh_entry(T, hit_primary[p] ? f[p].p : f[p].a, slot[p]);
    __builtin_nontemporal_store((uint8_t)(hit[p] ? 1 : 0), found + 64u * p);
    __builtin_nontemporal_store(hit[p] ? hit_value<TIMED>(val[p], T.now) : 0ull, vals + 64u * p);
  }
}

}  // namespace
}  // namespace ckpp
