// ckpp_update_dev.h -- per-key insert and delete (device functions shared by
// the batch kernels and the serving loop).
//
// Insert (Sec. 2 insertion procedure, Sec. 4.1 filter maintenance) and
// delete (Sec. 4.1) run as many independent lanes, one key at a time per
// lane, on a persistent grid.  Each bucket's lock word (bytes 28..31) is
// taken with a single compare-and-swap and never waited on: a lane that
// misses a lock drops every lock it holds and retries in its next loop
// iteration, so no lane ever spins on a lock that a lane of its own
// wavefront holds.  Every entry that moves is moved under the locks of both
// buckets it may live in, so every bloom-filter and moved-counter update --
// which concerns the primary bucket of the entry that moves -- happens under
// the lock of that bucket.  Inside a critical section every table word is
// read and written with device-coherent accesses, so a lock cycle flushes
// no cache (section_begin / section_end).
//
// A key's state machine:
//   DIRECT  lock p and a; if the key is present, replace its value
//           (UPDATED); else take the lowest free slot of p, else of a (set
//           the key's two bits in p's filter, moved[p] += 1) (INSERTED);
//           else, still under those locks, try a cuckoo path of one or two
//           displacements out of p (the buckets it touches are locked too),
//           and the key takes the freed slot of p (INSERTED); else WALK.
//   WALK    random walk over full buckets starting at p, reading without
//           locks, with one step of lookahead: at each bucket, if the other
//           bucket of some entry has a free slot, that entry (preferably one
//           going home to its primary) ends the path; else pick a victim --
//           preferably an entry that sits in its secondary bucket (it would
//           move back home), then one whose other bucket is not the bucket
//           just left -- and continue at the victim's other bucket, at most
//           max_kicks steps; no (bucket, slot) twice.  No path: FAILED.
//   MOVE    apply the path backwards, one displacement per iteration, each
//           under the locks of its two buckets and re-validated there; a
//           move from primary to secondary adds the entry to the source's
//           filter, a move back decrements the destination's counter and
//           resets its filter at zero (Sec. 4.1).  A stale path returns to
//           DIRECT (the moves done so far are valid moves); when the path is
//           applied, p has a free slot and the key returns to DIRECT.
// Every loop is bounded: walks by max_kicks, retries by the table's retry
// limit, whose exhaustion reports CKPP_RETRY for that key (nothing changed
// for it) and is counted separately.
//
// Timers (Sec. 4.2, tables with timers only): an entry's expiration time
// sits in the high 16 bits of its value word, so every move carries it
// along.  Only alive entries are present: an insert of a key whose entry has
// expired overwrites that entry where it stands (INSERTED), and a delete of
// it reports 0.  DIRECT takes a slot holding an expired entry as if it were
// free (lazy deletion), after a free one: the expired entry is removed first,
// with the counter update of its primary bucket when it sat in its secondary
// -- under the pair's locks when that primary is p or a, else under the
// primary's own lock, taken like the others (never waited on).  A cuckoo
// path still ends only at a bucket with a free slot.

#pragma once

#include "ckpp_device.h"
#include "ckpp_internal.h"

namespace ckpp {
namespace {

// Random draws of the path search: counter-based SplitMix64 streams keyed
// by the key's hash.  kGolden is SplitMix64's own increment (2^64 / golden
// ratio); the other two are arbitrary odd salts that separate the streams
// (the multiplier of the PCG/MMIX generator, and a second golden-ratio-like
// odd constant), with no arithmetic role beyond that.
constexpr uint64_t kGolden = 0x9e3779b97f4a7c15ull;
constexpr uint64_t kDisplaceSalt = 0x5851f42d4c957f2dull;
constexpr uint64_t kWalkSalt = 0xd1b54a32d192ed03ull;
constexpr uint32_t kMaxWalks = 64;         // path searches per key
constexpr uint32_t kNoBucket = 0xffffffffu;
// A cuckoo path entry: bucket (below 2^29) | slot << 29.
constexpr uint32_t kPathSlotShift = 29;
constexpr uint32_t kPathBucketMask = (1u << kPathSlotShift) - 1u;
static_assert(kMaxLog2Buckets <= kPathSlotShift, "path entries hold a bucket index");

__device__ __forceinline__ uint8_t *bucket_ptr(uint8_t *bk, uint32_t b) {
  return bk + (uint64_t)b * kBucketBytes;
}
__device__ __forceinline__ const uint8_t *bucket_ptr(const uint8_t *bk, uint32_t b) {
  return bk + (uint64_t)b * kBucketBytes;
}

__device__ __forceinline__ uint32_t *lock_word(uint8_t *bk, uint32_t b) {
  return reinterpret_cast<uint32_t *>(bucket_ptr(bk, b) + kLockOffset);
}

__device__ __forceinline__ bool try_lock(uint8_t *bk, uint32_t b) {
  uint32_t expected = 0u;
  return __hip_atomic_compare_exchange_strong(lock_word(bk, b), &expected, 1u, __ATOMIC_RELAXED,
                                              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void unlock(uint8_t *bk, uint32_t b) {
  __hip_atomic_store(lock_word(bk, b), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Ordering of a critical section.  Every table word a lane reads or writes
// under a lock goes through a device-coherent access (Coh below: relaxed
// agent-scope atomics, performed where every XCD's accesses meet), so
// taking and dropping a lock needs no flush of the per-XCD L2 caches.
// Acquire: the section's accesses are issued after the lock's CAS has
// returned (a compiler barrier keeps them there; the GPU issues a wave's
// memory accesses in order).  Release: the unlocking store waits until
// every access of the section has completed.
__device__ __forceinline__ void section_begin() { __atomic_signal_fence(__ATOMIC_SEQ_CST); }

__device__ __forceinline__ void section_end() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Takes the locks of buckets x != y in ascending order, or none.  The
// order makes retries live: of two lanes that need the same pair, the one
// that takes the lower lock first can always try the higher one, whereas
// two lanes taking the two locks at once could each get one, give both
// back, and repeat in lockstep forever.  On success the caller's later
// reads see every write made under these locks by earlier holders.
__device__ __forceinline__ bool lock_two(uint8_t *bk, uint32_t x, uint32_t y) {
  const uint32_t lo = x < y ? x : y, hi = x < y ? y : x;
  if (!try_lock(bk, lo)) return false;
  if (!try_lock(bk, hi)) {
    unlock(bk, lo);
    return false;
  }
  section_begin();
  return true;
}

// Publishes the writes made under the locks, then drops both locks.
__device__ __forceinline__ void unlock_two(uint8_t *bk, uint32_t x, uint32_t y) {
  section_end();
  unlock(bk, x);
  unlock(bk, y);
}

// A table word read and written with device-coherent accesses (relaxed
// agent-scope atomics): converts to its value, assigns with a store.
template <class T>
struct Coh {
  T *p;
  __device__ __forceinline__ operator T() const {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ __forceinline__ const Coh &operator=(T v) const {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return *this;
  }
  __device__ __forceinline__ const Coh &operator|=(T v) const { return *this = (T)(T(*this) | v); }
};

// A 16-byte key: two 8-byte halves (a lock guards it, so halves suffice).
template <>
struct Coh<uint4> {
  uint4 *p;
  __device__ __forceinline__ operator uint4() const {
    const uint64_t *q = reinterpret_cast<const uint64_t *>(p);
    const uint64_t lo = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t hi = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
  }
  __device__ __forceinline__ const Coh &operator=(uint4 v) const {
    uint64_t *q = reinterpret_cast<uint64_t *>(p);
    __hip_atomic_store(q, (uint64_t)v.x | ((uint64_t)v.y << 32), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(q + 1, (uint64_t)v.z | ((uint64_t)v.w << 32), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    return *this;
  }
};

// Address of table words of type T: `*` and `[]` give coherent words; p is
// the raw address (for read-modify-write atomics).
template <class T>
struct CohPtr {
  T *p;
  __device__ __forceinline__ Coh<T> operator*() const { return Coh<T>{p}; }
  __device__ __forceinline__ Coh<T> operator[](uint32_t i) const { return Coh<T>{p + i}; }
};

struct Head {
  uint4 q0;  // tags
  uint4 q1;  // bloom lo, bloom hi, meta, lock
};

__device__ __forceinline__ Head read_head(uint8_t *bk, uint32_t b) {
  uint4 *q = reinterpret_cast<uint4 *>(bucket_ptr(bk, b));
  Head h;
  h.q0 = Coh<uint4>{q};
  h.q1 = Coh<uint4>{q + 1};
  return h;
}

__device__ __forceinline__ CohPtr<uint32_t> meta_ptr(uint8_t *bk, uint32_t b) {
  return {reinterpret_cast<uint32_t *>(bucket_ptr(bk, b) + kMetaOffset)};
}
__device__ __forceinline__ CohPtr<uint64_t> bloom_ptr(uint8_t *bk, uint32_t b) {
  return {reinterpret_cast<uint64_t *>(bucket_ptr(bk, b) + 16)};
}
__device__ __forceinline__ CohPtr<uint16_t> tag_ptr(uint8_t *bk, uint32_t b) {
  return {reinterpret_cast<uint16_t *>(bucket_ptr(bk, b))};
}
__device__ __forceinline__ CohPtr<uint32_t> other_ptr(uint8_t *bk, uint32_t b) {
  return {reinterpret_cast<uint32_t *>(bucket_ptr(bk, b) + kOtherOffset)};
}
__device__ __forceinline__ CohPtr<uint4> key_ptr(uint8_t *bk, uint32_t b, uint32_t s) {
  return {reinterpret_cast<uint4 *>(bucket_ptr(bk, b) + key_offset(s))};
}
__device__ __forceinline__ CohPtr<uint64_t> value_ptr(uint8_t *bk, uint32_t b, uint32_t s) {
  return {reinterpret_cast<uint64_t *>(bucket_ptr(bk, b) + value_offset(s))};
}

// Slot of `key` in a bucket whose head is h (bucket locked), or -1.
__device__ __forceinline__ int find_slot(uint8_t *bk, uint32_t b, const Head &h, uint4 key,
                                         uint32_t tag) {
  uint32_t cand = tag_eq_mask(h.q0, tag) & meta_busy(h.q1.z);
  while (cand) {
    const uint32_t s = (uint32_t)__builtin_ctz(cand);
    cand &= cand - 1u;
    if (key_eq(*key_ptr(bk, b, s), key)) return (int)s;
  }
  return -1;
}

__device__ __forceinline__ void write_entry(uint8_t *bk, uint32_t b, uint32_t s, uint4 key,
                                            uint64_t value, uint32_t tag, uint32_t other) {
  *key_ptr(bk, b, s) = key;
  *value_ptr(bk, b, s) = value;
  tag_ptr(bk, b)[s] = (uint16_t)tag;
  other_ptr(bk, b)[s] = other;
}

// Index of the k-th set bit of m (k < popcount(m)).
__device__ __forceinline__ uint32_t nth_bit(uint32_t m, uint32_t k) {
  for (uint32_t i = 0; i < k; ++i) m &= m - 1u;
  return (uint32_t)__builtin_ctz(m);
}

__device__ __forceinline__ uint64_t load_relaxed(const uint8_t *p) {
  return __hip_atomic_load(reinterpret_cast<const uint64_t *>(p), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// The paths that few keys take (displacements, the walk, a move, lazy
// removal) are kept out of line: inlined, they raise the register count and
// slow the direct path every key takes (measured: 2^24 build to load 0.95 in
// 211 ms inlined, 181 ms out of line).
constexpr int kBusy = -2;    // a lock was taken by another lane: retry
// DIRECT found a displacement path, but a bucket beyond the pair was locked
// by another lane or changed before it was locked: retry DIRECT (at most
// kDisplaceRetries times per key, then the walk).
constexpr int kDisplaceBusy = -3;
constexpr uint32_t kDisplaceRetries = 4;
constexpr int kNeedPath = -1;

// Busy slots of bucket b whose entries have expired at `now`.
__device__ __forceinline__ uint32_t expired_mask(uint8_t *bk, uint32_t b, uint32_t busy,
                                                 uint32_t now) {
  uint32_t m = 0u;
#pragma unroll
  for (uint32_t s = 0; s < kSlots; ++s)
    if (((busy >> s) & 1u) && !word_alive(*value_ptr(bk, b, s), now)) m |= 1u << s;
  return m;
}

// Working copy of the metadata of the two buckets a key may live in (both
// locked), written back once the insert is decided.
struct Pair {
  uint32_t b[2];
  uint32_t meta[2];
};

// moved - 1, and the filter of bucket y emptied when it reaches zero
// (Sec. 4.1); y's lock is held.
__device__ __forceinline__ uint32_t moved_down(uint8_t *bk, uint32_t y, uint32_t meta) {
  uint32_t mv = meta_moved(meta);
  if (mv > 0u) {
    mv -= 1u;
    if (mv == 0u) *bloom_ptr(bk, y) = 0ull;
  }
  return make_meta(mv, meta_busy(meta), meta_sec(meta));
}

// Removes the expired entry of slot s of the pair's bucket xi (lazy
// deletion, Sec. 4.2): its busy and sec bits are cleared in the working
// copy; if it sat in its secondary bucket, the moved counter of its primary
// y drops by one -- in the working copy when y is the pair's other bucket,
// else under y's lock, taken here.  Returns false, having changed nothing,
// when y's lock is held by another lane.
__device__ __attribute__((noinline)) bool remove_expired(uint8_t *bk, Pair &P, int xi, uint32_t s, bool plain) {
  const uint32_t bit = 1u << s;
  if (!plain && (meta_sec(P.meta[xi]) & bit)) {
    const uint32_t y = other_ptr(bk, P.b[xi])[s];
    const int yi = y == P.b[0] ? 0 : (y == P.b[1] ? 1 : -1);
    if (yi >= 0) {
      P.meta[yi] = moved_down(bk, y, P.meta[yi]);
    } else {
      if (!try_lock(bk, y)) return false;
      section_begin();
      *meta_ptr(bk, y) = moved_down(bk, y, *meta_ptr(bk, y));
      section_end();
      unlock(bk, y);
    }
  }
  P.meta[xi] = make_meta(meta_moved(P.meta[xi]), meta_busy(P.meta[xi]) & ~bit,
                         meta_sec(P.meta[xi]) & ~bit);
  return true;
}

// Moves the entry of slot s of bucket x into the free slot fs of its other
// bucket y (both locked), with the filter maintenance of a cuckoo move
// (Sec. 4.1): an entry leaving its primary x adds its two bits to x's
// filter and 1 to x's moved counter; an entry going home to y takes 1 off
// y's counter and empties y's filter when it reaches zero.  The metadata
// words are read and written in memory.
__device__ void move_locked(uint8_t *bk, uint32_t x, uint32_t s, uint32_t y, uint32_t fs,
                            uint32_t log2b, uint64_t seed, bool plain) {
  const uint32_t mx = *meta_ptr(bk, x), my = *meta_ptr(bk, y);
  const uint4 k = *key_ptr(bk, x, s);
  const uint64_t w = *value_ptr(bk, x, s);
  const uint32_t tag = tag_ptr(bk, x)[s];
  const bool guest = (meta_sec(mx) >> s) & 1u;  // in its secondary x: y is its home
  write_entry(bk, y, fs, k, w, tag, x);
  uint32_t moved_x = meta_moved(mx), moved_y = meta_moved(my);
  if (!plain) {
    if (guest) {
      if (moved_y > 0u) {
        moved_y -= 1u;
        if (moved_y == 0u) *bloom_ptr(bk, y) = 0ull;
      }
    } else {
      *bloom_ptr(bk, x) |= key_fields(key_hash(k, seed), log2b).bloom_bits;
      moved_x += 1u;
    }
  }
  const uint32_t fb = 1u << fs, sb = 1u << s;
  *meta_ptr(bk, y) = make_meta(moved_y, meta_busy(my) | fb,
                               guest ? (meta_sec(my) & ~fb) : (meta_sec(my) | fb));
  *meta_ptr(bk, x) = make_meta(moved_x, meta_busy(mx) & ~sb, meta_sec(mx) & ~sb);
}

// Entries of a full bucket that may move (an entry leaving its primary
// must not overflow that primary's moved counter).
__device__ __forceinline__ uint32_t movable(uint32_t meta, bool plain) {
  uint32_t c = meta_busy(meta);
  if (!plain && meta_moved(meta) >= 0xffffu) c &= meta_sec(meta);
  return c;
}

// The other buckets of bucket b's entries and, for the entries in `cand`,
// which of those buckets have a free slot (their metadata words loaded
// together, without locks).  Every slot's load is issued, a non-candidate
// reading bucket b itself, so that no load waits inside a branch: two round
// trips in all.
__device__ __forceinline__ uint32_t room_of(const uint8_t *bk, uint32_t b, uint32_t cand,
                                            uint32_t (&other)[kSlots]) {
#pragma unroll
  for (uint32_t w = 0; w < 4; ++w) {
    const uint64_t o = load_relaxed(bucket_ptr(bk, b) + kOtherOffset + 8 * w);
    other[2 * w] = (uint32_t)o;
    other[2 * w + 1] = (uint32_t)(o >> 32);
  }
  uint32_t om[kSlots];
#pragma unroll
  for (uint32_t s = 0; s < kSlots; ++s)
    om[s] = (uint32_t)load_relaxed(bucket_ptr(bk, ((cand >> s) & 1u) ? other[s] : b) +
                                   kMetaOffset);
  uint32_t room = 0;
#pragma unroll
  for (uint32_t s = 0; s < kSlots; ++s)
    if (((cand >> s) & 1u) && meta_busy(om[s]) != 0xffu) room |= 1u << s;
  return room;
}

// a[i] for a small array indexed by a value known only at run time, as an
// OR of masked elements: an array indexed that way (or by a chain of
// selects, which the compiler turns back into an index) would live in
// scratch memory, and each load into it would wait for the one before.
__device__ __forceinline__ uint32_t pick_slot(const uint32_t (&a)[kSlots], uint32_t i) {
  uint32_t r = 0;
#pragma unroll
  for (uint32_t s = 0; s < kSlots; ++s) r |= a[s] & (0u - (uint32_t)(s == i));
  return r;
}

// Takes the lock of bucket b unless the caller holds it already.
__device__ __forceinline__ bool lock_extra(uint8_t *bk, uint32_t b, const KeyFields &f) {
  return b == f.p || b == f.a || try_lock(bk, b);
}
__device__ __forceinline__ void unlock_extra(uint8_t *bk, uint32_t b, const KeyFields &f) {
  if (b != f.p && b != f.a) unlock(bk, b);
}

// Cuckoo displacements done inside DIRECT, under the locks of the key's two
// buckets, when the primary p is full: the walk's lookahead from p, one
// level and, if no entry of p can move at once, two.  One step: an entry v
// of p whose other bucket y has a free slot (preferably one going home)
// moves there.  Two steps: an entry of some y1 = other(v) moves on to its
// own other bucket y2, which has a free slot, and v takes its place.  The
// buckets beyond p and a are locked here (never waited on), the path is
// re-checked under the locks, the moves are applied last to first with the
// filter maintenance of Sec. 4.1, and the key takes v's slot in p.  Almost
// every key that needs a cuckoo path needs at most two displacements, which
// then cost one critical section instead of a walk, one locked move per
// displacement and a second DIRECT step.  mp: p's meta word read under the
// lock.  Returns true when the key was placed; false, with nothing changed,
// when no such path exists (the caller falls back to the walk); kBusy,
// with nothing changed, when a bucket beyond the pair is locked by another
// lane or its state changed before the lock (the caller may retry DIRECT:
// another lane's move is brief, and a retry costs a few round trips where
// the walk costs tens).
__device__ __attribute__((noinline)) int displace_and_place(uint8_t *bk, uint32_t log2b, uint64_t seed, bool plain,
                                   const KeyFields &f, uint64_t h, uint4 key, uint64_t word,
                                   uint32_t mp) {
  const uint32_t cand = movable(mp, plain), sec = meta_sec(mp), p = f.p;
  uint32_t other[kSlots];
  const uint32_t room = room_of(bk, p, cand, other);
  uint32_t v = kSlots, y1 = kNoBucket, t = kSlots, y2 = kNoBucket;
  if (room) {
    const uint32_t pick = (room & sec) ? (room & sec) : room;
    v = nth_bit(pick, (uint32_t)(mix64(h ^ kDisplaceSalt) %
                                 (uint64_t)__builtin_popcount(pick)));
    y1 = pick_slot(other, v);
  } else {
    // second level, one candidate at a time in the order of the choice
    // (entries of p going home first), two round trips each: the metadata
    // word and other[] of the candidate's other bucket y1, then the
    // metadata words of y1's entries' other buckets, all of a round trip's
    // loads issued together (a non-movable slot reads y1 itself, so that
    // none waits inside a branch).  The first candidate whose y1 has an
    // entry that can move on to a bucket with a free slot wins (an entry of
    // y1 going home preferred); at the loads of the table's working loads
    // that is nearly always the first one tried.  Searching every candidate
    // at once takes 104 loads; measured on MI355X, one wavefront's lane
    // spends some 20 us issuing them and choosing, against about 1 us for a
    // candidate's two round trips.
    for (uint32_t order = 0; order < 2 && t == kSlots; ++order) {
      for (uint32_t c = cand & (order ? ~sec : sec); c && t == kSlots; c &= c - 1u) {
        const uint32_t s = (uint32_t)__builtin_ctz(c);
        const uint32_t b1 = pick_slot(other, s);
        const uint8_t *base1 = bucket_ptr(bk, b1);
        const uint32_t m1 = (uint32_t)load_relaxed(base1 + kMetaOffset);
        uint32_t o1[kSlots];
#pragma unroll
        for (uint32_t w = 0; w < 4; ++w) {
          const uint64_t o = load_relaxed(base1 + kOtherOffset + 8 * w);
          o1[2 * w] = (uint32_t)o;
          o1[2 * w + 1] = (uint32_t)(o >> 32);
        }
        const uint32_t mv = movable(m1, plain);
        uint32_t om[kSlots];
#pragma unroll
        for (uint32_t u = 0; u < kSlots; ++u)
          om[u] = (uint32_t)load_relaxed(bucket_ptr(bk, ((mv >> u) & 1u) ? o1[u] : b1) +
                                         kMetaOffset);
        uint32_t r = 0u;
#pragma unroll
        for (uint32_t u = 0; u < kSlots; ++u)
          if (((mv >> u) & 1u) && meta_busy(om[u]) != 0xffu) r |= 1u << u;
        if (r) {
          const uint32_t sc = meta_sec(m1);
          const uint32_t pick = (r & sc) ? (r & sc) : r;
          v = s;
          t = (uint32_t)__builtin_ctz(pick);
          y1 = b1;
          y2 = pick_slot(o1, t);
        }
      }
    }
    if (t == kSlots) return 0;
  }
  // lock the buckets beyond p and a (both compare-and-swaps issued
  // together: a failure here is not retried but falls back to the walk, so
  // it cannot repeat in lockstep), then re-check the path under the locks
  const bool ok1 = lock_extra(bk, y1, f);
  const bool ok2 = y2 == kNoBucket || lock_extra(bk, y2, f);
  if (!(ok1 && ok2)) {
    if (ok1) unlock_extra(bk, y1, f);
    if (ok2 && y2 != kNoBucket) unlock_extra(bk, y2, f);
    return kBusy;
  }
  section_begin();
  bool done = false;
  const uint32_t my1 = *meta_ptr(bk, y1);
  if (y2 == kNoBucket) {
    if (meta_busy(my1) != 0xffu) {
      move_locked(bk, f.p, v, y1, (uint32_t)__builtin_ctz(~meta_busy(my1) & 0xffu), log2b, seed,
                  plain);
      done = true;
    }
  } else {
    const uint32_t my2 = *meta_ptr(bk, y2);
    const bool still = ((meta_busy(my1) >> t) & 1u) && other_ptr(bk, y1)[t] == y2 &&
                       ((movable(my1, plain) >> t) & 1u) && meta_busy(my2) != 0xffu;
    if (still) {
      move_locked(bk, y1, t, y2, (uint32_t)__builtin_ctz(~meta_busy(my2) & 0xffu), log2b, seed,
                  plain);
      move_locked(bk, f.p, v, y1, t, log2b, seed, plain);
      done = true;
    }
  }
  if (done) {
    // the key takes slot v of p, its primary
    write_entry(bk, f.p, v, key, word, f.tag, f.a);
    const uint32_t m = *meta_ptr(bk, f.p), vb = 1u << v;
    *meta_ptr(bk, f.p) = make_meta(meta_moved(m), meta_busy(m) | vb, meta_sec(m) & ~vb);
  }
  section_end();
  if (y2 != kNoBucket) unlock_extra(bk, y2, f);
  unlock_extra(bk, y1, f);
  return done ? 1 : kBusy;
}

// DIRECT step of a table with timers; word = value | expiry << 48.
__device__ int insert_direct_timed(uint8_t *bk, uint4 key, uint64_t word, const KeyFields &f,
                                   uint64_t h, uint32_t log2b, uint64_t seed, bool plain,
                                   uint32_t now, bool retry_displace) {
  if (!lock_two(bk, f.p, f.a)) return kBusy;
  const Head hp = read_head(bk, f.p);
  const Head ha = read_head(bk, f.a);
  int r = kNeedPath;
  int s = find_slot(bk, f.p, hp, key, f.tag);
  uint32_t b = f.p;
  if (s < 0 && (plain || bloom_pass(hp.q1, f.bloom_bits))) {
    s = find_slot(bk, f.a, ha, key, f.tag);
    b = f.a;
  }
  if (s >= 0) {
    // the key's entry, alive (an update) or expired (overwritten in place)
    const Coh<uint64_t> vw = *value_ptr(bk, b, (uint32_t)s);
    r = word_alive(vw, now) ? CKPP_UPDATED : CKPP_INSERTED;
    vw = word;
  } else {
    Pair P{{f.p, f.a}, {hp.q1.z, ha.q1.z}};
    for (int xi = 0; xi < 2 && r == kNeedPath; ++xi) {
      if (xi == 1 && !plain && meta_moved(P.meta[0]) >= 0xffffu) break;
      const uint32_t x = P.b[xi];
      const uint32_t busy = meta_busy(P.meta[xi]);
      uint32_t fs;
      if (busy != 0xffu) {
        fs = (uint32_t)__builtin_ctz(~busy & 0xffu);
      } else {
        const uint32_t exp = expired_mask(bk, x, busy, now);
        if (!exp) continue;
        // prefer an entry whose removal needs no lock beyond the pair's
        uint32_t cheap = exp & ~meta_sec(P.meta[xi]);
        for (uint32_t e = exp & meta_sec(P.meta[xi]); e; e &= e - 1u) {
          const uint32_t v = (uint32_t)__builtin_ctz(e);
          const uint32_t y = other_ptr(bk, x)[v];
          if (y == f.p || y == f.a) cheap |= 1u << v;
        }
        fs = (uint32_t)__builtin_ctz(cheap ? cheap : exp);
        if (!remove_expired(bk, P, xi, fs, plain)) {
          r = kBusy;
          break;
        }
      }
      write_entry(bk, x, fs, key, word, f.tag, xi ? f.p : f.a);
      const uint32_t m = P.meta[xi], bit = 1u << fs;
      P.meta[xi] = make_meta(meta_moved(m), meta_busy(m) | bit,
                             xi ? (meta_sec(m) | bit) : (meta_sec(m) & ~bit));
      if (xi == 1 && !plain) {
        *bloom_ptr(bk, f.p) |= f.bloom_bits;
        P.meta[0] = make_meta(meta_moved(P.meta[0]) + 1u, meta_busy(P.meta[0]),
                              meta_sec(P.meta[0]));
      }
      r = CKPP_INSERTED;
    }
    if (r == CKPP_INSERTED) {
      *meta_ptr(bk, f.p) = P.meta[0];
      *meta_ptr(bk, f.a) = P.meta[1];
    } else if (r == kNeedPath) {
      const int d = displace_and_place(bk, log2b, seed, plain, f, h, key, word, hp.q1.z);
      if (d == 1) r = CKPP_INSERTED;
      else if (d == kBusy && retry_displace) r = kDisplaceBusy;
    }
  }
  unlock_two(bk, f.p, f.a);
  return r;
}

// DIRECT step of a table without timers.  retry_displace: a displacement
// path found but blocked by another lane's lock returns kDisplaceBusy (the
// caller retries DIRECT) rather than kNeedPath.
__device__ int insert_direct(uint8_t *bk, uint4 key, uint64_t value, const KeyFields &f,
                             uint64_t h, uint32_t log2b, uint64_t seed, bool plain,
                             bool retry_displace) {
  if (!lock_two(bk, f.p, f.a)) return kBusy;
  const Head hp = read_head(bk, f.p);
  const Head ha = read_head(bk, f.a);
  int r;
  int s = find_slot(bk, f.p, hp, key, f.tag);
  uint32_t b = f.p;
  if (s < 0 && (plain || bloom_pass(hp.q1, f.bloom_bits))) {
    s = find_slot(bk, f.a, ha, key, f.tag);
    b = f.a;
  }
  if (s >= 0) {
    *value_ptr(bk, b, (uint32_t)s) = value;
    r = CKPP_UPDATED;
  } else {
    const uint32_t mp = hp.q1.z, ma = ha.q1.z;
    const uint32_t busy_p = meta_busy(mp), busy_a = meta_busy(ma);
    if (busy_p != 0xffu) {
      const uint32_t fs = (uint32_t)__builtin_ctz(~busy_p & 0xffu);
      write_entry(bk, f.p, fs, key, value, f.tag, f.a);
      *meta_ptr(bk, f.p) = make_meta(meta_moved(mp), busy_p | (1u << fs), meta_sec(mp) & ~(1u << fs));
      r = CKPP_INSERTED;
    } else if (busy_a != 0xffu && (plain || meta_moved(mp) < 0xffffu)) {
      const uint32_t fs = (uint32_t)__builtin_ctz(~busy_a & 0xffu);
      write_entry(bk, f.a, fs, key, value, f.tag, f.p);
      *meta_ptr(bk, f.a) = make_meta(meta_moved(ma), busy_a | (1u << fs), meta_sec(ma) | (1u << fs));
      if (!plain) {
        *bloom_ptr(bk, f.p) |= f.bloom_bits;
        *meta_ptr(bk, f.p) = make_meta(meta_moved(mp) + 1u, busy_p, meta_sec(mp));
      }
      r = CKPP_INSERTED;
    } else {
      const int d = displace_and_place(bk, log2b, seed, plain, f, h, key, value, mp);
      r = d == 1 ? CKPP_INSERTED : (d == kBusy && retry_displace) ? kDisplaceBusy : kNeedPath;
    }
  }
  unlock_two(bk, f.p, f.a);
  return r;
}


// Random walk with one step of lookahead from bucket `start` (read without
// locks).  At each full bucket the other buckets of all its candidate
// entries are looked at together (their metadata words, loaded in
// parallel): if one of them has a free slot, moving that entry there ends
// the path (an entry sitting in its secondary bucket, i.e. going home,
// preferred); otherwise a victim is drawn as in a plain random walk (an
// entry going home, then one whose other bucket is not the bucket just
// left, then any) and the walk continues at its other bucket.  The same
// two memory round trips per step as a plain walk, but far fewer steps: at
// load 0.9 the longest paths shrink from tens of displacements to a few.
// path[i] holds bucket | slot << 29 of the i-th victim; *last receives the
// bucket with a free slot that ends the path.  Returns the path length, or
// -1.
__device__ __attribute__((noinline)) int walk(const uint8_t *bk, uint32_t start, uint64_t rbase, uint32_t max_kicks,
                    bool plain, uint32_t *path, uint32_t *last) {
  uint32_t cur = start, prev = kNoBucket;
  for (uint32_t step = 0; step < max_kicks; ++step) {
    const uint8_t *base = bucket_ptr(bk, cur);
    const uint32_t meta = (uint32_t)load_relaxed(base + kMetaOffset);
    uint32_t other[kSlots];
#pragma unroll
    for (uint32_t w = 0; w < 4; ++w) {
      const uint64_t o = load_relaxed(base + kOtherOffset + 8 * w);
      other[2 * w] = (uint32_t)o;
      other[2 * w + 1] = (uint32_t)(o >> 32);
    }
    uint32_t used = 0;
    for (uint32_t i = 0; i < step; ++i) {
      const uint32_t e = path[i];
      if ((e & kPathBucketMask) == cur) used |= 1u << (e >> kPathSlotShift);
    }
    const uint32_t sec = meta_sec(meta);
    uint32_t cand = meta_busy(meta) & ~used;
    if (!plain && meta_moved(meta) >= 0xffffu) cand &= sec;  // no owner may leave
    if (!cand) return -1;
    // lookahead: which candidates' other buckets have a free slot (every
    // slot's load issued, a non-candidate reading the current bucket, so
    // that all are in flight together)
    uint32_t om[kSlots];
#pragma unroll
    for (uint32_t s = 0; s < kSlots; ++s)
      om[s] = (uint32_t)load_relaxed(bucket_ptr(bk, ((cand >> s) & 1u) ? other[s] : cur) +
                                     kMetaOffset);
    uint32_t room = 0;
#pragma unroll
    for (uint32_t s = 0; s < kSlots; ++s)
      if (((cand >> s) & 1u) && meta_busy(om[s]) != 0xffu) room |= 1u << s;
    const uint64_t r = mix64(rbase + (uint64_t)(step + 1) * kGolden);
    if (room) {
      const uint32_t pick = (room & sec) ? (room & sec) : room;
      const uint32_t v = nth_bit(pick, (uint32_t)(r % (uint64_t)__builtin_popcount(pick)));
      path[step] = cur | (v << kPathSlotShift);
      *last = pick_slot(other, v);
      return (int)step + 1;
    }
    uint32_t pref = 0;
#pragma unroll
    for (uint32_t s = 0; s < kSlots; ++s)
      if (((cand >> s) & 1u) && other[s] != prev) pref |= 1u << s;
    const uint32_t home = pref & sec;
    const uint32_t pick = home ? home : (pref ? pref : cand);
    const uint32_t v = nth_bit(pick, (uint32_t)(r % (uint64_t)__builtin_popcount(pick)));
    path[step] = cur | (v << kPathSlotShift);
    prev = cur;
    cur = pick_slot(other, v);
  }
  return -1;
}

// Under the locks of x and y: moves the entry of slot s of bucket x to a
// free slot of bucket y, its other bucket, if the state still matches the
// path (the slot is taken, its entry's other bucket is y, y has a free
// slot, and an entry leaving its primary does not overflow the moved
// counter), with the filter maintenance of Sec. 4.1.  Returns 1 when
// moved, 0 when the state no longer matches (nothing changed).
__device__ int move_checked(uint8_t *bk, uint32_t x, uint32_t s, uint32_t y, uint32_t log2b,
                            uint64_t seed, bool plain) {
  int r = 0;
  const uint32_t mx = *meta_ptr(bk, x), my = *meta_ptr(bk, y);
  const uint32_t busy_x = meta_busy(mx), busy_y = meta_busy(my);
  if (((busy_x >> s) & 1u) && other_ptr(bk, x)[s] == y && busy_y != 0xffu) {
    const uint4 key = *key_ptr(bk, x, s);
    const uint64_t val = *value_ptr(bk, x, s);
    const KeyFields fe = key_fields(key_hash(key, seed), log2b);
    const bool from_primary = fe.p == x;
    const bool consistent = from_primary ? (fe.a == y) : (fe.a == x && fe.p == y);
    if (consistent && (plain || !from_primary || meta_moved(mx) < 0xffffu)) {
      const uint32_t fs = (uint32_t)__builtin_ctz(~busy_y & 0xffu);
      write_entry(bk, y, fs, key, val, tag_ptr(bk, x)[s], x);
      uint32_t moved_x = meta_moved(mx), moved_y = meta_moved(my);
      const uint32_t sec_y =
          from_primary ? (meta_sec(my) | (1u << fs)) : (meta_sec(my) & ~(1u << fs));
      if (!plain) {
        if (from_primary) {
          *bloom_ptr(bk, x) |= fe.bloom_bits;
          moved_x += 1u;
        } else if (moved_y > 0u) {
          moved_y -= 1u;
          if (moved_y == 0u) *bloom_ptr(bk, y) = 0ull;
        }
      }
      *meta_ptr(bk, y) = make_meta(moved_y, busy_y | (1u << fs), sec_y);
      *meta_ptr(bk, x) = make_meta(moved_x, busy_x & ~(1u << s), meta_sec(mx) & ~(1u << s));
      r = 1;
    }
  }
  return r;
}

// One displacement of the MOVE state: move_checked under the lock pair of
// x and y.  Returns 1 when done, 0 when the state no longer matches the
// path, kBusy when a lock was taken.
__device__ __attribute__((noinline)) int move_entry(uint8_t *bk, uint32_t x, uint32_t s, uint32_t y,
                          uint32_t log2b, uint64_t seed, bool plain) {
  if (x == y || !lock_two(bk, x, y)) return kBusy;
  const int r = move_checked(bk, x, s, y, log2b, seed, plain);
  unlock_two(bk, x, y);
  return r;
}

// Longest cuckoo path applied in one critical section (apply_path).
constexpr uint32_t kSectionPath = 8;

// Applies a cuckoo path of len <= kSectionPath displacements (path[0..len)
// as the walk wrote it, `last` the bucket that ends it) in one critical
// section, where the MOVE state takes a lock pair, a re-check and a release
// per displacement: every bucket of the path is locked, all the lock
// requests issued together and none waited for; then the moves run last to
// first, each with move_checked's re-check.  A lock held by another lane
// gives back every lock taken and returns kBusy with nothing moved (the
// caller then moves step by step, taking the pairs in ascending order,
// which keeps concurrent keys live).  A re-check that fails stops the moves
// and returns 0 (the moves already made stand: each is a valid move on its
// own, as in the MOVE state); 1 when every displacement is made.
//
// The lock requests are atomic ORs of 1 into the lock words (a lock is
// taken by the request that reads 0), one per entry of b[0..kSectionPath]
// whatever the path's length, so that none sits behind a branch: entries
// past the path, and repeats of a bucket, request b[0]'s or that bucket's
// lock again.  A lane's requests to one word are performed in order, so a
// repeat reads 1 when an earlier request of the lane took the lock; it can
// read 0 only when the earlier one found the lock held by another lane that
// has let it go since, and then this lane holds it through the repeat and
// gives it back with the others.
__device__ __attribute__((noinline)) int apply_path(uint8_t *bk, const uint32_t *path,
                                                    uint32_t len, uint32_t last, uint32_t log2b,
                                                    uint64_t seed, bool plain) {
  uint32_t b[kSectionPath + 1], sl[kSectionPath];
#pragma unroll
  for (uint32_t i = 0; i < kSectionPath; ++i) {
    const uint32_t e = i < len ? path[i] : 0u;
    b[i] = i < len ? (e & kPathBucketMask) : kNoBucket;
    sl[i] = e >> kPathSlotShift;
  }
  // `last` follows the path's buckets; entries past it request b[0] again
  b[kSectionPath] = kNoBucket;
#pragma unroll
  for (uint32_t i = 0; i <= kSectionPath; ++i) {
    if (i == len) b[i] = last;
  }
  uint32_t addr[kSectionPath + 1];
  bool first[kSectionPath + 1];  // the first entry of its bucket within the path
#pragma unroll
  for (uint32_t i = 0; i <= kSectionPath; ++i) {
    bool dup = b[i] == kNoBucket;
#pragma unroll
    for (uint32_t j = 0; j < i; ++j) dup = dup || b[j] == b[i];
    first[i] = !dup;
    addr[i] = b[i] == kNoBucket ? b[0] : b[i];
  }
  bool took[kSectionPath + 1];
#pragma unroll
  for (uint32_t i = 0; i <= kSectionPath; ++i)
    took[i] = __hip_atomic_fetch_or(lock_word(bk, addr[i]), 1u, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT) == 0u;
  bool all = true;
#pragma unroll
  for (uint32_t i = 0; i <= kSectionPath; ++i) all = all && (took[i] || !first[i]);
  if (!all) {
#pragma unroll
    for (uint32_t i = 0; i <= kSectionPath; ++i)
      if (took[i]) unlock(bk, addr[i]);
    return kBusy;
  }
  section_begin();
  int r = 1;
  for (uint32_t k = len; k > 0 && r == 1; --k) {
    const uint32_t i = k - 1u;
    uint32_t x = 0u, s = 0u, y = 0u;
#pragma unroll
    for (uint32_t j = 0; j < kSectionPath; ++j) {
      if (j == i) {
        x = b[j];
        s = sl[j];
        y = b[j + 1];
      }
    }
    r = x == y ? 0 : move_checked(bk, x, s, y, log2b, seed, plain);
  }
  section_end();
  // every bucket's lock was taken by its first request (the repeats read 1)
#pragma unroll
  for (uint32_t i = 0; i <= kSectionPath; ++i)
    if (took[i]) unlock(bk, addr[i]);
  return r;
}

// Outcome of one key's insert: its status, and whether the retry bound ran
// out (then the status is CKPP_RETRY).
struct InsertOutcome {
  int status;
  bool spun;
};

// Runs one key through the DIRECT / WALK / MOVE state machine until it is
// placed, updated or fails, for at most spin_limit iterations (then
// CKPP_RETRY: the key's value is neither stored nor changed; the moves
// applied so far only relocated other entries).  path: this lane's scratch,
// max(1, max_kicks) words.  TIMED: the table has timers; the entry gets
// expiration time `expiry`, and a value of 2^48 or more (the device layout's
// limit) fails at once with nothing changed.
template <bool TIMED = false>
__device__ InsertOutcome insert_one(uint8_t *bk, uint4 key, uint64_t value, uint32_t log2b,
                                    uint64_t seed, uint32_t max_kicks, bool plain,
                                    uint32_t *path, uint32_t spin_limit, uint32_t expiry = 0u,
                                    uint32_t now = 0u) {
  if (TIMED && (value >> kTimerShift) != 0ull) return InsertOutcome{CKPP_FAILED, false};
  const uint64_t word = TIMED ? (value | ((uint64_t)(expiry & 0xffffu) << kTimerShift)) : value;
  const uint64_t h = key_hash(key, seed);
  const KeyFields f = key_fields(h, log2b);
  enum { DIRECT, WALK, MOVE };
  int state = DIRECT, result = -1;
  uint32_t len = 0, next = 0, last = 0, walks = 0, iters = 0, dretries = 0;
  bool spun = false;
  while (result < 0) {
    if (++iters > spin_limit) {
      result = CKPP_RETRY;
      spun = true;
      break;
    }
    if (state == DIRECT) {
      const bool retry_displace = dretries < kDisplaceRetries;
      const int r = TIMED ? insert_direct_timed(bk, key, word, f, h, log2b, seed, plain, now,
                                                retry_displace)
                          : insert_direct(bk, key, value, f, h, log2b, seed, plain, retry_displace);
      if (r >= 0)
        result = r;
      else if (r == kNeedPath)
        state = WALK;
      else if (r == kDisplaceBusy)
        ++dretries;  // DIRECT again
    } else if (state == WALK) {
      if (walks >= kMaxWalks) {
        result = CKPP_FAILED;
        break;
      }
      const int L = walk(bk, f.p, h ^ ((uint64_t)walks * kWalkSalt), max_kicks, plain,
                         path, &last);
      ++walks;
      if (L <= 0) {
        result = CKPP_FAILED;
      } else {
        len = (uint32_t)L;
        next = len;
        state = MOVE;
        // a short path in one critical section; step by step if a lock is
        // held (then nothing was moved)
        if (len <= kSectionPath &&
            apply_path(bk, path, len, last, log2b, seed, plain) != kBusy)
          state = DIRECT;
      }
    } else {
      const uint32_t e = path[next - 1];
      const uint32_t x = e & kPathBucketMask, s = e >> kPathSlotShift;
      const uint32_t y = (next == len) ? last : (path[next] & kPathBucketMask);
      const int r = move_entry(bk, x, s, y, log2b, seed, plain);
      if (r == 1) {
        if (--next == 0) state = DIRECT;
      } else if (r == 0) {
        state = DIRECT;
      }
    }
  }
  return InsertOutcome{result, spun};
}

// Returns 1 if the key was removed, 0 if absent, kBusy to retry.  TIMED:
// an expired entry of the key is removed too, but reports 0 (Sec. 4.2).
template <bool TIMED>
__device__ int delete_direct(uint8_t *bk, uint4 key, const KeyFields &f, bool plain,
                             uint32_t now) {
  if (!lock_two(bk, f.p, f.a)) return kBusy;
  const Head hp = read_head(bk, f.p);
  int r = 0;
  int s = find_slot(bk, f.p, hp, key, f.tag);
  const uint32_t mp = hp.q1.z;
  if (s >= 0) {
    const uint32_t bit = 1u << s;
    r = (!TIMED || word_alive(*value_ptr(bk, f.p, (uint32_t)s), now)) ? 1 : 0;
    *meta_ptr(bk, f.p) = make_meta(meta_moved(mp), meta_busy(mp) & ~bit, meta_sec(mp) & ~bit);
  } else if (plain || bloom_pass(hp.q1, f.bloom_bits)) {
    const Head ha = read_head(bk, f.a);
    s = find_slot(bk, f.a, ha, key, f.tag);
    if (s >= 0) {
      const uint32_t bit = 1u << s, ma = ha.q1.z;
      r = (!TIMED || word_alive(*value_ptr(bk, f.a, (uint32_t)s), now)) ? 1 : 0;
      *meta_ptr(bk, f.a) = make_meta(meta_moved(ma), meta_busy(ma) & ~bit, meta_sec(ma) & ~bit);
      if (!plain && meta_moved(mp) > 0u) {
        const uint32_t moved = meta_moved(mp) - 1u;
        if (moved == 0u) *bloom_ptr(bk, f.p) = 0ull;
        *meta_ptr(bk, f.p) = make_meta(moved, meta_busy(mp), meta_sec(mp));
      }
    }
  }
  unlock_two(bk, f.p, f.a);
  return r;
}


// Deletes one key: 1 if it was removed, 0 if absent, CKPP_RETRY (nothing
// removed; the key may still be present) when its bucket locks stayed taken
// by other lanes for spin_limit attempts; *spun is set in that case.
template <bool TIMED = false>
__device__ int delete_one(uint8_t *bk, uint4 key, uint32_t log2b, uint64_t seed, bool plain,
                          uint32_t spin_limit, bool *spun, uint32_t now = 0u) {
  const KeyFields f = key_fields(key_hash(key, seed), log2b);
  int r = kBusy;
  uint32_t iters = 0;
  while (r == kBusy && iters < spin_limit) {
    ++iters;
    r = delete_direct<TIMED>(bk, key, f, plain, now);
  }
  *spun = r == kBusy;
  return r == kBusy ? CKPP_RETRY : r;
}

// Anti-revival scan (Sec. 4.2) over buckets [0, nb) by the lanes gtid of a
// grid of gthreads (blocks of 256): 16 neighbouring lanes read one bucket's
// 256 bytes, one 16-byte quarter each, and share the metadata word (lane
// 1), the value words (lanes 6, 7, 12, 13: the time in the high 16 bits)
// and the other buckets (lanes 14, 15) through cross-lane reads.  Lane 0 of
// the group clears the bucket's expired slots (busy and sec bits) with an
// atomic AND; the moved counter of the primary bucket of a removed entry
// that sat in its secondary drops by one through an atomic subtraction on
// that bucket's meta word (the counter is its low 16 bits and is at least 1
// while the entry is counted there), done by the lane that holds the
// entry's other bucket, so no lock is needed.  The subtraction that takes a
// counter from 1 to 0 empties that bucket's filter (Sec. 4.1: the filter is
// reset when its counter returns to zero): while the scan runs nothing
// raises a counter, so zero is final.  The caller runs nothing else on the
// table meanwhile.  U: the buckets a group reads before it examines the
// first (loads in flight per lane, for grids with few waves).  Returns the
// entries this lane removed.
template <uint32_t U = 1>
__device__ __forceinline__ uint64_t expire_slots_pass(uint8_t *bk, uint64_t nb, uint32_t now,
                                                      bool plain, uint64_t gtid,
                                                      uint64_t gthreads) {
  const uint32_t lane = threadIdx.x & 63u, r = lane & 15u, g0 = lane & 48u;
  const uint64_t groups = gthreads / 16u;
  uint64_t count = 0;
  for (uint64_t b0 = gtid / 16u; b0 < nb; b0 += U * groups) {
    // every load is issued before the first is used: indexes past the end
    // read the last bucket instead (no branch around a load, which would
    // wait for it inside the branch), and those buckets are skipped below
    uint4 qs[U];
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) {
      const uint64_t b = b0 + u * groups;
      qs[u] = reinterpret_cast<const uint4 *>(bucket_ptr(bk, (uint32_t)(b < nb ? b : nb - 1u)))[r];
    }
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) {
      const uint64_t b = b0 + u * groups;
      if (b >= nb) break;
      const uint4 q = qs[u];
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
          // y < nb: always, on a table that keeps its invariants
          if (((exp & meta_sec(meta)) >> (base + k)) & 1u && y < nb) {
            const uint32_t old = __hip_atomic_fetch_sub(meta_ptr(bk, y).p, 1u, __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
            if (meta_moved(old) == 1u) *bloom_ptr(bk, y) = 0ull;
          }
        }
      }
    }
  }
  return count;
}

}  // namespace
}  // namespace ckpp
