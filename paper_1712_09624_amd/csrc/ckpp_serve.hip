// ckpp_serve.hip -- the serving loop: one persistent kernel that takes
// bursts of lookups, inserts and deletes from device rings as the host
// submits them, in rounds (continuous batching).
//
// Host and loop talk through a small block of pinned, coherent host memory:
// the host writes each burst's cumulative ring tails and then the number of
// submitted bursts; the loop's leader (block 0, thread 0) polls that number
// and publishes the number of completed bursts there.  A round:
//
//   boundary  every block arrives at a grid barrier; once all have arrived
//             the leader publishes the previous round's completion, waits
//             for submitted bursts (or exits after idle_ms without any),
//             writes the round record (command, op range ends, time; every
//             word tagged with the boundary's epoch), which releases the
//             other blocks
//   lookups   every wave runs passes of 128 lookups (64 in the pessimistic
//             mode) over the round's lookup range (the lookup passes of the
//             batch kernels, unchanged); then the round's insert keys go into
//             a set
//   updates   after a barrier, the inserts (one lane per key, the batch
//             insert's state machine, unchanged, at most `path_lanes` lanes)
//             and the deletes (one lane per key, from the other end of the
//             grid) run side by side; a delete of a key the round also
//             inserts is deferred
//   deferred  only if some delete was deferred: after the next barrier
//             (every insert is done), the deferred deletes.  A round with
//             more updates than lanes, or more inserts than the set holds,
//             runs inserts, a barrier, deletes
//   end       every result (lookup answers, insert statuses, delete
//             results) was written through to memory with a system-scope
//             store, and each wave waits for its stores before its block
//             arrives at the next boundary, so the leader publishes a round
//             complete only once the host can read all of its results
//
// On a table with timers (Sec. 4.2) every burst carries the server's time
// at its submission, and a round takes only bursts of one time, so all of
// its operations run at that time: lookups find entries alive then (and may
// push their expiration times to now + ttl), inserts give their entries
// expiration time now + ttl, deletes remove alive and expired entries of
// their keys.  A round whose first burst asks for it (ckpp_server_set_time
// does, at least once every 16384 time units) starts with the anti-revival
// scan over the whole grid, and a barrier, before its lookups.
//
// The barriers use no atomics (each block stores its arrival in a flag line
// of its own; one wave polls them), and every polling load is relaxed, with
// one acquire fence after the wait: on this GPU an acquire load invalidates
// the cache, and a waiting wave must not keep invalidating the caches the
// working waves read through.  Every wait is bounded by the real-time
// counter and by an iteration count: a block that waits too long sets
// `abort`, every other wait sees it, and the whole grid leaves the loop, so
// the kernel always ends.  The grid is launched cooperatively, so all of
// its blocks are resident at once.

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstddef>
#include <emmintrin.h>
#include <new>
#include <stdint.h>
#include <string.h>
#include <thread>
#include <vector>

#include "ckpp_lookup_dev.h"
#include "ckpp_update_dev.h"

namespace ckpp {
namespace {

constexpr uint32_t kQueue = 4096;        // bursts in flight at most
// Threads per block of the loop: 8 wavefronts, two per SIMD (the kernel
// fits 256 registers per lane).  Against one wavefront per SIMD, measured on
// the serving workload: lookup phase at the peak 61 -> 53 us per round,
// peak 4.74 -> 5.04 G lookups/s, p50 at 25% / 50% offered load 88 -> 86 /
// 124 -> 112 us.
constexpr uint32_t kBlock = 512;
constexpr uint32_t kWaves = kBlock / 64;
constexpr uint64_t kTicksPerMs = 100000; // real-time counter: 100 MHz
constexpr uint64_t kPhaseMs = 20000;     // a phase may take this long at most
constexpr uint32_t kMaxPathLanes = 131072;  // every lane of a 256-block grid
// second bound on every spin loop, in iterations (each one sleeps and reads
// memory, so this is tens of seconds)
constexpr uint64_t kMaxSpins = 1ull << 26;

constexpr uint32_t kCmdRun = 1, kCmdExit = 2, kCmdDeferred = 3;
// The round's insert-key set holds at most this many entries (twice the
// inserts it takes); a round with more inserts runs inserts, then deletes.
constexpr uint64_t kMaxSetEntries = 1ull << 22;
// Result byte of a delete waiting for the round's inserts.
constexpr uint8_t kDeferred = 0xffu;
// A time change of the server is less than this; its anti-revival scan is
// due once the time is this far past the last one.
constexpr uint16_t kMaxTimeStep = 16384;
// Buckets each lane group of the loop's scan reads ahead (the loop has one
// block per compute unit, so each lane keeps several loads in flight).
constexpr uint32_t kScanUnroll = 16;

// Pinned host memory shared by the host and the loop.
// tails[k][3] of a burst: its time (bits 0..15), whether its round starts
// with the anti-revival scan (bit 16), and the number of time changes before
// it (bits 24..63; rounds never span two of them).
constexpr uint32_t kScanBit = 16, kTimeIndexShift = 24;
// latest[] of the last staged burst b, in one 16-byte block that the host
// writes with one store and the loop reads with one load: latest[0] holds
// the low 24 bits of b's lookup tail (bits 24..47) and of its insert tail
// (bits 0..23), latest[1] the low 24 bits of its delete tail (bits 24..47)
// and those of f (bits 0..23), a burst no later than the first one of b's
// time index (tables with timers; f = max(that burst, b - 8192), so that f
// is older than every burst in flight when the index is older still); bits
// 48..63 of both hold the tag kTagValid | (b mod 2^15).  The loop uses a
// block only when both tags agree, and only on servers whose budget is
// under 2^24 ops of a kind, so that a round's tails follow from these bits.
constexpr uint64_t kLow48 = (1ull << 48) - 1u, kLow24 = (1ull << 24) - 1u;
constexpr uint64_t kIndexFirstWindow = 2ull * kQueue;
constexpr uint64_t kFastTailsBudget = 1ull << 24;
constexpr uint32_t kTagValid = 0x8000u, kTagMask = 0x7fffu;
struct ServeHost {
  uint64_t submitted;  // host -> loop: bursts submitted
  uint64_t completed;  // loop -> host: bursts whose results are visible
  uint64_t rounds;     // loop -> host
  uint32_t stop;       // host -> loop: exit once idle
  uint32_t state;      // loop -> host: CKPP_SERVER_*
  alignas(16) uint64_t latest[2];  // host -> loop: the last staged burst's tagged tails
  // after burst k, at k % kQueue: lookup, insert, delete tails; time word
  uint64_t tails[kQueue][4];
};
static_assert(offsetof(ServeHost, latest) + sizeof(uint64_t[2]) <= 64,
              "the poll's words share one 64-byte line");
static_assert(kQueue <= kTagMask + 1u, "a tag names one burst of those in flight");

// Device memory of the loop (survives relaunches).
struct ServeDev {
  uint64_t done;              // bursts taken into rounds so far
  uint64_t lk0, lk1, in0, in1, de0, de1;  // the round's op ranges
  uint64_t rounds;            // rounds completed
  // leader's clock (real-time ticks): time from a phase's release until
  // every block has finished it, per phase; time spent at round boundaries
  // apart from waiting for work; time waiting for work
  uint64_t t_lookup, t_insert, t_delete, t_boundary, t_wait;
  uint64_t t_mark;            // when the leader last released a barrier
  uint32_t abort;             // a wait ran out of time
  uint32_t gen;               // barrier: last epoch the leader released
  uint32_t deferred;          // some delete of the round waits for its inserts
  uint32_t now;               // the round's time (tables with timers)
  uint32_t scan;              // the round starts with the anti-revival scan
  // the round record the leader writes at each boundary for the other
  // blocks: every word carries the boundary's epoch (mod 2^16) in bits
  // 48..63; rec[0]: the command (bits 32..47), the scan flag (bit 16) and
  // the time (bits 0..15); rec[1..3]: the low 48 bits of the round's lookup,
  // insert and delete range ends
  uint64_t rec[4];
};

// Barrier flags: block b stores the epoch it reached at arrive[b * kFlagStride]
// (one 128-byte line per block, so arrivals never contend).
constexpr uint32_t kFlagStride = 32;

struct ServeArgs {
  TableRef T;
  uint8_t *bk;
  uint32_t max_kicks;
  uint32_t plain;
  ServeHost *host;
  ServeDev *dev;
  uint32_t *arrive;  // barrier flags, gridDim.x lines
  uint64_t mask;     // capacity - 1
  const uint4 *lk_keys;
  uint8_t *lk_found;
  uint64_t *lk_vals;
  const uint4 *in_keys;
  const uint64_t *in_vals;
  uint8_t *in_status;
  const uint4 *de_keys;
  uint8_t *de_found;
  uint32_t *paths;
  uint32_t path_lanes;
  uint32_t spin_limit;  // the table's retry limit per insert/delete
  uint64_t idle_ticks;
  unsigned long long *nspin;
  uint4 *set_keys;    // the round's insert keys, open addressing
  uint32_t *set_tag;  // entry in use by the round whose tag it holds
  uint64_t set_mask;  // entries - 1
  uint32_t timed;     // the table has timers
  uint32_t fast_tails;  // a budget under 2^24: tails come with the poll
  uint32_t ttl;       // entry lifetime in time units (timers)
  uint32_t refresh;   // lookups that find an entry set its expiration time
  uint64_t nb;        // buckets
};

__device__ __forceinline__ uint64_t now_ticks() { return __builtin_amdgcn_s_memrealtime(); }

__device__ __forceinline__ uint64_t sys_load64(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void sys_store64(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void sys_store32(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}
// Polling loads: relaxed, so a spinning wave does not invalidate its caches
// on every iteration (an acquire load does, which would slow every other
// wave of the XCD while this one waits); the waiter issues one acquire
// fence once the awaited value has arrived.
__device__ __forceinline__ uint32_t poll32(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t poll_sys64(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint32_t poll_sys32(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// A barrier over the grid without atomics.  Every block reaches the same
// sequence of barriers and numbers them with the same epochs.  Thread 0 of
// each block stores the epoch in its own flag line; the leader wave (block
// 0, wave 0) polls all flags, 64 lanes at a time, until every block has
// arrived, then the leader stores the epoch in `gen` (release); the other
// blocks' thread 0 poll `gen`, and every waiter ends with an acquire fence.
// A wait that runs out of time or iterations sets `abort`, which every
// other wait gives up on.
//
// The arrival is a relaxed store after a wait for the block's own accesses
// (every wave waits before the block's __syncthreads): what a block writes
// in a phase for other blocks to read in the next is a table word written
// with a device-coherent access (under a bucket lock, by the anti-revival
// scan's atomics, or by a renewing lookup), or a set entry written with an
// atomic, all performed where the XCDs meet once waited for.  A release
// store would write back this XCD's whole L2 cache at every arrival of
// every block; measured on the serving workload, dropping those write-backs
// (with one system-scope release per block per round, for the host, at the
// time) took the update phase at 25% offered load from 49 to 35 us per
// round.  The results for the host now need no write-back either: they are
// written through (put_result, reg_pass_to's SYS stores).  The leader
// writes back nothing either: at a round boundary it publishes a tagged
// record with device-coherent stores (publish_round), and at a barrier
// inside a round nothing it wrote is read (release_epoch).
__device__ __forceinline__ void block_arrive(const ServeArgs &a, uint32_t epoch) {
  __builtin_amdgcn_s_waitcnt(0);
  __hip_atomic_store(a.arrive + (uint64_t)blockIdx.x * kFlagStride, epoch, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

// A result for the host: written through to memory (a system-scope
// store), visible once the writing wave has waited for its stores.
__device__ __forceinline__ void put_result(uint8_t *p, uint8_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ void set_abort(ServeDev *d) {
  __hip_atomic_store(&d->abort, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Non-leader blocks, thread 0: waits for the leader's release of `epoch`.
// Each poll reads `gen` and `abort` in one round trip.
__device__ bool wait_release(const ServeArgs &a, uint32_t epoch, uint64_t limit_ticks) {
  ServeDev *d = a.dev;
  const uint64_t t0 = now_ticks();
  for (uint64_t it = 0;; ++it) {
    const uint32_t g = poll32(&d->gen);
    const uint32_t ab = poll32(&d->abort);
    if ((int32_t)(g - epoch) >= 0) break;
    if (ab) return false;
    if (now_ticks() - t0 > limit_ticks || it > kMaxSpins) {
      set_abort(d);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return true;
}

// Leader wave (all 64 lanes of wave 0 of block 0): waits until every block
// has stored `epoch`.  Uniform result.  Each poll reads a lane's flags (four
// blocks a lane; indexes past the grid read the last block's flag again)
// and `abort` in one round trip: loads under a short-circuit `&&` would be
// issued one after another.
constexpr uint32_t kFlagsPerLane = 4;
__device__ bool gather(const ServeArgs &a, uint32_t epoch, uint64_t limit_ticks) {
  ServeDev *d = a.dev;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t last = gridDim.x - 1u;
  const uint64_t t0 = now_ticks();
  for (uint64_t it = 0;; ++it) {
    const uint32_t ab = poll32(&d->abort);
    bool mine = true;
    for (uint32_t b0 = 0; b0 < gridDim.x; b0 += 64u * kFlagsPerLane) {
      uint32_t f[kFlagsPerLane];
#pragma unroll
      for (uint32_t k = 0; k < kFlagsPerLane; ++k) {
        const uint32_t b = b0 + lane + 64u * k;
        f[k] = poll32(a.arrive + (uint64_t)(b < last ? b : last) * kFlagStride);
      }
#pragma unroll
      for (uint32_t k = 0; k < kFlagsPerLane; ++k) mine &= (int32_t)(f[k] - epoch) >= 0;
    }
    if (__builtin_amdgcn_ballot_w64(!mine) == 0ull) break;
    const bool stop = ab != 0u || now_ticks() - t0 > limit_ticks || it > kMaxSpins;
    if (__builtin_amdgcn_readfirstlane((int)stop)) {
      if (lane == 0u) set_abort(d);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return true;
}

// Leader at a round boundary: writes the round record for `epoch` with
// device-coherent stores (each word names its epoch, so a block takes it
// only whole; nothing else the blocks read was written since the last
// barrier, so no write-back of this XCD's L2 is needed), and `gen`, from
// which the next launch numbers its epochs.
__device__ __forceinline__ void publish_round(ServeDev *d, uint32_t epoch, uint32_t cmd,
                                              uint32_t scan, uint32_t now) {
  const uint64_t tag = (uint64_t)(epoch & 0xffffu) << 48;
  auto put = [](uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  put(&d->rec[1], tag | (d->lk1 & kLow48));
  put(&d->rec[2], tag | (d->in1 & kLow48));
  put(&d->rec[3], tag | (d->de1 & kLow48));
  put(&d->rec[0], tag | (uint64_t)cmd << 32 | (uint64_t)scan << 16 | (now & 0xffffu));
  __hip_atomic_store(&d->gen, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Non-leader blocks, thread 0, at a round boundary: waits until every word
// of the round record names `epoch` (r receives it).  Each poll reads the
// record and `abort` in one round trip.  False on abort or time-out.
__device__ bool wait_round(const ServeArgs &a, uint32_t epoch, uint64_t limit_ticks,
                           uint64_t (&r)[4]) {
  ServeDev *d = a.dev;
  const uint64_t tag = epoch & 0xffffu;
  const uint64_t t0 = now_ticks();
  for (uint64_t it = 0;; ++it) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
      r[k] = __hip_atomic_load(&d->rec[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t ab = poll32(&d->abort);
    if (ab) return false;
    if ((r[0] >> 48) == tag && (r[1] >> 48) == tag && (r[2] >> 48) == tag && (r[3] >> 48) == tag)
      return true;
    if (now_ticks() - t0 > limit_ticks || it > kMaxSpins) {
      set_abort(d);
      return false;
    }
    __builtin_amdgcn_s_sleep(2);
  }
}

// Leader, at a barrier inside a round: releases `epoch` to the waiting
// blocks.  What they read after it was written with device-coherent
// accesses (table words, set entries) or written through (results), all
// done before the blocks arrived, so the release is a relaxed store: a
// release store would write back this XCD's L2 cache.
__device__ __forceinline__ void release_epoch(ServeDev *d, uint32_t epoch) {
  __builtin_amdgcn_s_waitcnt(0);
  __hip_atomic_store(&d->gen, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The burst that the last staged burst's tagged tails (w) name, if both
// words carry the same tag and it is a burst from `done` on (fewer than
// kQueue are in flight); else ~0.
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint64_t latest_burst(u64x2 w, uint64_t done) {
  const uint32_t tag = (uint32_t)(w.x >> 48);
  if (!(tag & kTagValid) || (uint32_t)(w.y >> 48) != tag) return ~0ull;
  const uint64_t ahead = (tag - (uint32_t)done) & kTagMask;
  return ahead < kQueue ? done + ahead : ~0ull;
}

// Leader at a round boundary (every block has arrived): publish the round
// that just ended, wait for work, set the next round.  Returns the command.
__device__ uint32_t leader_next_round(const ServeArgs &a, bool ran_round) {
  ServeHost *h = a.host;
  ServeDev *d = a.dev;
  if (ran_round) {
    d->rounds += 1u;
    sys_store64(&h->rounds, d->rounds);
    sys_store64(&h->completed, d->done);
  }
  const uint64_t t0 = now_ticks();
  uint64_t s = 0;
  u64x2 w = {0ull, 0ull};
  bool have_tails = false;
  for (uint64_t it = 0;; ++it) {
    // one round trip to host memory: the submitted count, the stop flag and
    // the last staged burst's tagged tails (one line; the tails in one
    // 16-byte load of uncached host memory, volatile so that every poll
    // reads it)
    s = poll_sys64(&h->submitted);
    const uint32_t stop = poll_sys32(&h->stop);
    if (a.fast_tails) w = *reinterpret_cast<const volatile u64x2 *>(h->latest);
    if (a.fast_tails && s > d->done) {
      // submitted work is waiting: the round takes the bursts up to the
      // last staged one (the last submitted one or a later one whose
      // operations are in the rings too), whose tails came with the poll;
      // on a table with timers only while that burst's time index began
      // before this round (then every burst of the round has the last
      // round's time, and none starts a scan, which begins a new index)
      const uint64_t b = latest_burst(w, d->done);
      const uint64_t since = (d->done - w.y) & kLow24;  // done - f, mod 2^24
      const bool same_time = !a.timed || (since >= 1u && since < (1ull << 23));
      if (b != ~0ull && b + 1u >= s && same_time) {
        s = b + 1u;
        have_tails = true;
        break;
      }
    }
    if (s > d->done) break;
    if (stop) return kCmdExit;
    if (now_ticks() - t0 > a.idle_ticks || it > kMaxSpins) {
      // tell the host the loop is leaving, then look once more: a burst
      // submitted before the host saw EXITING is still taken
      sys_store32(&h->state, CKPP_SERVER_EXITING);
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "");
      s = sys_load64(&h->submitted);
      if (s > d->done) {
        sys_store32(&h->state, CKPP_SERVER_RUNNING);
        break;
      }
      return kCmdExit;
    }
    __builtin_amdgcn_s_sleep(4);
  }
  d->t_wait += now_ticks() - t0;
  if (have_tails) {
    // full tails from their low bits: a round's operations of a kind are
    // in flight together, at most the budget, under 2^24 (a table with
    // timers keeps the last round's time)
    d->scan = 0u;
    d->lk0 = d->lk1;
    d->in0 = d->in1;
    d->de0 = d->de1;
    d->lk1 += ((w.x >> 24) - d->lk1) & kLow24;
    d->in1 += (w.x - d->in1) & kLow24;
    d->de1 += ((w.y >> 24) - d->de1) & kLow24;
    d->done = s;
    return kCmdRun;
  }
  // the tails the host wrote before it published `s`
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
  if (a.timed) {
    // the round takes only the bursts from `done` on that share burst
    // done's time (s is cut back to the first burst after them): the time
    // index does not decrease with the burst number, so the last such burst
    // is found by bisection (usually none is needed)
    auto word = [&](uint64_t b) {
      return __hip_atomic_load(&h->tails[b % kQueue][3], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_SYSTEM);
    };
    const uint64_t first = word(d->done);
    const uint64_t idx = first >> kTimeIndexShift;
    if ((word(s - 1u) >> kTimeIndexShift) != idx) {
      uint64_t lo = d->done, hi = s - 1u;  // idx(lo) == idx != idx(hi)
      while (hi - lo > 1u) {
        const uint64_t mid = lo + (hi - lo) / 2u;
        if ((word(mid) >> kTimeIndexShift) == idx) lo = mid;
        else hi = mid;
      }
      s = lo + 1u;
    }
    d->now = (uint32_t)(first & 0xffffu);
    d->scan = (uint32_t)(first >> kScanBit) & 1u;
  }
  const uint64_t *t = h->tails[(s - 1u) % kQueue];
  d->lk0 = d->lk1;
  d->in0 = d->in1;
  d->de0 = d->de1;
  d->lk1 = __hip_atomic_load(t + 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  d->in1 = __hip_atomic_load(t + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  d->de1 = __hip_atomic_load(t + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  d->done = s;
  return kCmdRun;
}

// Lookups [l0, l1) of a round, PER per lane at a time in registers
// (reg_pass_to), the next PER keys loaded while a pass's first heads are in
// flight.  Lookup j of a lane's pass is i + 64 j, its ring slot (i + 64 j)
// & mask.
template <uint32_t PER, uint32_t MODE, bool TIMED>
__device__ void reg_lookups(const ServeArgs &a, const TableRef &T, uint32_t lane, uint64_t wave,
                            uint64_t nwaves, uint64_t l0, uint64_t l1) {
  const uint64_t step = nwaves * 64u * PER;
  uint64_t i = l0 + wave * 64u * PER + lane;
  uint4 k[PER];
#pragma unroll
  for (uint32_t j = 0; j < PER; ++j)
    k[j] = i + 64u * j < l1 ? load_stream(a.lk_keys + ((i + 64u * j) & a.mask)) : zero4();
  for (; i - lane < l1; i += step) {
    bool ok[PER];
    uint8_t *fo[PER];
    uint64_t *vo[PER];
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) {
      const uint64_t slot = (i + 64u * j) & a.mask;
      ok[j] = i + 64u * j < l1;
      fo[j] = a.lk_found + slot;
      vo[j] = a.lk_vals + slot;
    }
    uint4 nk[PER];
    reg_pass_to<MODE, TIMED, PER, true>(T, k, ok, fo, vo, [&] {
#pragma unroll
      for (uint32_t j = 0; j < PER; ++j) {
        const uint64_t n = i + step + 64u * j;
        nk[j] = n < l1 ? load_stream(a.lk_keys + (n & a.mask)) : zero4();
      }
    });
#pragma unroll
    for (uint32_t j = 0; j < PER; ++j) k[j] = nk[j];
  }
}

// The round's lookups [l0, l1), PER per lane per pass in registers
// (reg_pass_to, every mode): 4 when every lane of the grid has at least 4,
// else 2 or 1, so that a round's lookups spread over every wavefront (8 per
// lane measured slower than 4 on the loop's peak workload).
// The loop keeps few wavefronts per SIMD (the batch kernel runs many more),
// and with few to hide each other's stalls the batch kernel's LDS form
// (eight lanes fetching each line into LDS) spends its time in the lane
// exchanges and waits of that fetch; in registers a lookup's pass takes a
// few loads of its own.  TIMED: lookups at time `now` (T carries it, the
// refresh flag and the refreshed expiration time).
template <uint32_t MODE, bool TIMED>
__device__ void lookup_phase(const ServeArgs &a, const TableRef &T, uint64_t l0, uint64_t l1) {
  const uint64_t nwaves = (uint64_t)gridDim.x * kWaves;
  const uint64_t wave = (uint64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t n = l1 - l0, lanes = nwaves * 64u;
  if (n >= 4u * lanes) reg_lookups<4, MODE, TIMED>(a, T, lane, wave, nwaves, l0, l1);
  else if (n >= 2u * lanes) reg_lookups<2, MODE, TIMED>(a, T, lane, wave, nwaves, l0, l1);
  else reg_lookups<1, MODE, TIMED>(a, T, lane, wave, nwaves, l0, l1);
}

// Rank of lane g among `lanes` lanes (whole wavefronts) when the lanes are
// taken column by column: lane 0 of every wavefront, then lane 1 of every
// wavefront, and so on (from the top lane down when `top`).  A round's few
// updates then spread over every wavefront of the grid, a handful per
// wavefront, instead of filling whole wavefronts of the first blocks: a
// wavefront's 64 lanes run their operations in lockstep, each waiting for
// the slowest, and the memory requests of the round spread over all
// compute units.
__device__ __forceinline__ uint64_t column_rank(uint64_t g, uint64_t lanes, bool top) {
  const uint64_t waves = lanes / 64u, lane = g & 63u;
  return (top ? 63u - lane : lane) * waves + g / 64u;
}



// The round's insert keys in a set (open addressing, linear probing): an
// entry belongs to the round whose tag it carries, so the set is never
// cleared.  Built before a barrier, read after it.
__device__ __forceinline__ uint64_t set_slot(const ServeArgs &a, uint4 k) {
  return key_hash(k, kGolden) & a.set_mask;
}

__device__ void set_build(const ServeArgs &a, uint64_t i0, uint64_t i1, uint32_t tag) {
  const uint64_t nlanes = (uint64_t)gridDim.x * kBlock;
  const uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  for (uint64_t j = i0 + column_rank(g, nlanes, false); j < i1; j += nlanes) {
    const uint4 k = a.in_keys[j & a.mask];
    uint64_t pos = set_slot(a, k);
    for (uint64_t probe = 0; probe <= a.set_mask; ++probe, pos = (pos + 1u) & a.set_mask) {
      // one atomic per probe: an entry last tagged by an earlier round is
      // free and now this key's; one already carrying this round's tag
      // belongs to another key of the round (writing the same tag over it
      // changes nothing)
      const uint32_t t = __hip_atomic_exchange(a.set_tag + pos, tag, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
      if (t != tag) {
        uint32_t *dst = reinterpret_cast<uint32_t *>(a.set_keys + pos);
        __hip_atomic_store(dst + 0, k.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(dst + 1, k.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(dst + 2, k.z, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(dst + 3, k.w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  }
}

__device__ bool set_has(const ServeArgs &a, uint4 k, uint32_t tag) {
  uint64_t pos = set_slot(a, k);
  for (uint64_t probe = 0; probe <= a.set_mask; ++probe, pos = (pos + 1u) & a.set_mask) {
    if (a.set_tag[pos] != tag) return false;
    if (key_eq(a.set_keys[pos], k)) return true;
  }
  return false;
}

// TIMED: inserts at time `now`, whose entries expire at now + ttl.  Lanes
// g < path_lanes (whole wavefronts) take the inserts, in column rank.
template <bool TIMED>
__device__ void insert_phase(const ServeArgs &a, uint64_t i0, uint64_t i1, uint32_t now) {
  const uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= a.path_lanes) return;
  uint32_t *path = a.paths + g * (uint64_t)(a.max_kicks ? a.max_kicks : 1u);
  const uint32_t expiry = (now + a.ttl) & 0xffffu;
  for (uint64_t j = i0 + column_rank(g, a.path_lanes, false); j < i1; j += a.path_lanes) {
    const uint64_t slot = j & a.mask;
    const InsertOutcome o =
        insert_one<TIMED>(a.bk, a.in_keys[slot], a.in_vals[slot], a.T.log2b, a.T.seed,
                          a.max_kicks, a.plain != 0u, path, a.spin_limit, expiry, now);
    put_result(a.in_status + slot, (uint8_t)o.status);
    if (o.spun) atomicAdd(a.nspin, 1ull);
  }
}

// The round's deletes.  Every lane of the grid takes the deletes at offsets
// r, r + nlanes, ..., r its column rank from the top lane down (the other
// end of each wavefront from the insert lanes).  Inserts and deletes of a
// round share the wavefronts rather than taking one half of them each:
// a wavefront's time grows with the number of its lanes that run an
// update, since lanes in different states of an update run their steps one
// group after another.  filter: a delete of a key the round also inserts
// is deferred (its result byte set to kDeferred) until every insert of the
// round is done.  deferred_only: runs just the deferred deletes.  TIMED:
// deletes at time `now`.
template <bool TIMED>
__device__ void delete_phase(const ServeArgs &a, uint64_t d0, uint64_t d1, bool filter,
                             uint32_t tag, bool deferred_only, uint32_t now) {
  const uint64_t nlanes = (uint64_t)gridDim.x * kBlock;
  const uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  bool deferred = false;
  for (uint64_t o = column_rank(g, nlanes, true); d0 + o < d1; o += nlanes) {
    const uint64_t slot = (d0 + o) & a.mask;
    if (deferred_only &&
        __hip_atomic_load(a.de_found + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) !=
            kDeferred)
      continue;
    const uint4 k = a.de_keys[slot];
    if (filter && set_has(a, k, tag)) {
      put_result(a.de_found + slot, kDeferred);
      deferred = true;
      continue;
    }
    bool spun = false;
    put_result(a.de_found + slot,
               (uint8_t)delete_one<TIMED>(a.bk, k, a.T.log2b, a.T.seed, a.plain != 0u,
                                          a.spin_limit, &spun, now));
    if (spun) atomicAdd(a.nspin, 1ull);
  }
  if (deferred)
    __hip_atomic_store(&a.dev->deferred, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide barrier inside a round (every thread of every block calls it).
__device__ bool phase_barrier(const ServeArgs &a, uint32_t epoch, uint32_t phase,
                              uint32_t *s_ok) {
  __builtin_amdgcn_s_waitcnt(0);  // this wave's accesses of the phase are done
  __syncthreads();
  if (threadIdx.x == 0) block_arrive(a, epoch);
  if (blockIdx.x == 0) {
    if (threadIdx.x < 64u) {
      const bool ok = gather(a, epoch, kPhaseMs * kTicksPerMs);
      if (threadIdx.x == 0) {
        // the phase that just ended: lookups, inserts, or a step of the
        // anti-revival scan (counted with the round boundaries)
        const uint64_t t = now_ticks();
        *(phase == 0 ? &a.dev->t_lookup : phase == 1 ? &a.dev->t_insert : &a.dev->t_boundary) +=
            t - a.dev->t_mark;
        a.dev->t_mark = t;
        release_epoch(a.dev, epoch);
        *s_ok = ok ? 1u : 0u;
      }
    }
  } else if (threadIdx.x == 0) {
    *s_ok = wait_release(a, epoch, kPhaseMs * kTicksPerMs) ? 1u : 0u;
  }
  __syncthreads();
  return *s_ok != 0u;
}

// TIMED: the table has timers (the round's time and scan flag come with
// its ranges).
template <uint32_t MODE, bool TIMED>
__global__ void __launch_bounds__(kBlock) serve_loop(ServeArgs a) {
  // the round's ranges [l0, l1), [i0, i1), [d0, d1), time and scan flag;
  // the other blocks keep the last round's ends here between rounds
  __shared__ uint64_t s_range[8];
  __shared__ uint32_t s_cmd, s_ok;
  const bool leader = blockIdx.x == 0 && threadIdx.x == 0;
  ServeDev *d = a.dev;
  if (threadIdx.x == 0) {
    // the ends of the last launch's last round (the leader writes them only
    // after every block has arrived at the first boundary)
    auto get = [](const uint64_t *p) {
      return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    s_range[0] = s_range[1] = get(&d->lk1);
    s_range[2] = s_range[3] = get(&d->in1);
    s_range[4] = s_range[5] = get(&d->de1);
  }
  // epochs continue from the last launch's (nothing writes gen until every
  // block of this launch has arrived at its first barrier)
  uint32_t epoch = poll32(&d->gen);
  bool ran = false;
  // the leader's note of the phase that ends at the next boundary:
  // 0 lookups, 1 inserts (or inserts and deletes together), 2 deletes
  uint32_t last_phase = 0u;
  for (;;) {
    // round boundary
    ++epoch;
    __syncthreads();
    // every wave of the block has waited for its accesses (the end of the
    // round below), the results' write-through stores among them
    if (threadIdx.x == 0) block_arrive(a, epoch);
    if (blockIdx.x == 0) {
      if (threadIdx.x < 64u) {
        const bool ok = gather(a, epoch, kPhaseMs * kTicksPerMs);
        if (threadIdx.x == 0) {
          const uint64_t tg = now_ticks();
          if (ran) {  // the round's last phase ends here
            const uint64_t dt = tg - d->t_mark;
            if (last_phase == 2u) d->t_delete += dt;
            else if (last_phase == 1u) d->t_insert += dt;
            else d->t_lookup += dt;
          }
          const uint64_t w0 = d->t_wait;
          uint32_t cmd;
          if (ok && ran && __hip_atomic_load(&d->deferred, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT)) {
            // some deletes of the round wait for its inserts, which are all
            // done now: run them before the round is published complete
            // (a device-coherent store: blocks set the flag with atomics)
            __hip_atomic_store(&d->deferred, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            cmd = kCmdDeferred;
          } else {
            cmd = ok ? leader_next_round(a, ran) : kCmdExit;
          }
          const uint32_t scan = TIMED && cmd == kCmdRun ? d->scan : 0u;
          const uint32_t tnow = TIMED ? d->now : 0u;
          const uint64_t tr = now_ticks();
          d->t_boundary += (tr - tg) - (d->t_wait - w0);
          d->t_mark = tr;
          publish_round(d, epoch, cmd, scan, tnow);
          s_cmd = cmd;
          // the leader's own ranges (its own writes)
          s_range[0] = d->lk0;
          s_range[1] = d->lk1;
          s_range[2] = d->in0;
          s_range[3] = d->in1;
          s_range[4] = d->de0;
          s_range[5] = d->de1;
          s_range[6] = tnow;
          s_range[7] = scan;
        }
      }
    } else if (threadIdx.x == 0) {
      uint64_t r[4];
      s_cmd = wait_round(a, epoch, a.idle_ticks + kPhaseMs * kTicksPerMs, r)
                  ? (uint32_t)(r[0] >> 32) & 0xffffu
                  : kCmdExit;
      if (s_cmd == kCmdRun) {
        // full ends from their low 48 bits and the last round's ends (a
        // round's operations of a kind are fewer than 2^48)
        const uint64_t m = kLow48;
        s_range[0] = s_range[1];
        s_range[1] += (r[1] - s_range[1]) & m;
        s_range[2] = s_range[3];
        s_range[3] += (r[2] - s_range[3]) & m;
        s_range[4] = s_range[5];
        s_range[5] += (r[3] - s_range[5]) & m;
      }
      // a deferred round keeps the last round's ranges
      s_range[6] = r[0] & 0xffffu;
      s_range[7] = s_cmd == kCmdRun ? (r[0] >> 16) & 1u : 0u;
    }
    if (threadIdx.x == 0) {
      // the round's ring entries were written by the host or a copy engine
      // while the kernel ran: drop any cached copy of them
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
    }
    __syncthreads();
    if (s_cmd != kCmdRun && s_cmd != kCmdDeferred) break;
    const uint64_t l0 = s_range[0], l1 = s_range[1], i0 = s_range[2], i1 = s_range[3];
    const uint64_t d0 = s_range[4], d1 = s_range[5];
    const uint32_t now = (uint32_t)s_range[6];
    if (s_cmd == kCmdDeferred) {
      delete_phase<TIMED>(a, d0, d1, false, 0u, true, now);
      last_phase = 2u;
    } else {
      if (TIMED && s_range[7]) {
        // anti-revival scan: expired entries out, with the counter and
        // filter maintenance of a delete; a barrier before the lookups
        const uint64_t gtid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
        const uint64_t gthreads = (uint64_t)gridDim.x * kBlock;
        expire_slots_pass<kScanUnroll>(a.bk, a.nb, now, a.plain != 0u, gtid, gthreads);
        if (!phase_barrier(a, ++epoch, 2u, &s_ok)) break;
      }
      TableRef T = a.T;
      if (TIMED) {
        T.now = now;
        T.refresh = a.refresh;
        T.expiry = (now + a.ttl) & 0xffffu;
      }
      // a round with inserts and deletes runs them side by side, deferring
      // the deletes of keys it also inserts, when the updates are few enough
      // for each to get a lane of its own with half the lanes to spare
      // (building and probing the insert-key set costs about as much as the
      // barrier it saves once most lanes are busy) and the set has room;
      // else it runs the inserts, then the deletes
      const bool ins = i1 > i0, del = d1 > d0;
      const uint64_t nlanes = (uint64_t)gridDim.x * kBlock;
      const uint64_t lanes = nlanes < a.path_lanes ? nlanes : a.path_lanes;
      const bool merge = ins && del && 2u * (i1 - i0) <= a.set_mask + 1u &&
                         2u * ((i1 - i0) + (d1 - d0)) <= lanes;
      const uint32_t tag = epoch;  // unique to this round
      lookup_phase<MODE, TIMED>(a, T, l0, l1);
      if (merge) set_build(a, i0, i1, tag);
      last_phase = 0u;
      if (ins || del) {
        if (!phase_barrier(a, ++epoch, 0u, &s_ok)) break;
        if (!ins || !del || merge) {
          insert_phase<TIMED>(a, i0, i1, now);
          delete_phase<TIMED>(a, d0, d1, merge, tag, false, now);
          last_phase = ins ? 1u : 2u;
        } else {
          insert_phase<TIMED>(a, i0, i1, now);
          if (!phase_barrier(a, ++epoch, 1u, &s_ok)) break;
          delete_phase<TIMED>(a, d0, d1, false, 0u, false, now);
          last_phase = 2u;
        }
      }
    }
    // this wave's results of the round are written (into the L2 cache); the
    // block's thread 0 writes them back at the boundary
    __builtin_amdgcn_s_waitcnt(0);
    ran = true;
  }
  if (leader) {
    const uint32_t aborted = poll32(&d->abort);
    sys_store32(&a.host->state, aborted ? CKPP_SERVER_ABORTED : CKPP_SERVER_STOPPED);
  }
}

}  // namespace
}  // namespace ckpp

using ckpp::ServeArgs;
using ckpp::ServeDev;
using ckpp::ServeHost;

struct ckpp_server {
  ckpp_table *t;
  int device;
  ckpp_server_config_t cfg;
  uint32_t mode;
  uint32_t grid;
  hipStream_t stream;
  ServeHost *host;
  ServeDev *dev;
  uint32_t *paths;
  uint32_t *arrive;
  uint4 *set_keys;
  uint32_t *set_tag;
  ckpp_server_rings_t rings;
  ServeArgs args;
  uint64_t submitted;
  uint64_t tails[3];
  std::vector<uint64_t> burst_tails;  // kQueue x 3: cumulative tails after burst k
  uint64_t launches;
  bool launched;
  // tables with timers: the time of bursts submitted from now on, the time
  // of the last requested scan, time changes so far, whether a time was set
  uint16_t now;
  uint16_t last_scan;
  uint64_t time_index;
  uint64_t index_first;  // the first burst staged at the current time index
  bool time_set;
};

namespace {

using ckpp::DeviceGuard;
using ckpp::dev_status;

std::atomic<uint64_t> *host_u64(uint64_t *p) { return reinterpret_cast<std::atomic<uint64_t> *>(p); }
std::atomic<uint32_t> *host_u32(uint32_t *p) { return reinterpret_cast<std::atomic<uint32_t> *>(p); }

template <bool TIMED>
const void *loop_kernel(uint32_t mode) {
  if (mode == ckpp::kModeBoth)
    return reinterpret_cast<const void *>(&ckpp::serve_loop<ckpp::kModeBoth, TIMED>);
  if (mode == ckpp::kModeOptimistic)
    return reinterpret_cast<const void *>(&ckpp::serve_loop<ckpp::kModeOptimistic, TIMED>);
  return reinterpret_cast<const void *>(&ckpp::serve_loop<ckpp::kModeCuckoopp, TIMED>);
}

const void *loop_kernel(uint32_t mode, bool timed) {
  return timed ? loop_kernel<true>(mode) : loop_kernel<false>(mode);
}

hipError_t launch_loop(ckpp_server *s) {
  void *kargs[] = {&s->args};
  const void *fn = loop_kernel(s->mode, s->args.timed != 0u);
  host_u32(&s->host->state)->store(CKPP_SERVER_RUNNING, std::memory_order_seq_cst);
  hipError_t e = hipLaunchCooperativeKernel(fn, dim3(s->grid), dim3(ckpp::kBlock), kargs, 0,
                                            s->stream);
  if (e != hipSuccess) {
    host_u32(&s->host->state)->store(CKPP_SERVER_STOPPED, std::memory_order_seq_cst);
    return e;
  }
  s->launches += 1;
  s->launched = true;
  return hipSuccess;
}

// Makes sure a loop is running after a submit (see the exit protocol in
// leader_next_round).
int ensure_running(ckpp_server *s) {
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    const uint32_t st = host_u32(&s->host->state)->load(std::memory_order_seq_cst);
    if (st == CKPP_SERVER_RUNNING) return CKPP_OK;
    if (st == CKPP_SERVER_ABORTED) return CKPP_EDEVICE;
    if (st == CKPP_SERVER_EXITING &&
        std::chrono::steady_clock::now() - t0 < std::chrono::seconds(5)) {
      std::this_thread::yield();  // the loop decides within microseconds
      continue;
    }
    // stopped: the previous kernel has left (or is leaving) the loop
    if (hipStreamSynchronize(s->stream) != hipSuccess) return CKPP_EDEVICE;
    if (host_u32(&s->host->state)->load(std::memory_order_seq_cst) == CKPP_SERVER_ABORTED)
      return CKPP_EDEVICE;
    return dev_status(launch_loop(s));
  }
}

void free_server(ckpp_server *s) {
  (void)hipFree(s->rings.d_lookup_keys);
  (void)hipFree(s->rings.d_lookup_found);
  (void)hipFree(s->rings.d_lookup_values);
  (void)hipFree(s->rings.d_insert_keys);
  (void)hipFree(s->rings.d_insert_values);
  (void)hipFree(s->rings.d_insert_status);
  (void)hipFree(s->rings.d_delete_keys);
  (void)hipFree(s->rings.d_delete_found);
  (void)hipFree(s->paths);
  (void)hipFree(s->arrive);
  (void)hipFree(s->set_keys);
  (void)hipFree(s->set_tag);
  (void)hipFree(s->dev);
  if (s->host) (void)hipHostFree(s->host);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

bool pow2(uint64_t x) { return x && !(x & (x - 1)); }

}  // namespace

extern "C" {

int ckpp_server_create(ckpp_server **out, ckpp_table *t, const ckpp_server_config_t *cfg) {
  if (!out) return CKPP_EINVAL;
  *out = nullptr;
  if (!t || !cfg) return CKPP_EINVAL;
  const ckpp_server_config_t &c = *cfg;
  const bool timed = (t->flags & CKPP_TIMERS) != 0u;
  const uint32_t ttl = c.ttl & ~CKPP_SERVER_REFRESH;
  if (timed ? (ttl < 1 || ttl > 1023) : c.ttl != 0) return CKPP_EINVAL;
  if (!pow2(c.capacity) || c.capacity < 64 || c.capacity > (1ull << 30)) return CKPP_EINVAL;
  if (c.budget == 0 || c.budget > c.capacity) return CKPP_EINVAL;
  if (c.mode > CKPP_LOOKUP_OPTIMISTIC || c.blocks_per_cu < 1 || c.blocks_per_cu > 4) return CKPP_EINVAL;
  if (c.idle_ms < 1 || c.idle_ms > 60000) return CKPP_EINVAL;
  DeviceGuard g(t->device);
  if (!g.ok()) return CKPP_EDEVICE;
  ckpp_server *s = new (std::nothrow) ckpp_server();
  if (!s) return CKPP_ENOMEM;
  s->t = t;
  s->device = t->device;
  s->cfg = c;
  s->mode = c.mode;
  if (s->mode == CKPP_LOOKUP_DEFAULT && (t->flags & CKPP_PLAIN)) s->mode = CKPP_LOOKUP_BOTH;
  s->burst_tails.assign(3ull * ckpp::kQueue, 0ull);
  const uint64_t C = c.capacity;
  ckpp_server_rings_t &r = s->rings;
  r.capacity = C;
  hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipMalloc(&r.d_lookup_keys, C * 16);
  if (e == hipSuccess) e = hipMalloc(&r.d_lookup_found, C);
  if (e == hipSuccess) e = hipMalloc(&r.d_lookup_values, C * 8);
  if (e == hipSuccess) e = hipMalloc(&r.d_insert_keys, C * 16);
  if (e == hipSuccess) e = hipMalloc(&r.d_insert_values, C * 8);
  if (e == hipSuccess) e = hipMalloc(&r.d_insert_status, C);
  if (e == hipSuccess) e = hipMalloc(&r.d_delete_keys, C * 16);
  if (e == hipSuccess) e = hipMalloc(&r.d_delete_found, C);
  // the loop kernel's grid: co-resident blocks only
  int per_cu = 0;
  const void *fn = loop_kernel(s->mode, timed);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, ckpp::kBlock, 0);
  if (e == hipSuccess && per_cu < 1) e = hipErrorInvalidConfiguration;
  const uint32_t bpc = std::min<uint32_t>(c.blocks_per_cu, (uint32_t)std::max(per_cu, 1));
  s->grid = bpc * (uint32_t)t->num_cus;
  const uint32_t path_lanes = std::min<uint32_t>(ckpp::kMaxPathLanes, s->grid * ckpp::kBlock);
  const uint64_t path_words = (uint64_t)path_lanes * (t->max_kicks ? t->max_kicks : 1u);
  if (e == hipSuccess) e = hipMalloc(&s->paths, path_words * 4);
  if (e == hipSuccess) e = hipMalloc(&s->dev, sizeof(ServeDev));
  if (e == hipSuccess) e = hipMemset(s->dev, 0, sizeof(ServeDev));
  const uint64_t flag_bytes = (uint64_t)s->grid * ckpp::kFlagStride * 4u;
  if (e == hipSuccess) e = hipMalloc(&s->arrive, flag_bytes);
  if (e == hipSuccess) e = hipMemset(s->arrive, 0, flag_bytes);
  // the round's insert-key set: twice the inserts one round may take
  uint64_t set_entries = 64;
  while (set_entries < 2u * c.budget && set_entries < ckpp::kMaxSetEntries) set_entries <<= 1;
  if (e == hipSuccess) e = hipMalloc(&s->set_keys, set_entries * 16);
  if (e == hipSuccess) e = hipMalloc(&s->set_tag, set_entries * 4);
  if (e == hipSuccess) e = hipMemset(s->set_tag, 0, set_entries * 4);
  if (e == hipSuccess) e = hipHostMalloc(&s->host, sizeof(ServeHost), hipHostMallocCoherent);
  if (e == hipSuccess) memset(s->host, 0, sizeof(ServeHost));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_server(s);
    return dev_status(e);
  }
  ServeArgs &a = s->args;
  a.T = ckpp::TableRef{reinterpret_cast<const uint4 *>(t->d_table), t->seed, t->log2_buckets};
  a.bk = t->d_table;
  a.max_kicks = t->max_kicks;
  a.plain = (t->flags & CKPP_PLAIN) ? 1u : 0u;
  a.host = s->host;
  a.dev = s->dev;
  a.arrive = s->arrive;
  a.mask = C - 1u;
  a.lk_keys = reinterpret_cast<const uint4 *>(r.d_lookup_keys);
  a.lk_found = r.d_lookup_found;
  a.lk_vals = r.d_lookup_values;
  a.in_keys = reinterpret_cast<const uint4 *>(r.d_insert_keys);
  a.in_vals = r.d_insert_values;
  a.in_status = r.d_insert_status;
  a.de_keys = reinterpret_cast<const uint4 *>(r.d_delete_keys);
  a.de_found = r.d_delete_found;
  a.paths = s->paths;
  a.path_lanes = path_lanes;
  a.spin_limit = t->retry_limit;
  a.idle_ticks = (uint64_t)c.idle_ms * ckpp::kTicksPerMs;
  a.nspin = reinterpret_cast<unsigned long long *>(t->d_stats) + 127;
  a.set_keys = s->set_keys;
  a.set_tag = s->set_tag;
  a.set_mask = set_entries - 1u;
  a.timed = timed ? 1u : 0u;
  a.fast_tails = c.budget < ckpp::kFastTailsBudget ? 1u : 0u;
  a.ttl = timed ? ttl : 0u;
  a.refresh = timed && (c.ttl & CKPP_SERVER_REFRESH) ? 1u : 0u;
  a.nb = 1ull << t->log2_buckets;
  e = launch_loop(s);
  if (e != hipSuccess) {
    free_server(s);
    return dev_status(e);
  }
  *out = s;
  return CKPP_OK;
}

int ckpp_server_rings(const ckpp_server *s, ckpp_server_rings_t *out) {
  if (!s || !out) return CKPP_EINVAL;
  *out = s->rings;
  return CKPP_OK;
}

int ckpp_server_put(ckpp_server *s, uint32_t kind, uint64_t pos, const void *d_keys,
                    const uint64_t *d_values, uint32_t n, void *stream) {
  if (!s || kind > CKPP_OP_DELETE || n > s->rings.capacity) return CKPP_EINVAL;
  if (n == 0) return CKPP_OK;
  if (!d_keys || (kind == CKPP_OP_INSERT) != (d_values != nullptr)) return CKPP_EINVAL;
  DeviceGuard g(s->device);
  if (!g.ok()) return CKPP_EDEVICE;
  const ckpp_server_rings_t &r = s->rings;
  uint8_t *keys = static_cast<uint8_t *>(kind == CKPP_OP_LOOKUP   ? r.d_lookup_keys
                                         : kind == CKPP_OP_INSERT ? r.d_insert_keys
                                                                  : r.d_delete_keys);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const uint64_t C = r.capacity, first = pos % C, n1 = std::min<uint64_t>(n, C - first);
  const uint8_t *src = static_cast<const uint8_t *>(d_keys);
  hipError_t e = hipMemcpyAsync(keys + first * 16, src, n1 * 16, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess && n1 < n)
    e = hipMemcpyAsync(keys, src + n1 * 16, (n - n1) * 16, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess && d_values) {
    e = hipMemcpyAsync(r.d_insert_values + first, d_values, n1 * 8, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && n1 < n)
      e = hipMemcpyAsync(r.d_insert_values, d_values + n1, (n - n1) * 8, hipMemcpyDeviceToDevice,
                         st);
  }
  return dev_status(e);
}

int ckpp_server_get(ckpp_server *s, uint32_t kind, uint64_t pos, uint32_t n, uint8_t *d_flags,
                    uint64_t *d_values, void *stream) {
  if (!s || kind > CKPP_OP_DELETE || n > s->rings.capacity) return CKPP_EINVAL;
  if (n == 0) return CKPP_OK;
  if (!d_flags || (kind == CKPP_OP_LOOKUP) != (d_values != nullptr)) return CKPP_EINVAL;
  DeviceGuard g(s->device);
  if (!g.ok()) return CKPP_EDEVICE;
  const ckpp_server_rings_t &r = s->rings;
  const uint8_t *flags = kind == CKPP_OP_LOOKUP   ? r.d_lookup_found
                         : kind == CKPP_OP_INSERT ? r.d_insert_status
                                                  : r.d_delete_found;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const uint64_t C = r.capacity, first = pos % C, n1 = std::min<uint64_t>(n, C - first);
  hipError_t e = hipMemcpyAsync(d_flags, flags + first, n1, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess && n1 < n)
    e = hipMemcpyAsync(d_flags + n1, flags, n - n1, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess && d_values) {
    e = hipMemcpyAsync(d_values, r.d_lookup_values + first, n1 * 8, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && n1 < n)
      e = hipMemcpyAsync(d_values + n1, r.d_lookup_values, (n - n1) * 8, hipMemcpyDeviceToDevice,
                         st);
  }
  return dev_status(e);
}

int ckpp_server_status(ckpp_server *s, ckpp_server_status_t *out) {
  if (!s || !out) return CKPP_EINVAL;
  out->submitted = s->submitted;
  out->completed = host_u64(&s->host->completed)->load(std::memory_order_acquire);
  out->lookup_tail = s->tails[0];
  out->insert_tail = s->tails[1];
  out->delete_tail = s->tails[2];
  out->rounds = host_u64(&s->host->rounds)->load(std::memory_order_acquire);
  out->launches = s->launches;
  out->state = host_u32(&s->host->state)->load(std::memory_order_acquire);
  out->grid = s->grid;
  // the loop's phase clocks (device memory; a copy while it runs is a
  // snapshot as of the last round boundary)
  uint64_t t[5] = {0, 0, 0, 0, 0};
  DeviceGuard g(s->device);
  if (!g.ok() || hipMemcpy(t, &s->dev->t_lookup, sizeof(t), hipMemcpyDeviceToHost) != hipSuccess)
    return CKPP_EDEVICE;
  // real-time counter ticks are 10 ns
  out->lookup_ns = t[0] * 10u;
  out->insert_ns = t[1] * 10u;
  out->delete_ns = t[2] * 10u;
  out->boundary_ns = t[3] * 10u;
  out->wait_ns = t[4] * 10u;
  return CKPP_OK;
}

}  // extern "C"

namespace {

// Records a burst's tails for the loop without publishing it; CKPP_EBUSY
// when it does not fit the budget or the queue.  `done`: bursts completed.
// scan: the burst's round starts with the anti-revival scan.
int stage_burst(ckpp_server *s, uint64_t done, uint32_t n_lookup, uint32_t n_insert,
                uint32_t n_delete, bool scan = false) {
  if (s->submitted - done >= ckpp::kQueue) return CKPP_EBUSY;
  // ops in flight of each kind after this burst
  const uint64_t *dt = done ? &s->burst_tails[3 * ((done - 1) % ckpp::kQueue)] : nullptr;
  const uint64_t n[3] = {n_lookup, n_insert, n_delete};
  uint64_t nt[3];
  for (int k = 0; k < 3; ++k) {
    nt[k] = s->tails[k] + n[k];
    if (nt[k] - (dt ? dt[k] : 0ull) > s->cfg.budget) return CKPP_EBUSY;
  }
  const uint64_t b = s->submitted;
  uint64_t *slot = s->host->tails[b % ckpp::kQueue];
  for (int k = 0; k < 3; ++k) {
    host_u64(&slot[k])->store(nt[k], std::memory_order_relaxed);
    s->burst_tails[3 * (b % ckpp::kQueue) + k] = nt[k];
    s->tails[k] = nt[k];
  }
  const uint64_t tw = (s->time_index << ckpp::kTimeIndexShift) |
                      ((uint64_t)(scan ? 1u : 0u) << ckpp::kScanBit) | s->now;
  host_u64(&slot[3])->store(tw, std::memory_order_relaxed);
  // (operations are put in the rings before their burst is staged; the loop
  // takes a staged burst early only while submitted ones wait)
  if (s->args.fast_tails) {
    const uint64_t tag = (uint64_t)(ckpp::kTagValid | (uint32_t)(b & ckpp::kTagMask)) << 48;
    const uint64_t win = b >= ckpp::kIndexFirstWindow ? b - ckpp::kIndexFirstWindow : 0u;
    const uint64_t f = s->index_first > win ? s->index_first : win;
    const uint64_t w0 = tag | (nt[0] & ckpp::kLow24) << 24 | (nt[1] & ckpp::kLow24);
    const uint64_t w1 = tag | (nt[2] & ckpp::kLow24) << 24 | (f & ckpp::kLow24);
    // one aligned 16-byte store (single-copy atomic on x86-64 processors
    // with AVX; the tags catch a torn read anyway), after the stores above
    std::atomic_thread_fence(std::memory_order_release);
    _mm_store_si128(reinterpret_cast<__m128i *>(s->host->latest),
                    _mm_set_epi64x((long long)w1, (long long)w0));
  }
  s->submitted = b + 1;
  return CKPP_OK;
}

// Hands every staged burst to the loop (one store), relaunching it if it
// has left.
int publish(ckpp_server *s) {
  host_u64(&s->host->submitted)->store(s->submitted, std::memory_order_seq_cst);
  DeviceGuard g(s->device);
  if (!g.ok()) return CKPP_EDEVICE;
  return ensure_running(s);
}

}  // namespace

extern "C" {

int ckpp_server_submit(ckpp_server *s, uint32_t n_lookup, uint32_t n_insert, uint32_t n_delete,
                       uint64_t *burst) {
  if (!s) return CKPP_EINVAL;
  const uint64_t done = host_u64(&s->host->completed)->load(std::memory_order_acquire);
  const int rc = stage_burst(s, done, n_lookup, n_insert, n_delete);
  if (rc != CKPP_OK) return rc;
  if (burst) *burst = s->submitted - 1;
  return publish(s);
}

int ckpp_server_set_time(ckpp_server *s, uint16_t now) {
  if (!s || !s->args.timed) return CKPP_EINVAL;
  if (s->time_set && ((uint16_t)(now - s->now) >= ckpp::kMaxTimeStep)) return CKPP_EINVAL;
  if (s->time_set && now == s->now) return CKPP_OK;
  // the scan is due when this time is 16384 or more past the last one (an
  // expired entry looks alive again 64512 units after it expired, and no
  // time change exceeds 16383, so the scans are at most 32767 apart)
  const bool scan = !s->time_set || (uint16_t)(now - s->last_scan) >= ckpp::kMaxTimeStep;
  const uint16_t old_now = s->now;
  const uint64_t old_index = s->time_index;
  s->now = now;
  s->time_index += 1;
  const uint64_t old_first = s->index_first;
  s->index_first = s->submitted;
  if (scan) {
    const uint64_t done = host_u64(&s->host->completed)->load(std::memory_order_acquire);
    const int rc = stage_burst(s, done, 0u, 0u, 0u, true);
    if (rc != CKPP_OK) {
      s->now = old_now;
      s->time_index = old_index;
      s->index_first = old_first;
      return rc;
    }
    s->last_scan = now;
  }
  s->time_set = true;
  return scan ? publish(s) : CKPP_OK;
}

int ckpp_server_wait(ckpp_server *s, uint64_t burst, uint32_t timeout_ms) {
  if (!s || burst >= s->submitted) return CKPP_EINVAL;
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    if (host_u64(&s->host->completed)->load(std::memory_order_acquire) > burst) return CKPP_OK;
    const uint32_t st = host_u32(&s->host->state)->load(std::memory_order_acquire);
    if (st == CKPP_SERVER_ABORTED) return CKPP_EDEVICE;
    if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(timeout_ms))
      return CKPP_ETIMEOUT;
    std::this_thread::yield();
  }
}

int ckpp_server_replay(ckpp_server *s, uint64_t nbursts, const uint32_t *h_nlookup,
                       const uint32_t *h_ninsert, const uint32_t *h_ndelete,
                       const double *h_arrival_s, double *h_admit_s, double *h_done_s,
                       double timeout_s) {
  if (!s || (nbursts && (!h_nlookup || !h_ninsert || !h_ndelete || !h_arrival_s || !h_admit_s ||
                         !h_done_s)))
    return CKPP_EINVAL;
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  auto since = [&](clk::time_point t) { return std::chrono::duration<double>(t - t0).count(); };
  const uint64_t first = s->submitted;  // burst number of stream entry 0
  uint64_t next = 0, seen = 0;
  while (seen < nbursts) {
    const auto now = clk::now();
    const double ts = since(now);
    // every burst that has arrived and fits is staged, then all are
    // published with one store
    const uint64_t done = host_u64(&s->host->completed)->load(std::memory_order_acquire);
    const uint64_t staged = next;
    while (next < nbursts && h_arrival_s[next] <= ts) {
      if (stage_burst(s, done, h_nlookup[next], h_ninsert[next], h_ndelete[next]) != CKPP_OK)
        break;
      ++next;
    }
    if (next > staged) {
      const int rc = publish(s);
      if (rc != CKPP_OK) return rc;
      const double ta = since(clk::now());
      for (uint64_t i = staged; i < next; ++i) h_admit_s[i] = ta;
    }
    const uint64_t c = host_u64(&s->host->completed)->load(std::memory_order_acquire);
    if (c > first + seen) {
      const double td = since(clk::now());
      while (seen < nbursts && first + seen < c) h_done_s[seen++] = td;
    }
    if (host_u32(&s->host->state)->load(std::memory_order_acquire) == CKPP_SERVER_ABORTED)
      return CKPP_EDEVICE;
    if (ts > timeout_s) return CKPP_ETIMEOUT;
  }
  return CKPP_OK;
}

int ckpp_server_destroy(ckpp_server *s) {
  if (!s) return CKPP_OK;
  DeviceGuard g(s->device);
  host_u32(&s->host->stop)->store(1u, std::memory_order_seq_cst);
  (void)hipStreamSynchronize(s->stream);
  free_server(s);
  return CKPP_OK;
}

}  // extern "C"
