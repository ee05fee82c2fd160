// ckpp_device.h -- device-side view of a Cuckoo++ table (gfx950).
//
// Device layout: bucket b owns 256 bytes (two 128-byte L2 lines) at byte
// 256*b of one array.  A random 128-byte read costs one memory request, the
// same as a 64-byte one, so a bucket's metadata (Sec. 4.3) shares its first
// line with the keys and values of slots 0..3; the implicit index of the
// paper (record position derived from bucket and slot, Sec. 4.3) is kept.
//   line 0:   0..15  tag[8]   u16, slot s at bytes 2s
//            16..23  bloom    u64  (Sec. 4.1)
//            24..27  meta     moved u16 | busy u8 << 16 | sec u8 << 24
//            28..31  lock     u32  (zero outside a running insert/delete)
//            32..95  key[0..3]   16 bytes each
//            96..127 value[0..3]  8 bytes each
//   line 1: 128..191 key[4..7]
//           192..223 value[4..7]
//           224..255 other[0..7] u32: the entry's other bucket, so a cuckoo
//                    path is searched without reading keys (Sec. 4.3)
// Viewed as uint4 quarters: 16 per bucket; quarter r of line 0 is read by
// lane r of an 8-lane lookup group.
// On a table with timers (Sec. 4.2) the value word of a slot holds the value
// in its low 48 bits and the entry's 16-bit expiration time in its high 16
// bits: the time is read with the value, in the line that holds the key, so
// checking it costs a lookup no extra memory request.  Values of such a
// table are therefore limited to 48 bits (a documented precondition; the
// paper keeps the times beside the tags, Sec. 4.3).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ckpp {

constexpr uint32_t kSlots = 8;
constexpr uint32_t kBucketBytes = 256;
constexpr uint32_t kQuartersPerBucket = 16;  // 256-byte bucket = 16 x uint4
constexpr uint32_t kMetaOffset = 24;         // byte offset of the meta word
constexpr uint32_t kLockOffset = 28;         // byte offset of the lock word
constexpr uint32_t kOtherOffset = 224;       // byte offset of other[0]

// Byte offsets of the key and value of slot s within a bucket.
__device__ __forceinline__ uint32_t key_offset(uint32_t s) {
  return s < 4u ? 32u + 16u * s : 128u + 16u * (s - 4u);
}
__device__ __forceinline__ uint32_t value_offset(uint32_t s) {
  return s < 4u ? 96u + 8u * s : 192u + 8u * (s - 4u);
}

// SplitMix64 output finalizer (Steele, Lea, Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// Hash of a key held as four little-endian u32 words:
// h = mix(mix(lo ^ seed) ^ hi), lo = w0 | w1 << 32, hi = w2 | w3 << 32.
__device__ __forceinline__ uint64_t key_hash(uint4 k, uint64_t seed) {
  const uint64_t lo = (uint64_t)k.x | ((uint64_t)k.y << 32);
  const uint64_t hi = (uint64_t)k.z | ((uint64_t)k.w << 32);
  return mix64(mix64(lo ^ seed) ^ hi);
}

// Salt of the second hash word of tables above 2^24 buckets: an arbitrary
// odd 64-bit constant (the second prime of xxHash64), so that g is a mix of h
// independent of the first.
constexpr uint64_t kSecondWordSalt = 0xc2b2ae3d27d4eb4full;

// Fields of a key derived from its hash for 2^log2b buckets: primary p,
// alternate a (never equal to p), 16-bit tag, and the two bloom bits, taken
// from the alternate-bucket field (Sec. 4.1).  That field is h >> 24 up to
// 2^24 buckets; above, where it would overlap p, a second word
// g = mix(h ^ kSecondWordSalt) gives a = g mod 2^B and the bloom bit
// indices (g >> 32) mod 64 and (g >> 38) mod 64.  bidx packs the two
// indices (first | second << 6).
struct KeyFields {
  uint32_t p;
  uint32_t a;
  uint32_t tag;
  uint32_t bidx;
  uint64_t bloom_bits;
};

__device__ __forceinline__ KeyFields key_fields(uint64_t h, uint32_t log2b) {
  const uint32_t mask = (1u << log2b) - 1u;
  KeyFields f;
  f.p = (uint32_t)h & mask;
  f.tag = (uint32_t)(h >> 48);
  uint64_t field = h >> 24;
  uint32_t a = (uint32_t)field & mask;
  uint32_t b1 = (uint32_t)field & 63u, b2 = (uint32_t)(field >> 6) & 63u;
  if (log2b > 24u) {
    const uint64_t g = mix64(h ^ kSecondWordSalt);
    a = (uint32_t)g & mask;
    b1 = (uint32_t)(g >> 32) & 63u;
    b2 = (uint32_t)(g >> 38) & 63u;
  }
  f.a = (a == f.p) ? (a ^ 1u) : a;
  f.bidx = b1 | (b2 << 6);
  f.bloom_bits = (1ull << b1) | (1ull << b2);
  return f;
}

// Exact per-slot equality of the eight 16-bit tags with t: bit s of the
// result is set iff tag[s] == t.
__device__ __forceinline__ uint32_t tag_eq_mask(uint4 q0, uint32_t t) {
  uint32_t r = 0;
  r |= ((q0.x & 0xffffu) == t) ? 0x01u : 0u;
  r |= ((q0.x >> 16) == t) ? 0x02u : 0u;
  r |= ((q0.y & 0xffffu) == t) ? 0x04u : 0u;
  r |= ((q0.y >> 16) == t) ? 0x08u : 0u;
  r |= ((q0.z & 0xffffu) == t) ? 0x10u : 0u;
  r |= ((q0.z >> 16) == t) ? 0x20u : 0u;
  r |= ((q0.w & 0xffffu) == t) ? 0x40u : 0u;
  r |= ((q0.w >> 16) == t) ? 0x80u : 0u;
  return r;
}

__device__ __forceinline__ uint32_t meta_busy(uint32_t meta) { return (meta >> 16) & 0xffu; }
__device__ __forceinline__ uint32_t meta_sec(uint32_t meta) { return meta >> 24; }
__device__ __forceinline__ uint32_t meta_moved(uint32_t meta) { return meta & 0xffffu; }
__device__ __forceinline__ uint32_t make_meta(uint32_t moved, uint32_t busy, uint32_t sec) {
  return (moved & 0xffffu) | ((busy & 0xffu) << 16) | ((sec & 0xffu) << 24);
}

// The filter passes iff both of the key's bits are set: one AND of the
// 64-bit filter with the key's two-bit mask and one comparison (the test
// Sec. 6 counts as the whole run-time cost of the filter).
__device__ __forceinline__ bool bloom_pass(uint4 q1, uint64_t bits) {
  const uint64_t bloom = (uint64_t)q1.x | ((uint64_t)q1.y << 32);
  return (bloom & bits) == bits;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Streaming (non-temporal) 16-byte load: data read once, kept out of the
// caches that hold table lines.
__device__ __forceinline__ uint4 load_stream(const uint4 *p) {
  const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}

// Timers (Sec. 4.2): 16-bit times; an entry whose expiration time is e is
// alive at time `now` iff (e - now) mod 2^16 < 1024.
constexpr uint32_t kTimerShift = 48;
constexpr uint64_t kValueMask = (1ull << kTimerShift) - 1ull;
constexpr uint32_t kMaxDelay = 1024;

__device__ __forceinline__ bool word_alive(uint64_t word, uint32_t now) {
  return (((uint32_t)(word >> kTimerShift) - now) & 0xffffu) < kMaxDelay;
}

__device__ __forceinline__ bool key_eq(uint4 a, uint4 b) {
  return ((a.x ^ b.x) | (a.y ^ b.y) | (a.z ^ b.z) | (a.w ^ b.w)) == 0u;
}

}  // namespace ckpp
