/*
 * ckpp.h -- C ABI of the MI355X (gfx950) Cuckoo++ hash table library.
 *
 * N. Le Scouarnec, "Cuckoo++ Hash Tables: High-Performance Hash Tables for
 * Networking Applications", arXiv 1712.09624 (2017).
 *
 * A table is a bucketized two-choice cuckoo hash table (Sec. 2) of 2^B
 * buckets x 8 slots, mapping 16-byte keys (network 5-tuples, Sec. 1) to
 * 64-bit values, with the Cuckoo++ change (Sec. 4.1): each bucket carries a
 * 64-bit bloom filter of the keys that were displaced from it to their
 * secondary bucket, and a moved counter that resets the filter when it
 * returns to zero, so that most negative lookups read a single bucket.
 *
 * Conventions shared by every call:
 *  - Pointers named d_* are device pointers on the table's device; h_*
 *    are host pointers.  The caller owns every buffer it passes; the
 *    library keeps no reference to them after the stream reaches the call.
 *  - Keys are n x 16 bytes, contiguous, 16-byte aligned.  Values are u64.
 *  - `stream` is a hipStream_t (NULL: the device's null stream).  Batch
 *    calls only enqueue work and return; results are valid once the stream
 *    reaches them.  Batches on one table are ordered by their stream; a
 *    caller using several streams serializes them itself.
 *  - Every call validates its arguments first and returns CKPP_OK or an
 *    error code without enqueueing anything; n == 0 is a no-op returning
 *    CKPP_OK.  A failed kernel launch returns CKPP_EDEVICE.
 *  - The table's device memory is owned by the library: 256 * 2^B bytes
 *    (32 bytes per slot: bucket b holds its metadata and the keys and values
 *    of its 8 slots in two 128-byte lines), plus a small working area.
 *
 * Image layout (the interchange format of export/import, independent of the
 * device layout; fixed, little-endian):
 *   bucket b, 64 bytes at offset 64*b (one cache line, Sec. 4.3):
 *     0..15  tag[8]   u16  16-bit tag of each slot, from the key's hash
 *     16..23 bloom    u64  bloom filter of keys displaced from b (Sec. 4.1)
 *     24..25 moved    u16  moved counter of the filter (Sec. 4.1)
 *     26     busy     u8   bit s: slot s holds an entry
 *     27     sec      u8   bit s: that entry sits in its secondary bucket
 *     28..31 lock     u32  zero whenever no batch is running
 *     32..63 other[8] u32  the other bucket of each slot's entry (Sec. 4.3)
 *   key/value record of slot s of bucket b, 32 bytes at offset 32*(8*b+s)
 *   (implicit index, Sec. 4.3): key[16] | value u64 | reserved u64 (0).
 *
 * Hash (the paper uses CityHash64, Sec. 5): with the key read as
 * little-endian u64 halves lo and hi, h = f(f(lo ^ seed) ^ hi), where f is
 * the SplitMix64 output finalizer (Steele, Lea, Flood, OOPSLA 2014).
 * Primary bucket p = h mod 2^B; alternate a = (h >> 24) mod 2^B, xor 1 if
 * equal to p; tag = h >> 48; bloom bits (h >> 24) mod 64 and (h >> 30) mod
 * 64, two values from the secondary-hash field (Sec. 4.1).
 */
#ifndef CKPP_H
#define CKPP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ckpp_table ckpp_table;

/* Call status. */
enum {
    CKPP_OK = 0,
    CKPP_EINVAL = 1,  /* bad argument: null, misaligned, out of range */
    CKPP_ENOMEM = 2,  /* device allocation failed */
    CKPP_EDEVICE = 3, /* HIP runtime error (launch, copy, device) */
};

/* Per-key insert status (written to d_status). */
enum {
    CKPP_INSERTED = 0, /* the key was absent and now holds its value */
    CKPP_UPDATED = 1,  /* the key was present; its value was replaced */
    CKPP_FAILED = 2,   /* no cuckoo path within max_kicks (or the retry
                          bound on contended locks was reached): the
                          table's key/value contents are unchanged */
};

/* Flags of ckpp_create. */
#define CKPP_PLAIN 1u /* plain (pessimistic) cuckoo table: no bloom filter or
                         moved counter is kept; lookups read both buckets
                         (the comparison baseline of Sec. 3) */

/* Lookup modes (Sec. 3 and Sec. 4.1).  All modes give the same answers. */
enum {
    CKPP_LOOKUP_DEFAULT = 0,    /* Cuckoo++: the secondary bucket is read only
                                   when the key is not in the primary and the
                                   primary's bloom filter passes; on a plain
                                   table this is CKPP_LOOKUP_BOTH */
    CKPP_LOOKUP_BOTH = 1,       /* pessimistic: both buckets always fetched */
    CKPP_LOOKUP_OPTIMISTIC = 2, /* primary, then the secondary whenever the
                                   key is not in the primary (no filter) */
};

/* Creates an empty table of 2^log2_buckets buckets (1 <= log2_buckets <= 24)
 * on HIP device `device` and stores its handle in *out.  hash_seed seeds the
 * hash; max_kicks bounds the displacements of one cuckoo path (Sec. 2);
 * flags is 0 or CKPP_PLAIN.  Errors: CKPP_EINVAL (out null, B out of range,
 * unknown flag, bad device), CKPP_ENOMEM, CKPP_EDEVICE. */
int ckpp_create(ckpp_table **out, uint32_t log2_buckets, uint64_t hash_seed, uint32_t max_kicks,
                uint32_t flags, int device);

/* Frees the table and its device memory after its device is idle.
 * A null table is a no-op. */
int ckpp_destroy(ckpp_table *t);

/* Empties the table (all buckets and records zeroed), ordered on stream. */
int ckpp_clear(ckpp_table *t, void *stream);

/* Batched insert (Sec. 2, insertion; Sec. 4.1, filter maintenance): for each
 * key i, an existing key gets value d_values[i] (UPDATED); otherwise it goes
 * to a free slot of its primary bucket, else of its secondary bucket (its
 * bits are then set in the primary's filter and the primary's moved counter
 * is incremented), else a cuckoo path of at most max_kicks displacements
 * frees a slot (moves from primary to secondary add to the filter, moves
 * back subtract from the counter and reset the filter at zero).  Keys of one
 * batch must be pairwise distinct (the result is unspecified otherwise).
 * d_status (n bytes, nullable) receives CKPP_INSERTED / UPDATED / FAILED;
 * d_nfailed (one u64, nullable) is incremented by the number of FAILED keys.
 * The cuckoo-path scratch of the call (at most 4 * max_kicks bytes per
 * launched lane, at most 2^16 lanes) comes from the device's stream-ordered
 * memory pool and is returned to it on `stream`.
 * Errors: CKPP_EINVAL (null table/keys/values with n > 0, misaligned keys),
 * CKPP_ENOMEM (scratch allocation failed). */
int ckpp_insert_batch(ckpp_table *t, const void *d_keys, const uint64_t *d_values, uint64_t n,
                      uint8_t *d_status, uint64_t *d_nfailed, void *stream);

/* Batched lookup (Sec. 2, lookup; Sec. 4.1, pruning): d_found[i] = 1 and
 * d_values[i] = the key's value if key i is in the table, else 0 and 0.
 * mode is one of CKPP_LOOKUP_*.  d_found (n bytes) and d_values (n u64)
 * must not overlap the keys.  Must not run concurrently with an insert or
 * delete batch on the same table.
 * Errors: CKPP_EINVAL (null pointers with n > 0, misaligned, bad mode). */
int ckpp_lookup_batch(ckpp_table *t, const void *d_keys, uint64_t n, uint32_t mode,
                      uint8_t *d_found, uint64_t *d_values, void *stream);

/* Batched delete (Sec. 4.1, deletion): each present key is removed; if it
 * sat in its secondary bucket the moved counter of its primary is
 * decremented and the primary's filter reset when it reaches zero.
 * d_found (n bytes, nullable) receives 1 if the key was present.  When a key
 * appears twice in one batch exactly one of its entries reports 1. */
int ckpp_delete_batch(ckpp_table *t, const void *d_keys, uint64_t n, uint8_t *d_found,
                      void *stream);

/* Copies the table image to host memory (h_buckets: 64 * 2^B bytes, h_kv:
 * 256 * 2^B bytes; either may be null to skip it) after the stream's earlier
 * work; returns when the copy is complete. */
int ckpp_export(const ckpp_table *t, void *h_buckets, void *h_kv, void *stream);

/* Replaces the table's contents with an image (same sizes and layout as
 * ckpp_export; both pointers required); returns when the copy is complete.
 * The image must satisfy the table's invariants (each entry in one of its
 * two buckets with its tag and other bucket, exact moved counters, no
 * filter false negative, zero locks); lookups on any other image are
 * unspecified. */
int ckpp_import(ckpp_table *t, const void *h_buckets, const void *h_kv, void *stream);

/* Table statistics (Sec. 3 entries in secondary; Sec. 4.1 moved counters;
 * Sec. 5.3 filter false-positive rate).  The rate a uniformly random absent
 * key passes bucket b's filter is (popcount(bloom_b)/64)^2, so the mean rate
 * is bloom_pc2_sum / (4096 * nbuckets).  Slots 4..7 of a bucket sit in its
 * second 128-byte line: a lookup of a key stored there reads two lines of
 * that bucket. */
#define CKPP_MOVED_BINS 66 /* moved counter values 0..64, then "> 64" */
typedef struct {
    uint64_t nbuckets;
    uint64_t live;          /* occupied slots */
    uint64_t in_secondary;  /* entries stored in their secondary bucket */
    uint64_t bloom_pc_sum;  /* sum of popcount(bloom) over buckets */
    uint64_t bloom_pc2_sum; /* sum of popcount(bloom)^2 over buckets */
    uint64_t locked;        /* buckets whose lock word is non-zero */
    uint64_t high_slots;    /* occupied slots 4..7 */
    uint64_t high_slots_secondary; /* of which entries in their secondary */
    uint64_t retry_exhausted; /* keys of earlier insert/delete batches that
                                 gave up after the retry bound on contended
                                 locks (reported FAILED / not found) */
    uint64_t moved_hist[CKPP_MOVED_BINS];
} ckpp_stats_t;

/* Fills *h_out after the stream's earlier work; returns when done. */
int ckpp_stats(const ckpp_table *t, ckpp_stats_t *h_out, void *stream);

/* d_hash[i] = the table's 64-bit hash of key i (see the hash above). */
int ckpp_hash_batch(const ckpp_table *t, const void *d_keys, uint64_t n, uint64_t *d_hash,
                    void *stream);

/* Description of a table. */
typedef struct {
    uint32_t log2_buckets;
    uint32_t max_kicks;
    uint32_t flags;
    int device;
    uint64_t hash_seed;
    uint64_t image_bucket_bytes; /* sizes of the export/import arrays */
    uint64_t image_kv_bytes;
    uint64_t device_bytes;       /* device memory of the table */
    void *d_table;               /* device address of the table */
} ckpp_info_t;

int ckpp_info(const ckpp_table *t, ckpp_info_t *out);

/* Launch shape of the lookup kernel.  Each lane owns one lookup; the line
 * of a bucket is read by a group of lanes_per_lookup = 8 neighbouring lanes
 * (16 bytes each, one 128-byte request) straight into LDS, and each lane
 * then analyses its own line there.  lookups_per_lane: 1, or 2 (each lane
 * owns two lookups; the lines of the second half land in registers and are
 * parked in LDS after the first half is analysed: twice the requests in
 * flight; the pessimistic mode always uses 1); block: 64, 128 or 256 (1, 2
 * or 4 wavefronts, 8 KiB of LDS each, 16 KiB for the pessimistic mode);
 * blocks_per_cu: grid size in blocks per compute unit (0: enough blocks to
 * cover the batch in one pass).  Applies to every later lookup on t.  A new
 * table starts with {8, 2, 128, 0}, the fastest shape on 2^20..2^24-bucket
 * tables at load 0.9. */
typedef struct {
    uint32_t lanes_per_lookup;
    uint32_t lookups_per_lane;
    uint32_t block;
    uint32_t blocks_per_cu;
} ckpp_launch_t;

int ckpp_set_lookup_launch(ckpp_table *t, const ckpp_launch_t *cfg);
int ckpp_get_lookup_launch(const ckpp_table *t, ckpp_launch_t *cfg);

/* Measurement kernel for the roofline of the lookups: reads `nreads`
 * granules of `granule` bytes (16, 32, 64 or 128, aligned) at uniformly
 * random positions of the device buffer d_buf (`bytes` long, a multiple of
 * the granule) and folds the data into d_sink (one u64 per launched lane:
 * grid * block entries).  per_lane (1, 2, 4, 8) granules are kept in flight
 * per lane (or lane group).  cooperative = 0: each lane reads whole
 * granules with 16-byte loads; cooperative = 1: granule/16 neighbouring
 * lanes read one granule together, one 16-byte piece each (one coalesced
 * request per granule).  block: 64, 128 or 256.  The caller times it;
 * nreads / time is the random-access rate. */
int ckpp_probe_random_reads(const void *d_buf, uint64_t bytes, uint32_t granule, uint64_t nreads,
                            uint32_t per_lane, uint32_t cooperative, uint32_t block, uint32_t grid,
                            uint64_t seed, uint64_t *d_sink, void *stream);

/* Human-readable name of a status code. */
const char *ckpp_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* CKPP_H */
