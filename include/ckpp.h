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
 *   (implicit index, Sec. 4.3): key[16] | value u64 | reserved u64 (0; on
 *   a table with timers the entry's 16-bit expiration time).
 *
 * Hash (the paper uses CityHash64, Sec. 5): with the key read as
 * little-endian u64 halves lo and hi, h = f(f(lo ^ seed) ^ hi), where f is
 * the SplitMix64 output finalizer (Steele, Lea, Flood, OOPSLA 2014).
 * Primary bucket p = h mod 2^B and tag = h >> 48.  The alternate bucket and
 * the two bloom bits come from the secondary-hash field (Sec. 4.1):
 *   B <= 24: a = (h >> 24) mod 2^B; bloom bits (h >> 24) mod 64 and
 *            (h >> 30) mod 64;
 *   B >  24: that field would overlap p, so a second word
 *            g = f(h ^ 0xc2b2ae3d27d4eb4f) is used: a = g mod 2^B; bloom bits
 *            (g >> 32) mod 64 and (g >> 38) mod 64 (the constant is an
 *            arbitrary odd salt, the xxHash64 second prime);
 * and in both cases a = a xor 1 when a == p.
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
    CKPP_EBUSY = 4,   /* not admitted now (serving budget or queue full):
                         retry after completions */
    CKPP_ETIMEOUT = 5 /* a wait ran out of time */
};

/* Per-key insert status (written to d_status).  CKPP_RETRY is also the
 * per-key delete outcome of a delete that gave up (see ckpp_delete_batch). */
enum {
    CKPP_INSERTED = 0, /* the key was absent and now holds its value */
    CKPP_UPDATED = 1,  /* the key was present; its value was replaced */
    CKPP_FAILED = 2,   /* no cuckoo path within max_kicks (Sec. 2): the
                          table's key/value contents are unchanged */
    CKPP_RETRY = 3,    /* gave up after the table's retry limit of attempts
                          on bucket locks held by concurrent lanes of the
                          same batch (ckpp_set_retry_limit): nothing was
                          stored or changed for this key -- a present key
                          keeps its old value; the cuckoo moves made on
                          its behalf only relocated other entries.  The key
                          may be submitted again. */
};

/* Flags of ckpp_create. */
#define CKPP_PLAIN 1u /* plain (pessimistic) cuckoo table: no bloom filter or
                         moved counter is kept; lookups read both buckets
                         (the comparison baseline of Sec. 3) */
#define CKPP_TIMERS 2u /* table with timers (Sec. 4.2): every entry carries a
                          16-bit expiration time.  Device-layout limit: values
                          must be below 2^48 (see the timers section below).
                          Such a table is used through the *_at batch calls,
                          ckpp_plan_lookup_at, servers whose config sets a
                          ttl, and export/import, stats, clear and hash; the
                          untimed batch calls and ckpp_plan_lookup refuse it
                          (CKPP_EINVAL). */

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

/* Creates an empty table of 2^log2_buckets buckets (1 <= log2_buckets <= 29;
 * 256 bytes of device memory per bucket: 4 GiB at 2^24, 128 GiB at 2^29)
 * on HIP device `device` and stores its handle in *out.  hash_seed seeds the
 * hash; max_kicks bounds the displacements of one cuckoo path (Sec. 2);
 * flags: 0, CKPP_PLAIN and/or CKPP_TIMERS.  Errors: CKPP_EINVAL (out null, B out of range,
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
 * d_status (n bytes, nullable) receives CKPP_INSERTED / UPDATED / FAILED /
 * RETRY; d_nfailed (one u64, nullable) is incremented by the number of
 * FAILED keys (RETRY keys are counted in ckpp_stats_t.retry_exhausted).
 * The cuckoo-path scratch of the call (4 * max_kicks bytes per launched
 * lane, at most 2^16 lanes) is a buffer of the table's own, allocated on
 * the first batch that uses it and freed with the table; it holds as many
 * lanes as a launch uses, as long as that stays within 1/32 of the table's
 * device memory (at least 4096 lanes).  A batch needing more takes its
 * scratch from the device's stream-ordered memory pool and returns it on
 * `stream`.  Two insert batches of one table must therefore not overlap in
 * time (order them on one stream).
 * Errors: CKPP_EINVAL (null table/keys/values with n > 0, misaligned keys),
 * CKPP_ENOMEM (scratch allocation failed). */
int ckpp_insert_batch(ckpp_table *t, const void *d_keys, const uint64_t *d_values, uint64_t n,
                      uint8_t *d_status, uint64_t *d_nfailed, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the insert
 * of ckpp_insert_batch, same arguments, results and errors, that allocates
 * nothing.  Its cuckoo-path scratch is a fixed 8 MiB array in the library's
 * device memory, one per GPU, held until the process ends (instead of the
 * table's own buffer or the stream-ordered pool), so a launch uses at most
 * as many lanes as fit it: 8 MiB / (4 * max_kicks) lanes, in whole blocks
 * of 256 (4096 lanes at max_kicks 500; at least 256 for every max_kicks the
 * library accepts).  The array keeps the last call's contents; nothing in it
 * needs to start at zero (each lane writes its path before reading it).
 * Calls on one GPU share that array: two such calls that overlap in time
 * on the same GPU (on different streams, or from different threads) race
 * and corrupt each other's paths, so order them (one stream).  Not for
 * tables with timers.  Errors: as ckpp_insert_batch, CKPP_EINVAL also on a
 * table with timers, CKPP_EDEVICE if the array's address cannot be found. */
int ckpp_insert_batch_noalloc(ckpp_table *t, const void *d_keys, const uint64_t *d_values,
                              uint64_t n, uint8_t *d_status, uint64_t *d_nfailed, void *stream);

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
 * d_found (n bytes, nullable) receives 1 if the key was present (and is now
 * removed), 0 if it was absent, or CKPP_RETRY (3) if the delete gave up
 * after the table's retry limit of attempts on bucket locks held by
 * concurrent lanes: nothing was removed and the key may still be present.
 * When a key appears twice in one batch exactly one of its entries
 * reports 1. */
int ckpp_delete_batch(ckpp_table *t, const void *d_keys, uint64_t n, uint8_t *d_found,
                      void *stream);

/* ---- Timers (Sec. 4.2) -------------------------------------------------
 * On a table created with CKPP_TIMERS each entry has a 16-bit expiration
 * time in caller-chosen units; `now` is the current time in the same units,
 * modulo 2^16.  An entry with expiration time e is alive at `now` iff
 * (e - now) mod 2^16 < 1024: expiration times are set at most 1023 units
 * ahead, and an expired entry counts as absent.  Expired entries are deleted
 * lazily: an insert takes a slot holding one as if it were free (the slot's
 * entry is removed with the filter maintenance of a delete).  An expired
 * entry would look alive again 64512 units after it expired (the 16-bit
 * time wraps); ckpp_expire_scan removes every expired entry and must run at
 * least once every 64512 units.
 * Device-layout limit (a precondition of this library, not of the paper,
 * whose entries keep their times in separate 16-bit fields beside the tags,
 * Sec. 4.3): in device memory the time occupies the high 16 bits of the
 * entry's value word, so that a lookup reads it with the value (no extra
 * memory access), and values must be below 2^48.  An insert of a wider
 * value stores nothing and reports CKPP_FAILED for that key (a present key
 * keeps its old value and time); ckpp_import refuses an image with a wider
 * value in an occupied slot. */

/* Batched insert on a table with timers: as ckpp_insert_batch, where only
 * alive entries are present (an alive key is UPDATED; a key whose entry has
 * expired is overwritten in place and reported INSERTED), and key i's entry
 * gets expiration time d_expiry[i] (n u16, required; a time outside
 * [now, now + 1023] gives an entry that is not alive at `now`).  A value of
 * 2^48 or more is not stored: that key reports CKPP_FAILED.
 * Errors: as ckpp_insert_batch, and CKPP_EINVAL on a table without timers. */
int ckpp_insert_batch_at(ckpp_table *t, const void *d_keys, const uint64_t *d_values,
                         const uint16_t *d_expiry, uint64_t n, uint16_t now, uint8_t *d_status,
                         uint64_t *d_nfailed, void *stream);

/* Batched lookup on a table with timers: as ckpp_lookup_batch, where only
 * entries alive at `now` are found (values are the stored 48-bit values).
 * refresh = 1: every entry found gets expiration time `expiry` (Sec. 4.2: a
 * lookup may update it), which must lie in [now, now + 1023] mod 2^16 so
 * that the answers do not depend on the order of the batch's lookups; the
 * table is then written, so the batch must not run concurrently with other
 * lookups of the same table.  refresh = 0: nothing is written.
 * Errors: as ckpp_lookup_batch; CKPP_EINVAL on a table without timers,
 * refresh > 1, or a refresh time outside the window. */
int ckpp_lookup_batch_at(ckpp_table *t, const void *d_keys, uint64_t n, uint32_t mode,
                         uint16_t now, uint32_t refresh, uint16_t expiry, uint8_t *d_found,
                         uint64_t *d_values, void *stream);

/* Batched delete on a table with timers: as ckpp_delete_batch; an expired
 * entry of the key is removed too but reports 0 (only alive keys are found).
 * Errors: as ckpp_delete_batch, and CKPP_EINVAL on a table without timers. */
int ckpp_delete_batch_at(ckpp_table *t, const void *d_keys, uint64_t n, uint16_t now,
                         uint8_t *d_found, void *stream);

/* Anti-revival scan (Sec. 4.2): removes every entry expired at `now`, with
 * the filter maintenance of a delete (moved counters of the primaries of
 * removed displaced entries decrease; filters whose counter reaches zero are
 * emptied).  *d_removed (one u64, nullable) is incremented by the number of
 * entries removed.  Reads the whole table once (one kernel).
 * Errors: CKPP_EINVAL (table without timers, misaligned d_removed). */
int ckpp_expire_scan(ckpp_table *t, uint16_t now, uint64_t *d_removed, void *stream);

/* Copies the table image to host memory (h_buckets: 64 * 2^B bytes, h_kv:
 * 256 * 2^B bytes; either may be null to skip it) after the stream's earlier
 * work; returns when the copy is complete. */
int ckpp_export(const ckpp_table *t, void *h_buckets, void *h_kv, void *stream);

/* Replaces the table's contents with an image (same sizes and layout as
 * ckpp_export; both pointers required); returns when the copy is complete.
 * The image must satisfy the table's invariants (each entry in one of its
 * two buckets with its tag and other bucket, exact moved counters, no
 * filter false negative, zero locks); lookups on any other image are
 * unspecified.  An image that fails ckpp_check_image is refused with
 * CKPP_EINVAL and the table is unchanged.  On a table with timers a free
 * slot's record keeps only the low 48 bits of its value (free records are
 * never read). */
int ckpp_import(ckpp_table *t, const void *h_buckets, const void *h_kv, void *stream);

/* Host-only check of an image for a table of 2^log2_buckets buckets with
 * the given create flags (no device is used): CKPP_OK when every lock word
 * is zero, every sec mask lies within its busy mask, every occupied slot's
 * other bucket is below 2^log2_buckets (so that inserts, deletes and the
 * scan, which follow other[], stay inside the table) and, with
 * CKPP_TIMERS, every occupied slot's value is below 2^48 and its reserved
 * word below 2^16 (the device layout's limit); else CKPP_EINVAL.  This is
 * the check ckpp_import applies; it does not verify the remaining
 * invariants.  Sizes as in ckpp_export. */
int ckpp_check_image(uint32_t log2_buckets, uint32_t flags, const void *h_buckets,
                     const void *h_kv);

/* Table statistics (Sec. 3 entries in secondary; Sec. 4.1 moved counters;
 * Sec. 5.3 filter false-positive rate).  The rate a uniformly random absent
 * key passes bucket b's filter is (popcount(bloom_b)/64)^2, so the mean rate
 * is bloom_pc2_sum / (4096 * nbuckets).  Slots 4..7 of a bucket sit in its
 * second 128-byte line: a lookup of a key stored there reads two lines of
 * that bucket. */
#define CKPP_MOVED_BINS 66 /* moved counter values 0..64, then "> 64" */
typedef struct {
    uint64_t nbuckets;
    uint64_t live;          /* occupied slots (with timers: expired entries
                               not yet reused or scanned count too) */
    uint64_t in_secondary;  /* entries stored in their secondary bucket */
    uint64_t bloom_pc_sum;  /* sum of popcount(bloom) over buckets */
    uint64_t bloom_pc2_sum; /* sum of popcount(bloom)^2 over buckets */
    uint64_t locked;        /* buckets whose lock word is non-zero */
    uint64_t high_slots;    /* occupied slots 4..7 */
    uint64_t high_slots_secondary; /* of which entries in their secondary */
    uint64_t retry_exhausted; /* keys of earlier insert/delete batches (and
                                 served bursts) that gave up after the retry
                                 limit on contended locks: each reported
                                 CKPP_RETRY */
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

/* Launch shape of the lookup kernel.  lanes_per_lookup 8: each lane owns
 * one lookup; the line of a bucket is read by a group of 8 neighbouring
 * lanes (16 bytes each, one 128-byte request) straight into LDS, and each
 * lane then analyses its own line there; lookups_per_lane 1, or 2 (each
 * lane owns two lookups; the lines of the second half land in registers
 * and are parked in LDS after the first half is analysed: twice the
 * requests in flight; the pessimistic mode always uses 1).
 * lanes_per_lookup 4: each lane owns one lookup; a quad of 4 neighbouring
 * lanes reads each of its four lookups' lines into registers (32 bytes per
 * lane, one request per line) and analyses the line there, the lanes
 * exchanging keys and answers through DPP; lookups_per_lane 1 or 2 (a
 * quad then holds the lines of eight lookups); no LDS.
 * lanes_per_lookup 1: each lane reads the 32-byte head of its own bucket
 * (tags, filter, masks) into registers, and a candidate's key and value
 * only on a tag match; lookups_per_lane 1, 2 or 4; no LDS.
 * block: 64, 128 or 256 (1, 2 or 4 wavefronts; with 8 lanes, 8 KiB of LDS
 * each, 16 KiB for the pessimistic mode); blocks_per_cu: grid size in
 * blocks per compute unit (0: enough blocks to cover the batch in one
 * pass).  Applies to every later lookup on t.  A new table starts with
 * {8, 2, 128, 0}, the fastest shape on 2^20..2^24-bucket tables at load
 * 0.9; until a shape is set, batches of at most 4096 lookups run as
 * {1, 1, 64, blocks_per_cu} instead, which completes small batches
 * soonest.  Errors: CKPP_EINVAL (a shape outside these sets). */
typedef struct {
    uint32_t lanes_per_lookup;
    uint32_t lookups_per_lane;
    uint32_t block;
    uint32_t blocks_per_cu;
} ckpp_launch_t;

int ckpp_set_lookup_launch(ckpp_table *t, const ckpp_launch_t *cfg);
int ckpp_get_lookup_launch(const ckpp_table *t, ckpp_launch_t *cfg);

/* Retry limit of inserts and deletes (this library's bound; the paper's
 * table has one writer per core, Sec. 2, and never meets a held lock): the
 * number of attempts one key makes on bucket locks that other lanes of its
 * batch (or of its serving round) hold before it gives up with CKPP_RETRY.
 * Locks are never waited on, so every attempt ends.  1 <= limit <= 2^20;
 * a new table starts at 2^20, where no test or workload of this library has
 * reached it.  Applies to later batches and to servers created afterwards.
 * Errors: CKPP_EINVAL (null table, limit out of range). */
int ckpp_set_retry_limit(ckpp_table *t, uint32_t limit);
int ckpp_get_retry_limit(const ckpp_table *t, uint32_t *limit);

/* ---- Many tables, one launch -------------------------------------------
 * A plan serves the lookup batches of many tables (each one a Sec. 2 /
 * Sec. 4.1 lookup batch, exactly as ckpp_lookup_batch computes it) in a
 * single launch of a persistent kernel: the batches are cut into work items
 * of at most passes_per_item * 64 * lookups_per_lane lookups of one table,
 * and each wavefront takes the next item from a device counter until none
 * is left.  The grouping is this library's scheduling, not the paper's; the
 * results are those of one ckpp_lookup_batch call per table. */
typedef struct ckpp_plan ckpp_plan;

/* Launch shape of a plan's kernel.  lookups_per_lane: 1 or 2 with
 * lanes_per_lookup 8 or 4, 1, 2 or 4 with lanes_per_lookup 1 (as in
 * ckpp_launch_t); block: 64, 128 or 256; blocks_per_cu: 1..64, the
 * persistent grid is blocks_per_cu blocks per compute unit (at most one
 * wavefront per work item); passes_per_item: 1..64; schedule:
 * CKPP_PLAN_STATIC (wavefront w runs items w, w + W, ... for W wavefronts)
 * or CKPP_PLAN_DYNAMIC (each wavefront takes the next item from a device
 * counter); lanes_per_lookup: 8 (a bucket line read by 8 lanes into LDS),
 * 4 (a line read into a quad's registers) or 1 (each lane reads its
 * bucket's head into registers). */
enum { CKPP_PLAN_STATIC = 0, CKPP_PLAN_DYNAMIC = 1 };

typedef struct {
    uint32_t lookups_per_lane;
    uint32_t block;
    uint32_t blocks_per_cu;
    uint32_t passes_per_item;
    uint32_t schedule;
    uint32_t lanes_per_lookup;
} ckpp_plan_launch_t;

typedef struct {
    uint32_t ntables;
    uint32_t nitems;       /* work items under the current launch shape */
    uint64_t lookups;      /* sum of the batch sizes */
    uint64_t key_span;     /* max over tables of offset + count */
} ckpp_plan_info_t;

/* Builds a plan over ntables >= 1 tables, all on one device: table i's
 * batch is keys [h_offsets[i], h_offsets[i] + h_counts[i]) of the key
 * array later passed to ckpp_plan_lookup, and its results go to the same
 * positions of the output arrays; the ranges must not overlap (a count may
 * be 0).  h_modes (nullable: all CKPP_LOOKUP_DEFAULT) gives each table's
 * lookup mode; CKPP_LOOKUP_DEFAULT on a plain table is CKPP_LOOKUP_BOTH.
 * Tables with timers may take part: such a plan is run with
 * ckpp_plan_lookup_at.
 * The plan keeps the tables' device addresses, not the tables: it must be
 * destroyed before any of them, and inserts and deletes between plan
 * lookups are seen by the next one.  Host arrays are read during the call
 * only.  Starts with the launch shape {1, 128, 8, 1, CKPP_PLAN_STATIC, 8}.
 * Errors: CKPP_EINVAL (null arguments, ntables 0, overlapping ranges, bad
 * mode, tables on different devices), CKPP_ENOMEM, CKPP_EDEVICE. */
int ckpp_plan_create(ckpp_plan **out, ckpp_table *const *tables, uint32_t ntables,
                     const uint64_t *h_offsets, const uint64_t *h_counts,
                     const uint32_t *h_modes);

/* Frees the plan after its device is idle.  A null plan is a no-op. */
int ckpp_plan_destroy(ckpp_plan *p);

/* Runs every table's batch: d_keys holds key_span 16-byte keys (16-byte
 * aligned), d_found key_span bytes and d_values key_span u64 (8-byte
 * aligned); positions outside every range are neither read nor written.
 * One kernel launch on `stream`, no allocation, no memory set: the call may
 * be captured in a HIP graph.  The dynamic schedule's work counter lives in
 * the plan's device memory, so two launches of one plan must not overlap in
 * time (order them on one stream).  Must not run concurrently with inserts or deletes on its
 * tables.  Errors: CKPP_EINVAL (null or misaligned pointers, a plan with a
 * table with timers). */
int ckpp_plan_lookup(ckpp_plan *p, const void *d_keys, uint8_t *d_found, uint64_t *d_values,
                     void *stream);

/* As ckpp_plan_lookup for a plan with tables with timers (Sec. 4.2): each
 * such table's batch is that of ckpp_lookup_batch_at(table, ..., now,
 * refresh, expiry); the other tables' batches are as in ckpp_plan_lookup.
 * With refresh = 1 the tables with timers are written (the launch must not
 * run concurrently with other lookups of them), and expiry must lie in
 * [now, now + 1023] mod 2^16.  Errors: as ckpp_plan_lookup; CKPP_EINVAL on
 * a plan without a table with timers, refresh > 1, or a refresh time outside
 * the window. */
int ckpp_plan_lookup_at(ckpp_plan *p, const void *d_keys, uint8_t *d_found, uint64_t *d_values,
                        uint16_t now, uint32_t refresh, uint16_t expiry, void *stream);

/* Sets the launch shape (rebuilds the work items: synchronizes the device,
 * not for use under graph capture).  The work items move to new device
 * memory, so a HIP graph captured from an earlier ckpp_plan_lookup of this
 * plan must not be launched afterwards (capture it again).
 * Errors: CKPP_EINVAL (out of range). */
int ckpp_plan_set_launch(ckpp_plan *p, const ckpp_plan_launch_t *cfg);
int ckpp_plan_get_launch(const ckpp_plan *p, ckpp_plan_launch_t *cfg);
int ckpp_plan_info(const ckpp_plan *p, ckpp_plan_info_t *out);

/* ---- Serving: a device-resident request loop --------------------------
 * A server runs one persistent kernel over a table that stays in device
 * memory.  Producers place the operations of a burst in three device rings
 * (lookups: 16-byte keys; inserts: keys and u64 values; deletes: keys) at
 * the positions following the previous burst's, then submit the burst's
 * three counts.  The loop gathers every burst submitted before it starts a
 * round (continuous batching: bursts that arrive while a round runs join
 * the next one) and runs the round's lookups, then its inserts and
 * deletes, each phase over all of the round's bursts at once, with grid-wide
 * barriers between the phases; rounds run in submission order.  Inserts and
 * deletes of different keys run side by side; the deletes of keys that the
 * round also inserts run after all of its inserts (so a burst that inserts
 * and deletes a key ends without it).  So a lookup sees every insert and
 * delete of the bursts of earlier rounds and none of its own round's, and a
 * burst's results do not depend on which other bursts share its round as
 * long as their writes concern other keys (an insert may take a slot that a
 * delete of the same round frees, which only matters when the table is
 * full).  Each
 * operation is the Sec. 2 / Sec. 4.1 operation of ckpp_lookup_batch,
 * ckpp_insert_batch or ckpp_delete_batch (on a table with timers, that of
 * the _at call at its burst's time: see ckpp_server_set_time and the ttl of
 * the config); results land in the rings at the operation's position.  Admission: a burst is accepted only while the
 * operations submitted and not completed stay within the budget of each
 * ring (and fewer than 4096 bursts are in flight); otherwise CKPP_EBUSY.
 * Ring position of operation number i of a kind: i mod capacity.
 * When no burst arrives for idle_ms the kernel exits; the next submit
 * relaunches it.  The calls on one server share its submission state: make
 * them from one host thread at a time. */
typedef struct ckpp_server ckpp_server;

typedef struct {
    uint64_t capacity;      /* slots of each ring: a power of two, 2^6..2^30 */
    uint64_t budget;        /* ops of one kind in flight at most (<= capacity) */
    uint32_t mode;          /* lookup mode, CKPP_LOOKUP_* (DEFAULT: Cuckoo++,
                               both buckets on a plain table) */
    uint32_t blocks_per_cu; /* persistent grid: 1..4 blocks of 512 threads
                               per compute unit, capped at the number that
                               can be co-resident (one on gfx950) */
    uint32_t idle_ms;       /* 1..60000 */
    uint32_t ttl;           /* table without timers: 0.  Table with timers:
                               the lifetime of entries, 1..1023 time units
                               (an insert at time now gives its entry
                               expiration time now + ttl), or-ed with
                               CKPP_SERVER_REFRESH to have every lookup that
                               finds an entry set its expiration time to
                               now + ttl as well (Sec. 4.2) */
} ckpp_server_config_t;

#define CKPP_SERVER_REFRESH (1u << 16)

/* Device rings owned by the server (freed by ckpp_server_destroy). */
typedef struct {
    void *d_lookup_keys;        /* capacity x 16 bytes */
    uint8_t *d_lookup_found;    /* capacity bytes */
    uint64_t *d_lookup_values;  /* capacity u64 */
    void *d_insert_keys;        /* capacity x 16 bytes */
    uint64_t *d_insert_values;  /* capacity u64 */
    uint8_t *d_insert_status;   /* capacity bytes (CKPP_INSERTED/UPDATED/FAILED/RETRY) */
    void *d_delete_keys;        /* capacity x 16 bytes */
    uint8_t *d_delete_found;    /* capacity bytes (0, 1 or CKPP_RETRY, as in
                                   ckpp_delete_batch) */
    uint64_t capacity;
} ckpp_server_rings_t;

enum {
    CKPP_SERVER_STOPPED = 0, /* no loop kernel running */
    CKPP_SERVER_RUNNING = 1,
    CKPP_SERVER_EXITING = 2, /* the loop is deciding to exit for idleness */
    CKPP_SERVER_ABORTED = 3  /* a grid barrier ran out of time: the loop
                                stopped; the server is unusable */
};

typedef struct {
    uint64_t submitted;   /* bursts */
    uint64_t completed;   /* bursts whose results are in the rings */
    uint64_t lookup_tail, insert_tail, delete_tail; /* ops submitted per kind */
    uint64_t rounds;      /* rounds the loop ran */
    uint64_t launches;    /* loop kernel launches (1 + restarts) */
    uint32_t state;       /* CKPP_SERVER_* */
    uint32_t grid;        /* blocks of the loop kernel */
    /* the loop's own clock, summed over rounds, as of the last round
       boundary: from the release of each phase until every block finished
       it (insert_ns: the inserts, or inserts and deletes side by side;
       delete_ns: deletes after the inserts); at round boundaries apart from
       waiting; waiting for bursts */
    uint64_t lookup_ns, insert_ns, delete_ns, boundary_ns, wait_ns;
} ckpp_server_status_t;

/* Creates a server on table t (the table must not be used by other calls
 * while the server exists) and launches its loop.
 * Errors: CKPP_EINVAL (bad config: a ttl out of range for the table's kind
 * among others), CKPP_ENOMEM, CKPP_EDEVICE. */
int ckpp_server_create(ckpp_server **out, ckpp_table *t, const ckpp_server_config_t *cfg);

int ckpp_server_rings(const ckpp_server *s, ckpp_server_rings_t *out);

/* Kinds of operations (ring selectors). */
enum { CKPP_OP_LOOKUP = 0, CKPP_OP_INSERT = 1, CKPP_OP_DELETE = 2 };

/* Copies n operations of one kind from the caller's device buffers into the
 * ring slots of operation numbers pos .. pos + n - 1 (slot = number mod
 * capacity), ordered on `stream` (device-to-device copies; the caller
 * synchronizes before submitting).  d_values: the insert values (inserts
 * only, else null).  Errors: CKPP_EINVAL (n > capacity, null pointers). */
int ckpp_server_put(ckpp_server *s, uint32_t kind, uint64_t pos, const void *d_keys,
                    const uint64_t *d_values, uint32_t n, void *stream);

/* Copies the results of operations pos .. pos + n - 1 of one kind out of the
 * rings, ordered on `stream`: lookups -> d_flags (found) and d_values;
 * inserts -> d_flags (status); deletes -> d_flags (found).  Valid once the
 * operations' bursts are complete and before their slots are reused. */
int ckpp_server_get(ckpp_server *s, uint32_t kind, uint64_t pos, uint32_t n, uint8_t *d_flags,
                    uint64_t *d_values, void *stream);

/* Submits the next burst: its ops are at ring positions tail .. tail + n - 1
 * (mod capacity) of each kind, tail as ckpp_server_status reports before the
 * call, already written (and the writes complete) by the caller.  *burst
 * (nullable) receives the burst's number.  Errors: CKPP_EBUSY (over the
 * budget or too many bursts in flight: nothing was submitted),
 * CKPP_EDEVICE (the loop aborted or could not be relaunched). */
int ckpp_server_submit(ckpp_server *s, uint32_t n_lookup, uint32_t n_insert, uint32_t n_delete,
                       uint64_t *burst);

int ckpp_server_status(ckpp_server *s, ckpp_server_status_t *out);

/* Waits until bursts 0..burst are complete.  Errors: CKPP_ETIMEOUT,
 * CKPP_EDEVICE (the loop aborted). */
int ckpp_server_wait(ckpp_server *s, uint64_t burst, uint32_t timeout_ms);

/* Servers on tables with timers (Sec. 4.2): sets the time (as in
 * ckpp_lookup_batch_at, modulo 2^16) of the bursts submitted after this
 * call; every operation of a burst runs at its burst's time (a round takes
 * bursts of one time only).  The time starts at 0; the first call may set
 * any time, each later one must advance it by less than 16384 units
 * ((now - previous) mod 2^16 < 16384; the same time is a no-op).  The
 * server runs the anti-revival scan of ckpp_expire_scan itself, as the
 * first phase of a round at the new time, on the first call and whenever
 * the time has advanced 16384 units or more since its last scan: the call
 * then submits an empty burst for it (so it may return CKPP_EBUSY when 4096
 * bursts are in flight; nothing changes then).  As for the batch calls, no
 * entry of the table may have expired 64512 units or more before the first
 * time set (the scan keeps that true afterwards).
 * Errors: CKPP_EINVAL (null, a server without timers, a step of 16384 or
 * more), CKPP_EBUSY, CKPP_EDEVICE. */
int ckpp_server_set_time(ckpp_server *s, uint16_t now);

/* Open-loop replay (measurement): submits burst i of a pre-staged stream at
 * h_arrival_s[i] seconds after the call (later if the budget does not admit
 * it yet, in order), and records when it was admitted and when the host saw
 * it complete, in seconds after the call (h_admit_s, h_done_s: nbursts
 * each).  The stream's ops must already be in the rings at the positions
 * the bursts will take.  On a server with timers every burst runs at the
 * time set before the call.  Errors: CKPP_ETIMEOUT (not all done within
 * timeout_s), CKPP_EDEVICE. */
int ckpp_server_replay(ckpp_server *s, uint64_t nbursts, const uint32_t *h_nlookup,
                       const uint32_t *h_ninsert, const uint32_t *h_ndelete,
                       const double *h_arrival_s, double *h_admit_s, double *h_done_s,
                       double timeout_s);

/* Stops the loop (after the bursts already submitted complete), frees the
 * server.  A null server is a no-op. */
int ckpp_server_destroy(ckpp_server *s);

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

/* Measurement kernel for the latency of the insert and delete paths: one
 * lane makes `steps` dependent accesses to 128-byte lines chosen by a
 * hash of the previous access's value (so none can start before the one
 * before it ends), in d_buf (`bytes` long, a multiple of 256, 256-byte
 * aligned).  kind 0: plain load; 1: relaxed agent-scope atomic load; 2:
 * relaxed agent-scope compare-and-swap (expects 1, writes 1: it changes no
 * word); 3: atomic load, the same value stored back with an atomic store,
 * and a wait for the store to complete; 4: two compare-and-swaps of kind 2
 * on lines half the buffer apart, issued together; 5: 32 plain loads of
 * different lines, all issued before the first is waited for (the next
 * step's lines depend on all 32 values); 6: the same with relaxed
 * agent-scope atomic loads.  The buffer's contents are not changed.  d_out[0] receives the elapsed real-time counter ticks (100 MHz:
 * 10 ns each), d_out[1] a fold of the values read.  The caller times
 * nothing: ticks / steps is the latency of one step.  Errors: CKPP_EINVAL
 * (null or misaligned pointers, a size or kind out of range, steps 0). */
int ckpp_probe_latency(void *d_buf, uint64_t bytes, uint32_t kind, uint32_t steps, uint64_t seed,
                       uint64_t *d_out, void *stream);

/* Human-readable name of a status code. */
const char *ckpp_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* CKPP_H */
