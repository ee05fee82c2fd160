/*
 * ckpp_oracle.c -- reference oracle for the Cuckoo++ hash table.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, single-threaded
 * CPU definition that the GPU library is checked against.  Only the test
 * suite, the package smoke check and the CPU-baseline leg of the benchmark
 * may load it.  The product library never links, loads or calls it, and it
 * shares no code, header or constant table with the GPU library: both are
 * written independently from the paper.
 *
 * Paper: N. Le Scouarnec, "Cuckoo++ Hash Tables: High-Performance Hash Tables
 * for Networking Applications", arXiv 1712.09624 (2017).
 *
 * What the table computes is a dictionary from 16-byte keys to 64-bit values
 * (Sec. 2, Sec. 4).  The oracle nevertheless is a real bucketized two-choice
 * cuckoo table with 8 slots per bucket (Sec. 2, Sec. 4.3), because its
 * statistics (entries in secondary, moved counters, bloom occupancy), its
 * per-lookup memory-line counts and its table image are needed by the tests.
 *
 * Readings taken where the paper is silent (each is listed in the design
 * notes of the repository):
 *   - hash: a seeded 64-bit mixer of the four little-endian key words built
 *     from the SplitMix64 output finalizer (Steele, Lea, Flood, OOPSLA 2014);
 *     the paper uses CityHash64 (Sec. 5, common parameters).
 *   - split of the 64-bit hash h for 2^B buckets (B <= 29):
 *       primary   p = h mod 2^B
 *       tag       t = h >> 48                        (16-bit tags, Sec. 4.3)
 *       for B <= 24, the secondary-hash field is h >> 24:
 *         alternate a = (h >> 24) mod 2^B
 *         bloom bit indices (h >> 24) mod 64 and (h >> 30) mod 64
 *       for B > 24 that field would overlap p, so a second word
 *       g = fmix(h xor 0xc2b2ae3d27d4eb4f) takes its place:
 *         alternate a = g mod 2^B
 *         bloom bit indices (g >> 32) mod 64 and (g >> 38) mod 64
 *       and a = a xor 1 when a == p.  The two bloom bits come from the key's
 *       secondary hash (Sec. 4.1) in both cases.
 *   - placement: primary before secondary, lowest free slot first.
 *   - insert of a present key overwrites its value (status UPDATED).
 *   - cuckoo path: random walk from the primary bucket, at most max_kicks
 *     displacements, victims drawn from a counter-based SplitMix64 stream
 *     keyed by the inserted key's hash, an entry stored in its secondary
 *     bucket preferred as victim; the path is computed first and the moves
 *     are applied afterwards (Sec. 4.1, last paragraphs), so that a failed
 *     insert leaves the table unchanged.  This victim preference is the
 *     reading under which the table reproduces the paper's statistics
 *     (entries in secondary, Sec. 3; moved counters, Sec. 4.1; false
 *     positive rates, Sec. 5.3).
 *   - the moved counter is 16 bits; an insertion that would overflow it is
 *     refused.
 *   - lookup of an absent key returns value 0.
 *
 * Bucket image (64 bytes, one cache line, Sec. 4.3):
 *   0..15  tag[8]   u16      16-bit tags, one per slot
 *   16..23 bloom    u64      bloom filter of keys displaced from this bucket
 *   24..25 moved    u16      moved counter of the bloom filter (Sec. 4.1)
 *   26     busy     u8       bit s set <=> slot s holds an entry
 *   27     sec      u8       bit s set <=> the entry of slot s sits in its
 *                            secondary (alternate) bucket
 *   28..31 lock     u32      zero at batch boundaries (the GPU uses it)
 *   32..63 other[8] u32      the other bucket of the entry in slot s, so
 *                            that a cuckoo path is searched without reading
 *                            keys (Sec. 4.3)
 * Key/value record (32 bytes) for slot s of bucket b at index b*8+s of the
 * key/value array (implicit index, Sec. 4.3): key[16] | value u64 | pad u64.
 * On a table with timers (Sec. 4.2) the low 16 bits of the pad hold the
 * entry's expiration time; the pad is zero otherwise.
 */
#include <stddef.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORC_SLOTS 8

enum { ORC_INSERTED = 0, ORC_UPDATED = 1, ORC_FAILED = 2 };
enum { ORC_MODE_CUCKOOPP = 0, ORC_MODE_BOTH = 1, ORC_MODE_OPTIMISTIC = 2 };

typedef struct {
    uint16_t tag[ORC_SLOTS];
    uint64_t bloom;
    uint16_t moved;
    uint8_t busy;
    uint8_t sec;
    uint32_t lock;
    uint32_t other[ORC_SLOTS];
} orc_bucket;

typedef struct {
    uint8_t key[16];
    uint64_t value;
    uint64_t pad;
} orc_kv;

_Static_assert(sizeof(orc_bucket) == 64, "bucket is one 64-byte line");
_Static_assert(offsetof(orc_bucket, bloom) == 16, "bloom offset");
_Static_assert(offsetof(orc_bucket, moved) == 24, "moved offset");
_Static_assert(offsetof(orc_bucket, busy) == 26, "busy offset");
_Static_assert(offsetof(orc_bucket, sec) == 27, "sec offset");
_Static_assert(offsetof(orc_bucket, lock) == 28, "lock offset");
_Static_assert(offsetof(orc_bucket, other) == 32, "other offset");
_Static_assert(sizeof(orc_kv) == 32, "kv record is 32 bytes");

typedef struct {
    uint32_t log2_buckets;
    uint64_t nbuckets;
    uint64_t seed;
    uint32_t max_kicks;
    int plain; /* 1: no bloom filter / moved counter maintenance */
    int timed; /* 1: every entry carries a 16-bit expiration time (Sec. 4.2) */
    orc_bucket *buckets;
    orc_kv *kv;
    uint64_t live;
} orc_table;

typedef struct {
    uint64_t p, a;
    uint32_t tag;
    uint32_t b1, b2;
    uint64_t bloom_mask;
} orc_split_t;

/* Statistics of a table.  Two false-positive rates of the bloom filter:
 *  - the rate a negative lookup meets: its two bit indices are independent
 *    and uniform over 64, and independent of its primary bucket, so it
 *    passes bucket b's filter with probability (popcount(bloom_b)/64)^2;
 *    the mean over buckets is bloom_pc2_sum / (4096 * nbuckets);
 *  - the rate expected from the number of keys inserted in each filter
 *    (Sec. 5.3, false positive rate table): a 64-bit filter with 2 hash
 *    functions holding k = moved_b keys passes with probability
 *    (1 - (63/64)^(2k))^2; fpr_from_moved_sum adds it over buckets. */
#define ORC_MOVED_BINS 66 /* 0..64 and ">64" */
typedef struct {
    uint64_t nbuckets;
    uint64_t live;
    uint64_t in_secondary;
    uint64_t bloom_pc_sum;
    uint64_t bloom_pc2_sum;
    uint64_t locked;
    uint64_t moved_hist[ORC_MOVED_BINS];
    double fpr_from_moved_sum;
} orc_stats_t;

/* ------------------------------------------------------------------ hash */

/* SplitMix64 output finalizer (Steele, Lea, Flood, OOPSLA 2014). */
static uint64_t orc_fmix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

uint64_t orc_fmix64_export(uint64_t z) { return orc_fmix64(z); }

/* Seeded hash of a 16-byte key: the key is read as four little-endian u32
 * words w0..w3; lo = w0 | w1<<32, hi = w2 | w3<<32;
 * h = fmix(fmix(lo xor seed) xor hi). */
uint64_t orc_hash(const uint8_t *key, uint64_t seed)
{
    uint64_t lo = 0, hi = 0;
    for (int i = 7; i >= 0; i--) lo = (lo << 8) | key[i];
    for (int i = 15; i >= 8; i--) hi = (hi << 8) | key[i];
    return orc_fmix64(orc_fmix64(lo ^ seed) ^ hi);
}

void orc_split(uint64_t h, uint32_t log2_buckets, orc_split_t *out)
{
    uint64_t mask = (log2_buckets >= 64) ? ~0ULL : ((1ULL << log2_buckets) - 1);
    out->p = h & mask;
    out->tag = (uint32_t)(h >> 48);
    if (log2_buckets <= 24) {
        out->a = (h >> 24) & mask;
        out->b1 = (uint32_t)((h >> 24) & 63);
        out->b2 = (uint32_t)((h >> 30) & 63);
    } else {
        /* the field above bit 24 overlaps p: a second word of the hash */
        uint64_t g = orc_fmix64(h ^ 0xc2b2ae3d27d4eb4fULL);
        out->a = g & mask;
        out->b1 = (uint32_t)((g >> 32) & 63);
        out->b2 = (uint32_t)((g >> 38) & 63);
    }
    if (out->a == out->p) out->a ^= 1;
    out->bloom_mask = (1ULL << out->b1) | (1ULL << out->b2);
}

/* Counter-based SplitMix64 stream: element i of the stream whose state
 * starts at `base` (Steele, Lea, Flood 2014). */
static uint64_t orc_stream(uint64_t base, uint64_t i)
{
    return orc_fmix64(base + (i + 1) * 0x9e3779b97f4a7c15ULL);
}

/* --------------------------------------------------------------- create */

orc_table *orc_create(uint32_t log2_buckets, uint64_t seed, uint32_t max_kicks, int plain)
{
    if (log2_buckets < 1 || log2_buckets > 29) return NULL;
    orc_table *t = (orc_table *)calloc(1, sizeof(orc_table));
    if (!t) return NULL;
    t->log2_buckets = log2_buckets;
    t->nbuckets = 1ULL << log2_buckets;
    t->seed = seed;
    t->max_kicks = max_kicks;
    t->plain = plain ? 1 : 0;
    t->buckets = (orc_bucket *)aligned_alloc(64, t->nbuckets * sizeof(orc_bucket));
    t->kv = (orc_kv *)aligned_alloc(64, t->nbuckets * ORC_SLOTS * sizeof(orc_kv));
    if (!t->buckets || !t->kv) {
        free(t->buckets);
        free(t->kv);
        free(t);
        return NULL;
    }
    memset(t->buckets, 0, t->nbuckets * sizeof(orc_bucket));
    memset(t->kv, 0, t->nbuckets * ORC_SLOTS * sizeof(orc_kv));
    return t;
}

void orc_destroy(orc_table *t)
{
    if (!t) return;
    free(t->buckets);
    free(t->kv);
    free(t);
}

uint8_t *orc_buckets_ptr(orc_table *t) { return (uint8_t *)t->buckets; }
uint8_t *orc_kv_ptr(orc_table *t) { return (uint8_t *)t->kv; }
uint64_t orc_live(const orc_table *t) { return t->live; }

/* -------------------------------------------------------------- helpers */

static orc_kv *orc_rec(const orc_table *t, uint64_t b, int s)
{
    return &t->kv[b * ORC_SLOTS + (uint64_t)s];
}

/* Sec. 4.2: an entry with expiration time e is alive at time `now` iff
 * (e - now) mod 2^16 < 1024: expiration times are kept within 1024 units
 * of the current time, so the 16-bit difference tells valid entries from
 * expired ones (and from wrapped-around ones, until 64512 units after
 * expiry, which the periodic scan prevents).  Tables without timers have
 * no expired entries. */
#define ORC_MAX_DELAY 1024u

static int orc_expired(const orc_table *t, uint64_t b, int s, uint16_t now)
{
    if (!t->timed) return 0;
    uint16_t e = (uint16_t)t->kv[b * ORC_SLOTS + (uint64_t)s].pad;
    return (uint16_t)(e - now) >= ORC_MAX_DELAY;
}

enum { ORC_ANY = 0, ORC_ALIVE = 1, ORC_DEAD = 2 };

/* Slot of `key` in bucket b, or -1.  Candidates are the busy slots whose
 * tag equals the key's tag (and, on a table with timers, that are alive
 * or expired as `want` asks); each candidate's full key is compared, in
 * ascending slot order (Sec. 2, lookup procedure).  *kv_lines counts the
 * distinct 64-byte lines of the key/value array that were read. */
static int orc_find_in(const orc_table *t, uint64_t b, uint32_t tag, const uint8_t *key,
                       uint32_t *kv_lines, int want, uint16_t now)
{
    const orc_bucket *bk = &t->buckets[b];
    int64_t last_line = -1;
    for (int s = 0; s < ORC_SLOTS; s++) {
        if (!(bk->busy & (1u << s))) continue;
        if (bk->tag[s] != tag) continue;
        if (want != ORC_ANY && orc_expired(t, b, s, now) != (want == ORC_DEAD)) continue;
        int64_t line = (int64_t)((b * ORC_SLOTS + (uint64_t)s) >> 1);
        if (kv_lines && line != last_line) (*kv_lines)++;
        last_line = line;
        if (memcmp(orc_rec(t, b, s)->key, key, 16) == 0) return s;
    }
    return -1;
}

static int orc_lowest_free(const orc_bucket *bk)
{
    for (int s = 0; s < ORC_SLOTS; s++)
        if (!(bk->busy & (1u << s))) return s;
    return -1;
}

/* Lowest slot that is free or holds an expired entry (Sec. 4.2: an insert
 * overwrites expired entries as if their slots were free). */
static int orc_lowest_available(const orc_table *t, uint64_t b, uint16_t now)
{
    const orc_bucket *bk = &t->buckets[b];
    for (int s = 0; s < ORC_SLOTS; s++)
        if (!(bk->busy & (1u << s)) || orc_expired(t, b, s, now)) return s;
    return -1;
}

static int orc_bloom_pass(const orc_table *t, uint64_t p, uint64_t m)
{
    return (t->buckets[p].bloom & m) == m;
}

static void orc_place(orc_table *t, uint64_t b, int s, const uint8_t *key, uint64_t value,
                      uint32_t tag, uint64_t other, int in_secondary, uint16_t expiry)
{
    orc_kv *r = orc_rec(t, b, s);
    memcpy(r->key, key, 16);
    r->value = value;
    r->pad = t->timed ? (uint64_t)expiry : 0;
    orc_bucket *bk = &t->buckets[b];
    bk->tag[s] = (uint16_t)tag;
    bk->other[s] = (uint32_t)other;
    bk->busy |= (uint8_t)(1u << s);
    if (in_secondary)
        bk->sec |= (uint8_t)(1u << s);
    else
        bk->sec &= (uint8_t)~(1u << s);
}

/* A key is added to the bloom filter of its primary bucket p when it is
 * stored in its secondary bucket: its two bits are set and the moved
 * counter is incremented (Sec. 4.1). */
static void orc_bloom_add(orc_table *t, uint64_t p, uint64_t m)
{
    if (t->plain) return;
    t->buckets[p].bloom |= m;
    t->buckets[p].moved += 1;
}

/* A key whose primary is p leaves its secondary bucket (deletion, or a move
 * back to the primary): the moved counter is decremented and the bloom
 * filter is reset to empty when it reaches zero (Sec. 4.1). */
static void orc_bloom_remove(orc_table *t, uint64_t p)
{
    if (t->plain) return;
    t->buckets[p].moved -= 1;
    if (t->buckets[p].moved == 0) t->buckets[p].bloom = 0;
}

static int orc_moved_full(const orc_table *t, uint64_t p)
{
    return !t->plain && t->buckets[p].moved == 0xFFFF;
}

/* --------------------------------------------------------------- lookup */

/* Lookup (Sec. 2 and Sec. 4.1).  mode CUCKOOPP: primary bucket, then the
 * secondary bucket only if the key was not found and the primary's bloom
 * filter passes.  mode BOTH: both buckets are always fetched (pessimistic).
 * mode OPTIMISTIC: primary, then secondary whenever not found (Sec. 3).
 * A plain table keeps no bloom filter, so there CUCKOOPP probes the
 * secondary whenever the key is not in the primary.
 * The answer is the same for every mode; *bucket_lines and *kv_lines report
 * the 64-byte lines fetched from the bucket and key/value arrays. */
int orc_lookup_at(orc_table *t, const uint8_t *key, int mode, uint16_t now, int refresh,
                  uint16_t expiry, uint64_t *value, uint32_t *bucket_lines, uint32_t *kv_lines)
{
    orc_split_t sp;
    orc_split(orc_hash(key, t->seed), t->log2_buckets, &sp);
    uint32_t bl = (mode == ORC_MODE_BOTH) ? 2 : 1, kl = 0;
    int found = 0;
    uint64_t v = 0, b = sp.p;
    int s = orc_find_in(t, sp.p, sp.tag, key, &kl, ORC_ALIVE, now);
    if (s < 0) {
        int probe_secondary;
        if (mode == ORC_MODE_CUCKOOPP && !t->plain)
            probe_secondary = orc_bloom_pass(t, sp.p, sp.bloom_mask);
        else
            probe_secondary = 1;
        if (probe_secondary) {
            if (mode != ORC_MODE_BOTH) bl += 1;
            s = orc_find_in(t, sp.a, sp.tag, key, &kl, ORC_ALIVE, now);
            b = sp.a;
        }
    }
    if (s >= 0) {
        found = 1;
        v = orc_rec(t, b, s)->value;
        /* Sec. 4.2: a lookup may set a new expiration time of the entry */
        if (refresh && t->timed) orc_rec(t, b, s)->pad = expiry;
    }
    if (value) *value = v;
    if (bucket_lines) *bucket_lines = bl;
    if (kv_lines) *kv_lines = kl;
    return found;
}

/* Lookup without timers (every entry alive, nothing written). */
int orc_lookup(const orc_table *t, const uint8_t *key, int mode, uint64_t *value,
               uint32_t *bucket_lines, uint32_t *kv_lines)
{
    return orc_lookup_at((orc_table *)t, key, mode, 0, 0, 0, value, bucket_lines, kv_lines);
}

/* ----------------------------------------------------------- cuckoo path */

typedef struct {
    uint64_t b;
    int s;
} orc_step;

static int orc_on_path(const orc_step *path, int len, uint64_t b, int s)
{
    for (int i = 0; i < len; i++)
        if (path[i].b == b && path[i].s == s) return 1;
    return 0;
}

/* Moves the entry of slot (x, s) into free slot f of its other bucket y,
 * maintaining the bloom filter and moved counter of the entry's primary
 * bucket: a move from primary to secondary acts like an insertion into the
 * bloom filter, a move from secondary to primary like a deletion (Sec. 4.1,
 * cuckoo path). */
static void orc_move(orc_table *t, uint64_t x, int s, int f)
{
    orc_bucket *bx = &t->buckets[x];
    uint64_t y = bx->other[s];
    orc_kv *r = orc_rec(t, x, s);
    orc_split_t sp;
    orc_split(orc_hash(r->key, t->seed), t->log2_buckets, &sp);
    int was_secondary = (bx->sec >> s) & 1;
    orc_place(t, y, f, r->key, r->value, bx->tag[s], x, !was_secondary, (uint16_t)r->pad);
    if (was_secondary)
        orc_bloom_remove(t, sp.p); /* y is the primary */
    else
        orc_bloom_add(t, sp.p, sp.bloom_mask); /* x is the primary */
    bx->busy &= (uint8_t)~(1u << s);
    bx->sec &= (uint8_t)~(1u << s);
}

/* Searches a cuckoo path that frees a slot of bucket start (Sec. 2 and
 * Sec. 4.1): a random walk over full buckets; at bucket b a victim slot v
 * is drawn and the walk continues at the victim's other bucket, until a
 * bucket with a free slot is reached.  Victim choice, in order of
 * preference: an entry stored in its secondary bucket (the move sends it
 * back to its primary, keeping most entries in their primary, Sec. 3 and
 * Sec. 4.1), then any entry whose other bucket is not the bucket just
 * left, then any entry.  A (bucket, slot) pair is never used twice, so the
 * recorded moves stay valid when replayed backwards; a move that would
 * overflow a moved counter is never chosen.
 * Returns the path length (number of displacements) or -1. */
static int orc_find_path(const orc_table *t, uint64_t start, uint64_t h, orc_step *path)
{
    uint64_t cur = start, prev = UINT64_MAX;
    for (uint32_t step = 0; step < t->max_kicks; step++) {
        const orc_bucket *bk = &t->buckets[cur];
        int cand[ORC_SLOTS], ncand = 0, pref[ORC_SLOTS], npref = 0, home[ORC_SLOTS], nhome = 0;
        for (int s = 0; s < ORC_SLOTS; s++) {
            if (orc_on_path(path, (int)step, cur, s)) continue;
            int guest = (bk->sec >> s) & 1;
            /* a primary-to-secondary move adds to cur's moved counter */
            if (!guest && orc_moved_full(t, cur)) continue;
            cand[ncand++] = s;
            if (bk->other[s] == prev) continue;
            pref[npref++] = s;
            if (guest) home[nhome++] = s;
        }
        if (ncand == 0) return -1;
        uint64_t r = orc_stream(h, step);
        int v;
        if (nhome > 0)
            v = home[r % (uint64_t)nhome];
        else if (npref > 0)
            v = pref[r % (uint64_t)npref];
        else
            v = cand[r % (uint64_t)ncand];
        path[step].b = cur;
        path[step].s = v;
        uint64_t nxt = bk->other[v];
        if (t->buckets[nxt].busy != 0xFF) return (int)step + 1;
        prev = cur;
        cur = nxt;
    }
    return -1;
}

/* --------------------------------------------------------------- insert */

/* Removes the entry of slot s of bucket b (its key is not looked at): if it
 * sat in its secondary bucket, the moved counter of its primary (the slot's
 * other bucket) is decremented and that bloom filter reset at zero (Sec.
 * 4.1). */
static void orc_remove_slot(orc_table *t, uint64_t b, int s)
{
    orc_bucket *bk = &t->buckets[b];
    if ((bk->sec >> s) & 1) orc_bloom_remove(t, bk->other[s]);
    bk->busy &= (uint8_t)~(1u << s);
    bk->sec &= (uint8_t)~(1u << s);
    t->live--;
}

/* Insert (Sec. 2 and Sec. 4.1): update in place if present; else the
 * lowest free slot of the primary bucket; else the lowest free slot of the
 * secondary bucket, adding the key to the primary's bloom filter; else a
 * cuckoo path is computed and applied, freeing a slot of the primary.
 * With timers (Sec. 4.2) only alive entries are "present", the key's
 * expiration time is set (also on an update), an expired copy of the key
 * is overwritten where it stands, and a slot holding an expired entry
 * counts as free: the expired entry is removed first (lazy deletion).
 * The cuckoo path moves expired entries like any other and ends only at a
 * bucket with a slot that is really free. */
int orc_insert_at(orc_table *t, const uint8_t *key, uint64_t value, uint16_t expiry,
                  uint16_t now)
{
    uint64_t h = orc_hash(key, t->seed);
    orc_split_t sp;
    orc_split(h, t->log2_buckets, &sp);
    const int pass = t->plain || orc_bloom_pass(t, sp.p, sp.bloom_mask);

    for (int want = ORC_ALIVE; want <= ORC_DEAD; want++) {
        if (want == ORC_DEAD && !t->timed) break;
        for (int k = 0; k < 2; k++) {
            uint64_t b = k ? sp.a : sp.p;
            if (k && !pass) break;
            int s = orc_find_in(t, b, sp.tag, key, NULL, want, now);
            if (s >= 0) {
                orc_rec(t, b, s)->value = value;
                if (t->timed) orc_rec(t, b, s)->pad = expiry;
                return want == ORC_ALIVE ? ORC_UPDATED : ORC_INSERTED;
            }
        }
    }

    int s = orc_lowest_available(t, sp.p, now);
    if (s >= 0) {
        if (t->buckets[sp.p].busy & (1u << s)) orc_remove_slot(t, sp.p, s);
        orc_place(t, sp.p, s, key, value, sp.tag, sp.a, 0, expiry);
        t->live++;
        return ORC_INSERTED;
    }
    s = orc_lowest_available(t, sp.a, now);
    if (s >= 0 && !orc_moved_full(t, sp.p)) {
        if (t->buckets[sp.a].busy & (1u << s)) orc_remove_slot(t, sp.a, s);
        orc_place(t, sp.a, s, key, value, sp.tag, sp.p, 1, expiry);
        orc_bloom_add(t, sp.p, sp.bloom_mask);
        t->live++;
        return ORC_INSERTED;
    }

    orc_step *path = (orc_step *)malloc(sizeof(orc_step) * (t->max_kicks ? t->max_kicks : 1));
    if (!path) return ORC_FAILED;
    int len = orc_find_path(t, sp.p, h, path);
    if (len < 0) {
        free(path);
        return ORC_FAILED;
    }
    /* Apply the displacements from the end of the path back to its start:
     * the last victim goes into the free slot found, every earlier victim
     * into the slot vacated by the next one. */
    uint64_t last_b = t->buckets[path[len - 1].b].other[path[len - 1].s];
    int f = orc_lowest_free(&t->buckets[last_b]);
    for (int i = len - 1; i >= 0; i--) {
        orc_move(t, path[i].b, path[i].s, f);
        f = path[i].s;
    }
    /* the walk started at the primary, whose slot path[0].s is now free */
    orc_place(t, sp.p, path[0].s, key, value, sp.tag, sp.a, 0, expiry);
    t->live++;
    free(path);
    return ORC_INSERTED;
}

/* Insert without timers. */
int orc_insert(orc_table *t, const uint8_t *key, uint64_t value)
{
    return orc_insert_at(t, key, value, 0, 0);
}

/* --------------------------------------------------------------- delete */

/* Delete (Sec. 4.1): find the key as a lookup does and free its slot; if it
 * sat in its secondary bucket, decrement the moved counter of its primary
 * and reset the primary's bloom filter when the counter reaches zero.
 * With timers an expired copy is removed too, but only an alive one counts
 * as found (Sec. 4.2: expired entries are absent). */
int orc_delete_at(orc_table *t, const uint8_t *key, uint16_t now)
{
    orc_split_t sp;
    orc_split(orc_hash(key, t->seed), t->log2_buckets, &sp);
    int s = orc_find_in(t, sp.p, sp.tag, key, NULL, ORC_ANY, now);
    uint64_t b = sp.p;
    if (s < 0 && (t->plain || orc_bloom_pass(t, sp.p, sp.bloom_mask))) {
        s = orc_find_in(t, sp.a, sp.tag, key, NULL, ORC_ANY, now);
        b = sp.a;
    }
    if (s < 0) return 0;
    const int alive = !orc_expired(t, b, s, now);
    orc_remove_slot(t, b, s);
    return alive;
}

/* Delete without timers. */
int orc_delete(orc_table *t, const uint8_t *key)
{
    return orc_delete_at(t, key, 0);
}

/* Anti-revival scan (Sec. 4.2): every expired entry is removed, so that it
 * cannot become alive again when the 16-bit clock wraps around; the scan
 * must run at least every 64512 time units.  Returns the entries removed. */
uint64_t orc_expire_scan(orc_table *t, uint16_t now)
{
    uint64_t removed = 0;
    for (uint64_t b = 0; b < t->nbuckets; b++)
        for (int s = 0; s < ORC_SLOTS; s++)
            if ((t->buckets[b].busy & (1u << s)) && orc_expired(t, b, s, now)) {
                orc_remove_slot(t, b, s);
                removed++;
            }
    return removed;
}

/* A table whose entries carry expiration times (Sec. 4.2). */
orc_table *orc_create_timed(uint32_t log2_buckets, uint64_t seed, uint32_t max_kicks, int plain)
{
    orc_table *t = orc_create(log2_buckets, seed, max_kicks, plain);
    if (t) t->timed = 1;
    return t;
}

/* -------------------------------------------------------------- batches */

/* Batch forms process the keys in index order.  keys: n x 16 bytes. */
void orc_insert_batch(orc_table *t, const uint8_t *keys, const uint64_t *values, uint64_t n,
                      uint8_t *status)
{
    for (uint64_t i = 0; i < n; i++) {
        int st = orc_insert(t, keys + 16 * i, values[i]);
        if (status) status[i] = (uint8_t)st;
    }
}

/* Returns the total bucket lines and kv lines fetched through the two
 * accumulators (nullable). */
void orc_lookup_batch(const orc_table *t, const uint8_t *keys, uint64_t n, int mode,
                      uint8_t *found, uint64_t *values, uint64_t *bucket_lines_total,
                      uint64_t *kv_lines_total)
{
    uint64_t bt = 0, kt = 0;
    for (uint64_t i = 0; i < n; i++) {
        uint32_t bl, kl;
        uint64_t v;
        int f = orc_lookup(t, keys + 16 * i, mode, &v, &bl, &kl);
        if (found) found[i] = (uint8_t)f;
        if (values) values[i] = v;
        bt += bl;
        kt += kl;
    }
    if (bucket_lines_total) *bucket_lines_total = bt;
    if (kv_lines_total) *kv_lines_total = kt;
}

void orc_delete_batch(orc_table *t, const uint8_t *keys, uint64_t n, uint8_t *found)
{
    for (uint64_t i = 0; i < n; i++) {
        int f = orc_delete(t, keys + 16 * i);
        if (found) found[i] = (uint8_t)f;
    }
}

/* Timed batch forms: expiry has one entry per key (inserts); a lookup with
 * refresh sets the expiration time of every alive entry it finds. */
void orc_insert_batch_at(orc_table *t, const uint8_t *keys, const uint64_t *values,
                         const uint16_t *expiry, uint64_t n, uint16_t now, uint8_t *status)
{
    for (uint64_t i = 0; i < n; i++) {
        int st = orc_insert_at(t, keys + 16 * i, values[i], expiry[i], now);
        if (status) status[i] = (uint8_t)st;
    }
}

void orc_lookup_batch_at(orc_table *t, const uint8_t *keys, uint64_t n, int mode, uint16_t now,
                         int refresh, uint16_t expiry, uint8_t *found, uint64_t *values)
{
    for (uint64_t i = 0; i < n; i++) {
        uint64_t v;
        int f = orc_lookup_at(t, keys + 16 * i, mode, now, refresh, expiry, &v, NULL, NULL);
        if (found) found[i] = (uint8_t)f;
        if (values) values[i] = v;
    }
}

void orc_delete_batch_at(orc_table *t, const uint8_t *keys, uint64_t n, uint16_t now,
                         uint8_t *found)
{
    for (uint64_t i = 0; i < n; i++) {
        int f = orc_delete_at(t, keys + 16 * i, now);
        if (found) found[i] = (uint8_t)f;
    }
}

/* ---------------------------------------------------------------- stats */

static int orc_popcount64(uint64_t x)
{
    int c = 0;
    while (x) {
        x &= x - 1;
        c++;
    }
    return c;
}

/* Statistics of any table image (the oracle's own, or one under test). */
void orc_image_stats(const uint8_t *buckets, uint32_t log2_buckets, orc_stats_t *st)
{
    const orc_bucket *bk = (const orc_bucket *)buckets;
    uint64_t nb = 1ULL << log2_buckets;
    memset(st, 0, sizeof(*st));
    st->nbuckets = nb;
    for (uint64_t b = 0; b < nb; b++) {
        st->live += (uint64_t)orc_popcount64(bk[b].busy);
        st->in_secondary += (uint64_t)orc_popcount64(bk[b].sec);
        uint64_t pc = (uint64_t)orc_popcount64(bk[b].bloom);
        st->bloom_pc_sum += pc;
        st->bloom_pc2_sum += pc * pc;
        if (bk[b].lock) st->locked++;
        uint32_t m = bk[b].moved;
        st->moved_hist[m < ORC_MOVED_BINS - 1 ? m : ORC_MOVED_BINS - 1]++;
        double q = 1.0;
        for (uint32_t i = 0; i < 2 * m; i++) q *= 63.0 / 64.0;
        st->fpr_from_moved_sum += (1.0 - q) * (1.0 - q);
    }
}

void orc_stats(const orc_table *t, orc_stats_t *st)
{
    orc_image_stats((const uint8_t *)t->buckets, t->log2_buckets, st);
}

uint64_t orc_stats_size(void) { return sizeof(orc_stats_t); }

/* ------------------------------------------------------ image invariants */

/* Checks the structural invariants of a table image (its own or one under
 * test) and returns 0 when they all hold, else the number of the first
 * violated invariant, with a message:
 *   I1 every busy slot (b, s) holds a key k with b in {p(k), a(k)},
 *      tag == t(k), other[s] == the other of the two, sec bit <=> b == a(k)
 *   I2 no key is stored twice
 *   I3 moved[b] == number of stored keys with primary b that sit in their
 *      secondary bucket (0 everywhere on a plain table)
 *   I4 for every such key both of its bits are set in bloom[b]
 *   I5 moved[b] == 0 implies bloom[b] == 0
 *   I6 the pad word of every busy slot is zero on a table without timers;
 *      with timers it holds only a 16-bit expiration time (the value may
 *      take all 64 bits: Sec. 4.3 keeps the times beside the tags)
 *   I9 lock words are zero and sec is a subset of busy
 * Statement of I3-I5 follows Sec. 4.1 (bloom filter, moved counter and its
 * reset at zero).  flags: bit 0 plain table, bit 1 table with timers. */
int orc_check_image(const uint8_t *buckets, const uint8_t *kvbytes, uint32_t log2_buckets,
                    uint64_t seed, int flags, char *msg, uint64_t msglen)
{
    const int plain = flags & 1, timed = (flags >> 1) & 1;
    const orc_bucket *bk = (const orc_bucket *)buckets;
    const orc_kv *kv = (const orc_kv *)kvbytes;
    uint64_t nb = 1ULL << log2_buckets;
    uint32_t *count = (uint32_t *)calloc(nb, sizeof(uint32_t));
    uint64_t *need = (uint64_t *)calloc(nb, sizeof(uint64_t));
    int rc = 0;
    if (!count || !need) {
        snprintf(msg, msglen, "out of memory");
        free(count);
        free(need);
        return -1;
    }
    for (uint64_t b = 0; b < nb && !rc; b++) {
        if (bk[b].lock != 0) {
            snprintf(msg, msglen, "I9: bucket %llu lock word %u", (unsigned long long)b, bk[b].lock);
            rc = 9;
            break;
        }
        if (bk[b].sec & ~bk[b].busy) {
            snprintf(msg, msglen, "I9: bucket %llu sec 0x%02x not within busy 0x%02x",
                     (unsigned long long)b, bk[b].sec, bk[b].busy);
            rc = 9;
            break;
        }
        for (int s = 0; s < ORC_SLOTS && !rc; s++) {
            if (!(bk[b].busy & (1u << s))) continue;
            const uint8_t *key = kv[b * ORC_SLOTS + (uint64_t)s].key;
            const orc_kv *rec = &kv[b * ORC_SLOTS + (uint64_t)s];
            if (timed ? (rec->pad >> 16) != 0 : rec->pad != 0) {
                snprintf(msg, msglen, "I6: bucket %llu slot %d value %016llx pad %016llx",
                         (unsigned long long)b, s, (unsigned long long)rec->value,
                         (unsigned long long)rec->pad);
                rc = 6;
                break;
            }
            orc_split_t sp;
            orc_split(orc_hash(key, seed), log2_buckets, &sp);
            int in_p = (b == sp.p), in_a = (b == sp.a);
            if (!in_p && !in_a) {
                snprintf(msg, msglen, "I1: key in bucket %llu slot %d belongs to %llu/%llu",
                         (unsigned long long)b, s, (unsigned long long)sp.p,
                         (unsigned long long)sp.a);
                rc = 1;
                break;
            }
            uint64_t oth = in_p ? sp.a : sp.p;
            int sec = (bk[b].sec >> s) & 1;
            if (bk[b].tag[s] != sp.tag || bk[b].other[s] != oth || sec != in_a) {
                snprintf(msg, msglen,
                         "I1: bucket %llu slot %d tag %u/%u other %u/%llu sec %d/%d",
                         (unsigned long long)b, s, bk[b].tag[s], sp.tag, bk[b].other[s],
                         (unsigned long long)oth, sec, in_a);
                rc = 1;
                break;
            }
            /* I2: a second copy could only sit in b or in its other bucket */
            for (int pass = 0; pass < 2 && !rc; pass++) {
                uint64_t c = pass ? oth : b;
                for (int u = 0; u < ORC_SLOTS; u++) {
                    if (c == b && u == s) continue;
                    if (!(bk[c].busy & (1u << u))) continue;
                    if (memcmp(kv[c * ORC_SLOTS + (uint64_t)u].key, key, 16) == 0) {
                        snprintf(msg, msglen, "I2: key of bucket %llu slot %d also in %llu slot %d",
                                 (unsigned long long)b, s, (unsigned long long)c, u);
                        rc = 2;
                        break;
                    }
                }
            }
            if (in_a) {
                count[sp.p]++;
                need[sp.p] |= sp.bloom_mask;
            }
        }
    }
    for (uint64_t b = 0; b < nb && !rc; b++) {
        uint32_t want = plain ? 0 : count[b];
        if (bk[b].moved != want) {
            snprintf(msg, msglen, "I3: bucket %llu moved %u, displaced keys %u%s",
                     (unsigned long long)b, bk[b].moved, count[b], plain ? " (plain)" : "");
            rc = 3;
            break;
        }
        if (!plain && (bk[b].bloom & need[b]) != need[b]) {
            snprintf(msg, msglen, "I4: bucket %llu bloom %016llx misses bits %016llx",
                     (unsigned long long)b, (unsigned long long)bk[b].bloom,
                     (unsigned long long)need[b]);
            rc = 4;
            break;
        }
        if (bk[b].moved == 0 && bk[b].bloom != 0) {
            snprintf(msg, msglen, "I5: bucket %llu moved 0 but bloom %016llx",
                     (unsigned long long)b, (unsigned long long)bk[b].bloom);
            rc = 5;
            break;
        }
    }
    if (!rc && msglen) msg[0] = 0;
    free(count);
    free(need);
    return rc;
}
