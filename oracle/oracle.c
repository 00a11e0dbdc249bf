/*
 * CPU oracle for the equi hash join.  TEST INFRASTRUCTURE ONLY: the tests,
 * the smoke check and the CPU-baseline leg of the benchmark call it; the
 * product path never does.
 *
 * What it computes (Section 3.1, Algorithm 1, steps b1-b4 and p1-p4): the
 * multiset of (rid_R, rid_S) pairs, one for every tuple r of R and s of S with
 * r.key == s.key, plus its size.  Duplicate keys are allowed on both sides, so
 * a key that occurs a times in R and b times in S yields a*b pairs.
 *
 * How (kept deliberately plain, single-threaded, in the paper's order):
 *   Build, for each tuple of R in input order:
 *     b1  bucket = MurmurHash2(key) mod (number of buckets)
 *     b2  visit the bucket header (tuple count + head of the key list)
 *     b3  walk the bucket's key list; create a key node if the key is new
 *     b4  append the record id to that key's rid list
 *   Probe, for each tuple of S in input order:
 *     p1  bucket = MurmurHash2(key) mod (number of buckets)
 *     p2  visit the bucket header
 *     p3  walk the bucket's key list looking for the key
 *     p4  for every rid in the matching key's rid list emit (rid, s.rid)
 * The table layout is the one Section 3.1 describes: an array of bucket
 * headers (count, pointer to key list); a key list of the distinct keys that
 * hash to the bucket; per key a list of record ids.  "Pointers" are int32
 * indices into node pools (-1 = none); the number of buckets is the smallest
 * power of two >= |R|.
 *
 * Hash: MurmurHash 2.0 (Section 5.1) on the key's four bytes, written from
 * Austin Appleby's public-domain description of the algorithm.  The join
 * result does not depend on the hash.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint32_t count;    /* tuples of R in this bucket */
    int32_t key_head;  /* first key node, -1 if none */
} bucket_header;

typedef struct {
    int32_t key;
    int32_t next;      /* next key node of the same bucket */
    int32_t rid_head;  /* first rid node of this key */
    int32_t rid_tail;  /* last rid node of this key (append keeps input order) */
} key_node;

typedef struct {
    int32_t rid;
    int32_t next;
} rid_node;

typedef struct oracle_table {
    uint64_t nbuckets;
    bucket_header* buckets;
    key_node* keys;
    int64_t nkeys;
    rid_node* rids;
    int64_t nrids;
} oracle_table;

/* MurmurHash 2.0, 32-bit, for one 4-byte little-endian block. */
static uint32_t murmur2_key(int32_t key, uint32_t seed) {
    const uint32_t m = 0x5bd1e995u;
    const int r = 24;
    uint32_t h = seed ^ 4u;
    uint32_t k = (uint32_t)key;
    k *= m;
    k ^= k >> r;
    k *= m;
    h *= m;
    h ^= k;
    h ^= h >> 13;
    h *= m;
    h ^= h >> 15;
    return h;
}

#define ORACLE_SEED 0x2545F491u

static uint64_t bucket_of(const oracle_table* t, int32_t key) {
    return (uint64_t)murmur2_key(key, ORACLE_SEED) & (t->nbuckets - 1);
}

void oracle_free(oracle_table* t) {
    if (!t) return;
    free(t->buckets);
    free(t->keys);
    free(t->rids);
    free(t);
}

/* Builds the table over R (b1-b4).  Returns NULL if memory runs out. */
oracle_table* oracle_build(const int32_t* r_key, const int32_t* r_rid, uint64_t n_r) {
    oracle_table* t = (oracle_table*)calloc(1, sizeof(oracle_table));
    if (!t) return NULL;
    uint64_t nb = 1;
    while (nb < n_r) nb <<= 1;
    t->nbuckets = nb;
    t->buckets = (bucket_header*)malloc(nb * sizeof(bucket_header));
    t->keys = (key_node*)malloc((n_r ? n_r : 1) * sizeof(key_node));
    t->rids = (rid_node*)malloc((n_r ? n_r : 1) * sizeof(rid_node));
    if (!t->buckets || !t->keys || !t->rids) {
        oracle_free(t);
        return NULL;
    }
    for (uint64_t b = 0; b < nb; ++b) {
        t->buckets[b].count = 0;
        t->buckets[b].key_head = -1;
    }
    for (uint64_t i = 0; i < n_r; ++i) {
        const int32_t key = r_key[i];
        bucket_header* hdr = &t->buckets[bucket_of(t, key)];   /* b1, b2 */
        int32_t kn = hdr->key_head;                             /* b3 */
        while (kn >= 0 && t->keys[kn].key != key) kn = t->keys[kn].next;
        if (kn < 0) {
            kn = (int32_t)t->nkeys++;
            t->keys[kn].key = key;
            t->keys[kn].next = hdr->key_head;
            t->keys[kn].rid_head = -1;
            t->keys[kn].rid_tail = -1;
            hdr->key_head = kn;
        }
        const int32_t rn = (int32_t)t->nrids++;                 /* b4 */
        t->rids[rn].rid = r_rid[i];
        t->rids[rn].next = -1;
        if (t->keys[kn].rid_tail < 0)
            t->keys[kn].rid_head = rn;
        else
            t->rids[t->keys[kn].rid_tail].next = rn;
        t->keys[kn].rid_tail = rn;
        hdr->count += 1;
    }
    return t;
}

static int32_t find_key(const oracle_table* t, int32_t key) {
    const bucket_header* hdr = &t->buckets[bucket_of(t, key)];  /* p1, p2 */
    int32_t kn = hdr->key_head;                                 /* p3 */
    while (kn >= 0 && t->keys[kn].key != key) kn = t->keys[kn].next;
    return kn;
}

/* Number of result pairs for probing with S (p1-p4 without output). */
uint64_t oracle_probe_count(const oracle_table* t, const int32_t* s_key, uint64_t n_s) {
    uint64_t total = 0;
    for (uint64_t j = 0; j < n_s; ++j) {
        const int32_t kn = find_key(t, s_key[j]);
        if (kn < 0) continue;
        for (int32_t rn = t->keys[kn].rid_head; rn >= 0; rn = t->rids[rn].next) total += 1;
    }
    return total;
}

/* Probes with S (p1-p4) and writes up to `capacity` pairs in probe order.
   Returns the total number of pairs, which may exceed `capacity`. */
uint64_t oracle_probe_emit(const oracle_table* t, const int32_t* s_key, const int32_t* s_rid,
                           uint64_t n_s, int32_t* out_r, int32_t* out_s, uint64_t capacity) {
    uint64_t total = 0;
    for (uint64_t j = 0; j < n_s; ++j) {
        const int32_t kn = find_key(t, s_key[j]);
        if (kn < 0) continue;
        for (int32_t rn = t->keys[kn].rid_head; rn >= 0; rn = t->rids[rn].next) {   /* p4 */
            if (total < capacity) {
                out_r[total] = t->rids[rn].rid;
                out_s[total] = s_rid[j];
            }
            total += 1;
        }
    }
    return total;
}

/* Introspection for tests: bucket count, distinct keys, and a bucket's tuple count. */
uint64_t oracle_nbuckets(const oracle_table* t) { return t->nbuckets; }
int64_t oracle_nkeys(const oracle_table* t) { return t->nkeys; }
uint32_t oracle_bucket_count(const oracle_table* t, uint64_t b) { return t->buckets[b].count; }
uint32_t oracle_hash(int32_t key) { return murmur2_key(key, ORACLE_SEED); }
uint32_t oracle_murmur2(int32_t key, uint32_t seed) { return murmur2_key(key, seed); }
