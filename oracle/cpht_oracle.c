/*
 * Sequential CPU oracle for compact bucketed cuckoo hashing and compact
 * two-level iceberg hashing ("Compact Parallel Hash Tables on the GPU",
 * Hegeman, Woltgens, Wijs, Laarman, arXiv 2406.09255).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow, obviously correct
 * model the GPU library is checked against.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, constant table or generator with the GPU library; the two
 * sides implement the same published definitions independently.
 *
 * Everything here is integer arithmetic.  One operation at a time, one slot
 * at a time, no blocking and no reordering beyond what the paper states.
 *
 * Contents
 *   1. splitmix64 (Vigna's public-domain generator), used only to expand a
 *      64-bit seed into permutation constants and cuckoo victim choices.
 *   2. The quotienting permutation pi_i and its inverse (Sec. 2.4; the
 *      permutation family itself is not given in the paper, Sec. 4.3, so a
 *      seeded xor-shift/multiply bijection is used).
 *   3. Slot encoding: EMPTY is the all-zero word; an occupied slot holds an
 *      occupancy bit, a tag (hash index j for cuckoo, Sec. 2.2 / Alg. 4; the
 *      secondary index for iceberg, Sec. 3 Alg. 1) and the remainder
 *      (Sec. 2.4), or the full permuted key for a non-compact table.  A
 *      deleted key leaves a tombstone, the word 1 (occupancy bit clear): a
 *      slot that is not EMPTY but holds no key, so the non-empty slots of an
 *      iceberg bucket stay consecutive (Sec. 2.2 "Lookup", Sec. 3
 *      "Limitations").
 *   4. Iceberg find-or-put, run sequentially as the simplified find-or-put of
 *      Appendix A (Alg. 5) over the slot order of Definition 1.
 *   5. Iceberg lookup (Sec. 2.3 "Lookup", levels 1 and 2).
 *   6. Compact cuckoo put (Sec. 4.4, Alg. 4) and lookup (Sec. 4.4 "Lookup").
 *   6b. Delete by tombstone, both schemes.
 *   4b. The third iceberg level (Sec. 2.3: linked lists outside the table,
 *      the list chosen by h_0(k)): lists of 128-byte slabs taken from a
 *      fixed pool; a key goes there only when its primary bucket and both
 *      secondary buckets are full.
 *   7. A table checker for raw table images (well-formedness and the order
 *      property of Appendix A Definition 2, no duplicates (Lemma 1), prefix
 *      filling of iceberg buckets, and the cuckoo early-exit invariant of
 *      Sec. 2.2 / 4.4).
 *
 * Parity unpinned: the load at which the first FULL answer appears (and the
 * fill reached after it) depends on the permutations, the chain bound C and
 * the victim rule; the paper gives only soft bounds (cuckoo with 16 or 32
 * slots per bucket reaches 0.95, iceberg with 32 primary slots 0.9), which
 * the tests check, and the GPU's value is reported beside this model's.
 *
 * Raw table image layout (shared contract with the GPU library, documented in
 * the public header): level x is an array of 2^nb_x buckets of B_x slots of
 * s_x bits; slot q of bucket b sits at byte offset (b*B_x + q)*s_x/8, little
 * endian.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>

/* ------------------------------------------------------------------------ */
/* 1. splitmix64                                                            */
/* ------------------------------------------------------------------------ */

/* Output function of splitmix64 (Steele, Lea, Flood; Vigna's reference C). */
uint64_t or_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* The (i+1)-th output of splitmix64 started from state `seed`: the state
 * advances by the golden-ratio increment before every output. */
uint64_t or_sm64(uint64_t seed, uint64_t i)
{
    return or_mix64(seed + (i + 1) * 0x9E3779B97F4A7C15ULL);
}

/* ------------------------------------------------------------------------ */
/* 2. Permutations pi_i on w-bit strings (Sec. 2.4)                         */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint32_t w;        /* key width in bits, 1..64 */
    uint32_t h;        /* xor-shift distance ceil(w/2) */
    uint64_t mask;     /* 2^w - 1 */
    uint64_t m[3];     /* odd multipliers mod 2^w */
    uint64_t minv[3];  /* their inverses mod 2^w */
    uint64_t c[3];     /* xor constants (w bits) */
} or_perm_t;

static uint64_t wmask(uint32_t w) { return w >= 64 ? ~0ULL : ((1ULL << w) - 1); }

/* Inverse of an odd m modulo 2^64 (then masked to 2^w): Newton-Hensel
 * iteration y <- y*(2 - m*y), which doubles the number of correct low bits
 * each step; y = m is correct to 3 bits, so 5 steps give 96 >= 64 bits. */
uint64_t or_mulinv(uint64_t m, uint32_t w)
{
    uint64_t y = m;
    for (int it = 0; it < 5; ++it) y = y * (2 - m * y);
    return y & wmask(w);
}

/* Permutation number i in {0,1,2} of the family seeded by `seed`:
 * m_q = (sm64(seed, 3i+q) | 1) mod 2^w and c_q = sm64(seed, 9+3i+q) mod 2^w. */
void or_perm_init(or_perm_t* p, uint32_t w, uint64_t seed, uint32_t i)
{
    p->w = w;
    p->h = (w + 1) / 2;
    p->mask = wmask(w);
    for (uint32_t q = 0; q < 3; ++q) {
        p->m[q] = (or_sm64(seed, 3 * i + q) | 1ULL) & p->mask;
        p->c[q] = or_sm64(seed, 9 + 3 * i + q) & p->mask;
        p->minv[q] = or_mulinv(p->m[q], w);
    }
}

/* pi(x): three rounds of (x ^= x >> h; x *= m_q; x ^= c_q) mod 2^w, then a
 * final x ^= x >> h.  Each step is a bijection on w-bit strings: the shift is
 * by h >= w/2 so x ^ (x >> h) is its own inverse, m_q is odd, and xor with a
 * constant is an involution. */
uint64_t or_perm(const or_perm_t* p, uint64_t x)
{
    x &= p->mask;
    for (int q = 0; q < 3; ++q) {
        x ^= x >> p->h;
        x = (x * p->m[q]) & p->mask;
        x ^= p->c[q];
    }
    x ^= x >> p->h;
    return x;
}

/* pi^{-1}: the steps of or_perm undone in reverse order. */
uint64_t or_unperm(const or_perm_t* p, uint64_t y)
{
    y &= p->mask;
    y ^= y >> p->h;
    for (int q = 2; q >= 0; --q) {
        y ^= p->c[q];
        y = (y * p->minv[q]) & p->mask;
        y ^= y >> p->h;
    }
    return y;
}

/* Array form for the tests: out[k] = pi_i(in[k]) or pi_i^{-1}(in[k]). */
int or_perm_apply(uint32_t w, uint64_t seed, uint32_t i, int inverse,
                  const uint64_t* in, uint64_t* out, uint64_t n)
{
    if (w < 1 || w > 64 || i > 2) return -1;
    or_perm_t p;
    or_perm_init(&p, w, seed, i);
    for (uint64_t k = 0; k < n; ++k) out[k] = inverse ? or_unperm(&p, in[k]) : or_perm(&p, in[k]);
    return 0;
}

/* Expose the constants so a test can check m*minv == 1 (mod 2^w). */
int or_perm_constants(uint32_t w, uint64_t seed, uint32_t i, uint64_t* m3, uint64_t* minv3, uint64_t* c3)
{
    if (w < 1 || w > 64 || i > 2) return -1;
    or_perm_t p;
    or_perm_init(&p, w, seed, i);
    for (int q = 0; q < 3; ++q) { m3[q] = p.m[q]; minv3[q] = p.minv[q]; c3[q] = p.c[q]; }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 3. Table configuration and slot encoding                                 */
/* ------------------------------------------------------------------------ */

enum { OR_CUCKOO = 0, OR_ICEBERG = 1 };
enum { OR_NONE = 0, OR_PUT = 1, OR_FOUND = 2, OR_FULL = 3 };
#define OR_TOMB 1ULL /* tombstone: not EMPTY, occupancy bit clear, matches no stored form */

/* Field order mirrors the ctypes structure in oracle/__init__.py. */
typedef struct {
    uint32_t scheme;       /* OR_CUCKOO or OR_ICEBERG */
    uint32_t w;            /* key bits */
    uint32_t log2_slots0;  /* cuckoo: all slots; iceberg: primary level */
    uint32_t log2_slots1;  /* iceberg: secondary level */
    uint32_t B0, B1;       /* slots per bucket */
    uint32_t s0, s1;       /* slot bits: 16, 32 or 64 */
    uint32_t H;            /* cuckoo hash functions (2..3) */
    uint32_t C;            /* cuckoo eviction chain bound */
    uint32_t compact;      /* 1: store remainders; 0: store the full pi(k) */
    uint32_t log2_lists;   /* iceberg level 3: number of lists (log2) */
    uint32_t pool_slabs;   /* iceberg level 3: slabs in the pool; 0 = two levels only */
    uint32_t pad;
    uint64_t seed;
} or_cfg_t;

typedef struct {
    uint32_t nb;      /* log2 number of buckets */
    uint32_t B;       /* slots per bucket */
    uint32_t s;       /* slot bits */
    uint32_t pbits;   /* payload bits: remainder (w - nb) or full key (w) */
    uint32_t tbits;   /* tag bits */
    uint64_t nslots;
    uint64_t* slot;   /* one 64-bit word per slot, holding the s-bit value */
} or_level_t;

/* Level 3: 2^log2_lists lists, each a chain of slabs of 128 bytes.  A slab
 * has B slots of s bits (s = 32, or 64 for 64-bit primary slots); its last
 * slot holds the id of the next slab (0 = end of list).  Slab ids count from
 * 1; slab id sits at pool position id - 1.  Addressing and encoding are a
 * level's: the list is the high log2_lists bits of pi_0(k), the stored form
 * the occupancy bit and the remaining bits (all w bits if not compact). */
typedef struct {
    int on;
    or_level_t L;      /* nb = log2_lists, B = slots per slab, slot = the pool */
    uint64_t nlists;
    uint32_t nslabs;   /* pool capacity */
    uint32_t used;     /* slabs handed out so far */
    uint64_t* head;    /* first slab id of each list */
} or_l3_t;

typedef struct {
    or_cfg_t cfg;
    or_perm_t perm[3];
    or_level_t lv[2];
    or_l3_t l3;
    int nlevels;
    uint32_t line_bytes;
} or_table_t;

static uint32_t ilog2u(uint64_t v) { uint32_t r = 0; while ((1ULL << r) < v) ++r; return r; }
static int is_pow2(uint64_t v) { return v && !(v & (v - 1)); }

/* Tag bits: cuckoo stores the hash index j < H (ceil(log2 H) bits); the
 * iceberg secondary level stores which of the two secondary buckets (1 bit);
 * the iceberg primary level stores no tag. */
static int level_init(or_level_t* L, const or_cfg_t* c, uint32_t log2_slots, uint32_t B,
                      uint32_t s, uint32_t tbits)
{
    if (!is_pow2(B) || (1ULL << log2_slots) < B) return -1;
    if (s != 16 && s != 32 && s != 64) return -1;
    L->B = B;
    L->s = s;
    L->nb = log2_slots - ilog2u(B);
    if (L->nb > c->w) return -1;
    L->pbits = c->compact ? c->w - L->nb : c->w;
    L->tbits = tbits;
    if (L->pbits + L->tbits + 1 > s) return -1; /* remainder + tag + occupancy must fit */
    L->nslots = 1ULL << log2_slots;
    L->slot = (uint64_t*)calloc(L->nslots, sizeof(uint64_t));
    return L->slot ? 0 : -2;
}

/* Largest key width the level can store: log2(#buckets) address bits are
 * implied by the bucket, and the slot holds remainder + tag + occupancy bit
 * (Sec. 5.1: 2^22 buckets and 16-bit slots give 22 + 15 = 37 bits). */
uint32_t or_max_key_bits(uint32_t log2_slots, uint32_t B, uint32_t s, uint32_t tbits, uint32_t compact)
{
    uint32_t nb = log2_slots - ilog2u(B);
    if (s < tbits + 1) return 0;
    uint32_t room = s - 1 - tbits;
    uint32_t w = compact ? nb + room : room;
    return w > 64 ? 64 : w;
}

or_table_t* or_new(const or_cfg_t* c)
{
    if (c->w < 1 || c->w > 64) return NULL;
    or_table_t* t = (or_table_t*)calloc(1, sizeof(or_table_t));
    if (!t) return NULL;
    t->cfg = *c;
    t->line_bytes = 128;
    int err = 0;
    if (c->scheme == OR_CUCKOO) {
        if (c->H < 2 || c->H > 3 || c->C < 1) err = -1;
        else err = level_init(&t->lv[0], c, c->log2_slots0, c->B0, c->s0, ilog2u(c->H));
        t->nlevels = 1;
        for (uint32_t j = 0; j < 3; ++j) or_perm_init(&t->perm[j], c->w, c->seed, j);
    } else if (c->scheme == OR_ICEBERG) {
        err = level_init(&t->lv[0], c, c->log2_slots0, c->B0, c->s0, 0);
        if (!err) err = level_init(&t->lv[1], c, c->log2_slots1, c->B1, c->s1, 1);
        if (!err && c->pool_slabs > 0) {
            or_l3_t* q = &t->l3;
            uint32_t s3 = c->s0 == 64 ? 64 : 32;
            uint32_t b3 = 1024 / s3;
            q->L.B = b3;
            q->L.s = s3;
            q->L.nb = c->log2_lists;
            q->L.pbits = c->compact ? c->w - c->log2_lists : c->w;
            q->L.tbits = 0;
            if (c->log2_lists > c->w || c->log2_lists > 30 || q->L.pbits + 1 > s3) err = -1;
            if (!err) {
                q->L.nslots = (uint64_t)c->pool_slabs * b3;
                q->L.slot = (uint64_t*)calloc(q->L.nslots, sizeof(uint64_t));
                q->nlists = 1ULL << c->log2_lists;
                q->head = (uint64_t*)calloc(q->nlists, sizeof(uint64_t));
                q->nslabs = c->pool_slabs;
                q->on = 1;
                if (!q->L.slot || !q->head) err = -2;
            }
        }
        t->nlevels = 2;
        for (uint32_t j = 0; j < 3; ++j) or_perm_init(&t->perm[j], c->w, c->seed, j);
    } else {
        err = -1;
    }
    if (err) {
        free(t->lv[0].slot);
        free(t->lv[1].slot);
        free(t->l3.L.slot);
        free(t->l3.head);
        free(t);
        return NULL;
    }
    return t;
}

void or_free(or_table_t* t)
{
    if (!t) return;
    free(t->lv[0].slot);
    free(t->lv[1].slot);
    free(t->l3.L.slot);
    free(t->l3.head);
    free(t);
}

/* Address a_i(k): the high nb bits of pi_i(k) (Sec. 2.4 "the first N bits"). */
static uint64_t addr_of(const or_table_t* t, const or_level_t* L, uint32_t i, uint64_t k)
{
    uint64_t x = or_perm(&t->perm[i], k);
    return L->nb == 0 ? 0 : x >> (t->cfg.w - L->nb);
}

/* Stored form r'_i(k) with tag `tag`: occupancy bit | tag << pbits | payload,
 * where the payload is the remainder r_i(k) (the low w-nb bits of pi_i(k))
 * for a compact table, or all w bits of pi_i(k) for a non-compact one. */
static uint64_t enc_of(const or_table_t* t, const or_level_t* L, uint32_t i, uint64_t k, uint64_t tag)
{
    uint64_t x = or_perm(&t->perm[i], k);
    uint64_t payload = x & wmask(L->pbits);
    return (1ULL << (L->s - 1)) | (tag << L->pbits) | payload;
}

/* Inverse of the above: the key stored in bucket b as slot value v under
 * permutation i (Sec. 2.4: k = pi^{-1}(a(k).r(k))). */
static uint64_t dec_of(const or_table_t* t, const or_level_t* L, uint32_t i, uint64_t b, uint64_t v)
{
    uint64_t payload = v & wmask(L->pbits);
    uint64_t x = t->cfg.compact ? ((L->nb == 0 ? 0 : (b << (t->cfg.w - L->nb))) | payload) : payload;
    return or_unperm(&t->perm[i], x);
}

static uint64_t tag_of(const or_level_t* L, uint64_t v) { return (v >> L->pbits) & wmask(L->tbits); }

static uint64_t* bucket_ptr(or_level_t* L, uint64_t b) { return L->slot + b * L->B; }

/* A slot value holds a key iff its occupancy bit is set (EMPTY and the
 * tombstone both have it clear). */
static int holds_key(const or_level_t* L, uint64_t v) { return (int)((v >> (L->s - 1)) & 1); }

/* Cache lines touched by reading one whole bucket. */
static uint32_t bucket_lines(const or_table_t* t, const or_level_t* L)
{
    uint64_t bytes = (uint64_t)L->B * L->s / 8;
    return (uint32_t)((bytes + t->line_bytes - 1) / t->line_bytes);
}

/* ------------------------------------------------------------------------ */
/* 4. Iceberg find-or-put: Appendix A, Definition 1 and Alg. 5               */
/* ------------------------------------------------------------------------ */

/* Slot identities of Definition 1: x = 0 is the primary bucket, x = 1 and
 * x = 2 the first and second secondary bucket; y is the row in the bucket. */
typedef struct { uint32_t x, y; } or_sid_t;

/* The well-order of Definition 1:
 *   (0,x) < (1+y,z) for all x, y, z;
 *   (x,y) < (x,z) iff y < z;
 *   (1,x) < (2,y) iff x < y   (so on equal rows the second bucket comes first).
 * Returns 1 iff a strictly precedes b. */
int or_order_less(uint32_t ax, uint32_t ay, uint32_t bx, uint32_t by)
{
    if (ax == 0 && bx != 0) return 1;
    if (ax != 0 && bx == 0) return 0;
    if (ax == bx) return ay < by;
    if (ax == 1 && bx == 2) return ay < by;
    /* ax == 2, bx == 1: (2,ay) < (1,by) iff not (1,by) < (2,ay), the pairs being distinct */
    return !(by < ay);
}

/* All slot identities for bucket sizes B0, B1, sorted by the order above
 * (insertion sort using or_order_less only).  Returns the count. */
int or_order_list(uint32_t B0, uint32_t B1, uint32_t* xs, uint32_t* ys)
{
    int n = 0;
    for (uint32_t y = 0; y < B0; ++y) { xs[n] = 0; ys[n] = y; ++n; }
    for (uint32_t x = 1; x <= 2; ++x)
        for (uint32_t y = 0; y < B1; ++y) { xs[n] = x; ys[n] = y; ++n; }
    for (int i = 1; i < n; ++i) {
        uint32_t kx = xs[i], ky = ys[i];
        int j = i - 1;
        while (j >= 0 && or_order_less(kx, ky, xs[j], ys[j])) { xs[j + 1] = xs[j]; ys[j + 1] = ys[j]; --j; }
        xs[j + 1] = kx; ys[j + 1] = ky;
    }
    return n;
}

/* Everything the sequential model needs about key k: its three buckets and
 * the stored forms r'_0(k) = r_0(k), r'_1(k) = (r_1(k), 0), r'_2(k) = (r_2(k), 1). */
typedef struct {
    uint64_t a[3];
    uint64_t e[3];
} or_ice_key_t;

static void ice_key(const or_table_t* t, uint64_t k, or_ice_key_t* q)
{
    const or_level_t* L0 = &t->lv[0];
    const or_level_t* L1 = &t->lv[1];
    q->a[0] = addr_of(t, L0, 0, k);
    q->e[0] = enc_of(t, L0, 0, k, 0);
    q->a[1] = addr_of(t, L1, 1, k);
    q->e[1] = enc_of(t, L1, 1, k, 0);
    q->a[2] = addr_of(t, L1, 2, k);
    q->e[2] = enc_of(t, L1, 2, k, 1);
}

/* Slot (x,y) for key q: T_sg(x)[a_x(k)][y]. */
static uint64_t* ice_slot(or_table_t* t, const or_ice_key_t* q, uint32_t x, uint32_t y)
{
    or_level_t* L = &t->lv[x == 0 ? 0 : 1];
    return bucket_ptr(L, q->a[x]) + y;
}

/* ---- 4b. Level 3 ---------------------------------------------------- */

static uint64_t* l3_slab(or_table_t* t, uint64_t id) { return t->l3.L.slot + (id - 1) * t->l3.L.B; }

/* Find-or-put in k's list: slots in list order (slab by slab, slot by slot);
 * k's stored form before the first empty slot -> FOUND, else the first empty
 * slot takes it -> PUT; a full last slab gets a new slab from the pool, FULL
 * when the pool is used up. */
static int l3_fop(or_table_t* t, uint64_t k, uint32_t* lines)
{
    or_level_t* L = &t->l3.L;
    const uint64_t e = enc_of(t, L, 0, k, 0);
    const uint32_t nslot = L->B - 1;
    uint64_t* link = &t->l3.head[addr_of(t, L, 0, k)];
    for (;;) {
        if (*link == 0) {
            if (t->l3.used == t->l3.nslabs) return OR_FULL;
            *link = ++t->l3.used;
        }
        uint64_t* sb = l3_slab(t, *link);
        if (lines) ++*lines;
        for (uint32_t i = 0; i < nslot; ++i) {
            if (sb[i] == e) return OR_FOUND;
            if (sb[i] == 0) { sb[i] = e; return OR_PUT; }
        }
        link = &sb[nslot];
    }
}

/* The slot of k's list holding k's stored form, or NULL (the walk stops at
 * an empty slot: slots fill in list order). */
static uint64_t* l3_lookup(or_table_t* t, uint64_t k, uint32_t* lines)
{
    or_level_t* L = &t->l3.L;
    const uint64_t e = enc_of(t, L, 0, k, 0);
    const uint32_t nslot = L->B - 1;
    uint64_t id = t->l3.head[addr_of(t, L, 0, k)];
    while (id) {
        uint64_t* sb = l3_slab(t, id);
        if (lines) ++*lines;
        for (uint32_t i = 0; i < nslot; ++i) {
            if (sb[i] == e) return &sb[i];
            if (sb[i] == 0) return NULL;
        }
        id = sb[nslot];
    }
    return NULL;
}

/* One find-or-put, sequentially (Alg. 5): look at every slot of the key's
 * three buckets; if one holds r'_x(k) the result is FOUND; if none is empty
 * the result is FULL; otherwise write r'_x(k) into the least empty slot under
 * the order of Definition 1 and return PUT.  `order` is the sorted slot list. */
static int ice_fop_one(or_table_t* t, uint64_t k, const uint32_t* ox, const uint32_t* oy, int nord,
                       uint32_t* lines)
{
    or_ice_key_t q;
    ice_key(t, k, &q);
    int full_primary = 1;
    for (uint32_t y = 0; y < t->cfg.B0; ++y)
        if (*ice_slot(t, &q, 0, y) == 0) full_primary = 0;
    /* Bucket reads as the two-level algorithm (Alg. 1) performs them: the
     * primary always, both secondaries only once the primary is full. */
    if (lines) {
        int found0 = 0;
        for (uint32_t y = 0; y < t->cfg.B0; ++y)
            if (*ice_slot(t, &q, 0, y) == q.e[0]) found0 = 1;
        *lines = bucket_lines(t, &t->lv[0]);
        if (!found0 && full_primary) *lines += 2 * bucket_lines(t, &t->lv[1]);
    }
    for (int i = 0; i < nord; ++i)
        if (*ice_slot(t, &q, ox[i], oy[i]) == q.e[ox[i]]) return OR_FOUND;
    for (int i = 0; i < nord; ++i) {
        uint64_t* s = ice_slot(t, &q, ox[i], oy[i]);
        if (*s == 0) {
            *s = q.e[ox[i]];
            return OR_PUT;
        }
    }
    /* all three buckets full without k: the third level, if there is one */
    return t->l3.on ? l3_fop(t, k, lines) : OR_FULL;
}

/* Iceberg lookup (Sec. 2.3 "Lookup", levels 1 and 2): the primary bucket
 * decides unless it is full and lacks k; then the two secondary buckets
 * decide (a key is absent if neither holds its tagged remainder). */
static int ice_find_one(or_table_t* t, uint64_t k, uint32_t* lines)
{
    or_ice_key_t q;
    ice_key(t, k, &q);
    if (lines) *lines = bucket_lines(t, &t->lv[0]);
    int has_empty = 0;
    for (uint32_t y = 0; y < t->cfg.B0; ++y) {
        uint64_t v = *ice_slot(t, &q, 0, y);
        if (v == q.e[0]) return 1;
        if (v == 0) has_empty = 1;
    }
    if (has_empty) return 0;
    if (lines) *lines += 2 * bucket_lines(t, &t->lv[1]);
    int room = 0;
    for (uint32_t x = 1; x <= 2; ++x)
        for (uint32_t y = 0; y < t->cfg.B1; ++y) {
            uint64_t v = *ice_slot(t, &q, x, y);
            if (v == q.e[x]) return 1;
            if (v == 0) room = 1;
        }
    /* k reaches level 3 only through two full secondary buckets */
    if (room || !t->l3.on) return 0;
    return l3_lookup(t, k, lines) != NULL;
}

/* ------------------------------------------------------------------------ */
/* 6. Compact cuckoo (Sec. 2.2 and Sec. 4.4, Alg. 4)                        */
/* ------------------------------------------------------------------------ */

/* Victim row when bucket T[a] is full (Alg. 4 leaves the rule open: "based
 * on c, k"): the low log2(B) bits of splitmix64 seeded with k ^ (c << 32). */
static uint32_t ck_victim(uint64_t k, uint32_t c, uint32_t B)
{
    return (uint32_t)(or_sm64(k ^ ((uint64_t)c << 32), 0) & (B - 1));
}

/* Alg. 4, one key, sequentially.  j is the hash index the carried key k is
 * tried with; a Swap leaves the evicted pair in the locals, whose key is
 * recovered by the inverse permutation of its own stored index and then
 * continues with the next hash function.  After C rounds the carried key is
 * dropped and the result is FULL. */
static int ck_put_one(or_table_t* t, uint64_t k, uint32_t* lines)
{
    or_level_t* L = &t->lv[0];
    const uint32_t H = t->cfg.H;
    uint32_t j = 0;
    if (lines) *lines = 0;
    for (uint32_t c = 1; c <= t->cfg.C; ++c) {
        uint64_t a = addr_of(t, L, j, k);
        uint64_t v = enc_of(t, L, j, k, j);
        uint64_t* b = bucket_ptr(L, a);
        if (lines) *lines += bucket_lines(t, L);
        for (uint32_t i = 0; i < L->B; ++i) {
            if (b[i] == 0) {
                b[i] = v;
                return OR_PUT;
            }
        }
        uint32_t i = ck_victim(k, c, L->B);
        uint64_t old = b[i];
        b[i] = v;
        if (!holds_key(L, old)) return OR_PUT; /* the victim was a tombstone: nothing to carry */
        uint32_t jj = (uint32_t)tag_of(L, old);
        k = dec_of(t, L, jj, a, old);
        j = (jj + 1) % H;
    }
    return OR_FULL;
}

/* Cuckoo lookup (Sec. 2.2 "Lookup", Sec. 4.4): try a_0(k), a_1(k), ... in
 * order; stop at the bucket holding (r_j(k), j), or at the first bucket that
 * is not full (k can then not be further on). */
static int ck_find_one(or_table_t* t, uint64_t k, uint32_t* lines)
{
    or_level_t* L = &t->lv[0];
    if (lines) *lines = 0;
    for (uint32_t j = 0; j < t->cfg.H; ++j) {
        uint64_t a = addr_of(t, L, j, k);
        uint64_t v = enc_of(t, L, j, k, j);
        uint64_t* b = bucket_ptr(L, a);
        if (lines) *lines += bucket_lines(t, L);
        int has_empty = 0;
        for (uint32_t i = 0; i < L->B; ++i) {
            if (b[i] == v) return 1;
            if (b[i] == 0) has_empty = 1;
        }
        if (has_empty) return 0;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 6b. Delete by tombstone                                                  */
/* ------------------------------------------------------------------------ */

/* Delete k: the slot holding k's stored form (in any of the buckets k may
 * occupy: a_0..a_{H-1} for cuckoo; primary and both secondaries for iceberg)
 * becomes a tombstone.  A key is stored at most once, so the first match is
 * the only one.  Returns 1 if k was stored, else 0.  Tombstones are never
 * written back to EMPTY: lookups and the prefix rule treat them as occupied,
 * find-or-put and the first-empty claim never reuse them, and a cuckoo
 * eviction that picks one as its victim simply overwrites it. */
static int del_one(or_table_t* t, uint64_t k)
{
    if (t->cfg.scheme == OR_ICEBERG) {
        or_ice_key_t q;
        ice_key(t, k, &q);
        for (uint32_t x = 0; x <= 2; ++x) {
            uint32_t By = x == 0 ? t->cfg.B0 : t->cfg.B1;
            for (uint32_t y = 0; y < By; ++y) {
                uint64_t* s = ice_slot(t, &q, x, y);
                if (*s == q.e[x]) { *s = OR_TOMB; return 1; }
            }
        }
        if (t->l3.on) {
            uint64_t* s = l3_lookup(t, k, NULL);
            if (s) { *s = OR_TOMB; return 1; }
        }
        return 0;
    }
    or_level_t* L = &t->lv[0];
    for (uint32_t j = 0; j < t->cfg.H; ++j) {
        uint64_t* b = bucket_ptr(L, addr_of(t, L, j, k));
        uint64_t v = enc_of(t, L, j, k, j);
        for (uint32_t i = 0; i < L->B; ++i)
            if (b[i] == v) { b[i] = OR_TOMB; return 1; }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Batch entry points (operations applied one after another, in order)      */
/* ------------------------------------------------------------------------ */

/* Insert: iceberg find-or-put (PUT/FOUND/FULL) or cuckoo put (PUT/FULL). */
int or_insert(or_table_t* t, const uint64_t* keys, uint64_t n, uint8_t* out, uint32_t* lines)
{
    if (t->cfg.scheme == OR_ICEBERG) {
        uint32_t nmax = t->cfg.B0 + 2 * t->cfg.B1;
        uint32_t* ox = (uint32_t*)malloc(nmax * sizeof(uint32_t));
        uint32_t* oy = (uint32_t*)malloc(nmax * sizeof(uint32_t));
        if (!ox || !oy) { free(ox); free(oy); return -2; }
        int nord = or_order_list(t->cfg.B0, t->cfg.B1, ox, oy);
        for (uint64_t i = 0; i < n; ++i)
            out[i] = (uint8_t)ice_fop_one(t, keys[i], ox, oy, nord, lines ? lines + i : NULL);
        free(ox);
        free(oy);
    } else {
        for (uint64_t i = 0; i < n; ++i) out[i] = (uint8_t)ck_put_one(t, keys[i], lines ? lines + i : NULL);
    }
    return 0;
}

int or_find(or_table_t* t, const uint64_t* keys, uint64_t n, uint8_t* out, uint32_t* lines)
{
    for (uint64_t i = 0; i < n; ++i) {
        uint32_t* l = lines ? lines + i : NULL;
        out[i] = (uint8_t)(t->cfg.scheme == OR_ICEBERG ? ice_find_one(t, keys[i], l) : ck_find_one(t, keys[i], l));
    }
    return 0;
}

int or_delete(or_table_t* t, const uint64_t* keys, uint64_t n, uint8_t* out)
{
    for (uint64_t i = 0; i < n; ++i) out[i] = (uint8_t)del_one(t, keys[i]);
    return 0;
}

/* Mixed batch: op 0 = find (answer 0/1), op 1 = insert (PUT/FOUND/FULL),
 * applied in index order.  Iceberg only: cuckoo is static (Sec. 4.4). */
int or_mixed(or_table_t* t, const uint64_t* keys, const uint8_t* ops, uint64_t n, uint8_t* out)
{
    if (t->cfg.scheme != OR_ICEBERG) return -1;
    uint32_t nmax = t->cfg.B0 + 2 * t->cfg.B1;
    uint32_t* ox = (uint32_t*)malloc(nmax * sizeof(uint32_t));
    uint32_t* oy = (uint32_t*)malloc(nmax * sizeof(uint32_t));
    if (!ox || !oy) { free(ox); free(oy); return -2; }
    int nord = or_order_list(t->cfg.B0, t->cfg.B1, ox, oy);
    for (uint64_t i = 0; i < n; ++i)
        out[i] = (uint8_t)(ops[i] ? ice_fop_one(t, keys[i], ox, oy, nord, NULL) : ice_find_one(t, keys[i], NULL));
    free(ox);
    free(oy);
    return 0;
}

/* Slots holding a key over all levels (the numerator of the fill factor,
 * Sec. 2.1; tombstones hold no key). */
uint64_t or_occupied(const or_table_t* t)
{
    uint64_t c = 0;
    for (int x = 0; x < t->nlevels; ++x)
        for (uint64_t i = 0; i < t->lv[x].nslots; ++i) c += (uint64_t)holds_key(&t->lv[x], t->lv[x].slot[i]);
    if (t->l3.on)  /* link slots hold slab ids < 2^31: never an occupancy bit */
        for (uint64_t i = 0; i < t->l3.L.nslots; ++i) c += (uint64_t)holds_key(&t->l3.L, t->l3.L.slot[i]);
    return c;
}

/* Tombstones over all levels. */
uint64_t or_tombstones(const or_table_t* t)
{
    uint64_t c = 0;
    for (int x = 0; x < t->nlevels; ++x)
        for (uint64_t i = 0; i < t->lv[x].nslots; ++i) c += t->lv[x].slot[i] == OR_TOMB;
    if (t->l3.on)
        for (uint64_t i = 0; i < t->l3.L.nslots; ++i)
            c += (i % t->l3.L.B != t->l3.L.B - 1) && t->l3.L.slot[i] == OR_TOMB;
    return c;
}

/* Slabs of level 3 handed out so far. */
uint32_t or_l3_used(const or_table_t* t) { return t->l3.used; }

uint64_t or_capacity(const or_table_t* t)
{
    uint64_t c = 0;
    for (int x = 0; x < t->nlevels; ++x) c += t->lv[x].nslots;
    return c;
}

/* Raw images: level 0 primary, level 1 secondary, level 2 the level-3
 * slab pool (pool_slabs x 128 bytes, slot layout as the other levels, the
 * last slot of a slab holding the next slab id), level 3 the list heads
 * (one little-endian uint32 slab id per list). */
static or_level_t* image_level(or_table_t* t, int level)
{
    if (level >= 0 && level < t->nlevels) return &t->lv[level];
    if (level == 2 && t->l3.on) return &t->l3.L;
    return NULL;
}

uint64_t or_level_bytes(const or_table_t* t, int level)
{
    if (level == 3) return t->l3.on ? t->l3.nlists * 4 : 0;
    const or_level_t* L = image_level((or_table_t*)t, level);
    return L ? L->nslots * L->s / 8 : 0;
}

/* Write level `level` into dst as a raw image (layout in the file header). */
int or_export(const or_table_t* t, int level, void* dst, uint64_t bytes)
{
    uint8_t* d = (uint8_t*)dst;
    if (bytes != or_level_bytes(t, level) || bytes == 0) return -1;
    if (level == 3) {
        for (uint64_t h = 0; h < t->l3.nlists; ++h)
            for (uint32_t byte = 0; byte < 4; ++byte) d[h * 4 + byte] = (uint8_t)(t->l3.head[h] >> (8 * byte));
        return 0;
    }
    const or_level_t* L = image_level((or_table_t*)t, level);
    uint32_t sb = L->s / 8;
    for (uint64_t i = 0; i < L->nslots; ++i)
        for (uint32_t byte = 0; byte < sb; ++byte) d[i * sb + byte] = (uint8_t)(L->slot[i] >> (8 * byte));
    return 0;
}

/* Load a raw image into level `level` (used by the checker). */
static int import_level(or_table_t* t, int level, const void* src)
{
    const uint8_t* s = (const uint8_t*)src;
    if (level == 3) {
        for (uint64_t h = 0; h < t->l3.nlists; ++h) {
            uint64_t v = 0;
            for (uint32_t byte = 0; byte < 4; ++byte) v |= (uint64_t)s[h * 4 + byte] << (8 * byte);
            t->l3.head[h] = v;
        }
        return 0;
    }
    or_level_t* L = image_level(t, level);
    uint32_t sb = L->s / 8;
    for (uint64_t i = 0; i < L->nslots; ++i) {
        uint64_t v = 0;
        for (uint32_t byte = 0; byte < sb; ++byte) v |= (uint64_t)s[i * sb + byte] << (8 * byte);
        L->slot[i] = v;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 7. Table checker                                                         */
/* ------------------------------------------------------------------------ */

static int cmp_u64(const void* a, const void* b)
{
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : x > y;
}

#define FAIL(...) do { if (msg) snprintf(msg, msglen, __VA_ARGS__); rc = 1; goto done; } while (0)

/* Check raw level images against the configuration and return the decoded
 * key set (sorted) in keys_out (capacity >= occupied slots).  Checks:
 *   - every slot is EMPTY, a tombstone, or a valid stored form: occupancy
 *     bit set, unused high bits clear, tag in range (Definition 2, first
 *     item);
 *   - iceberg: the non-empty slots of every bucket form a prefix (the
 *     find-or-put takes the first empty slot, Alg. 1/2; the order property
 *     of Definition 2 needs it).  Not for cuckoo: the put of Alg. 4 may take
 *     any empty slot, and its lookup asks only whether a bucket holds the key
 *     and whether it has an empty slot (Sec. 4.4, Lookup);
 *   - for a non-compact table the stored pi_j(k) addresses its own bucket;
 *   - no key is stored twice (Lemma 1);
 *   - iceberg: the order property of Definition 2 for every stored key;
 *   - cuckoo: a key stored under hash j > 0 has a full bucket a_{j-1}(k)
 *     (the invariant the early-exit lookup relies on, Sec. 2.2 / 4.4).
 * Returns 0 if all hold, 1 with a message otherwise, <0 on bad arguments. */
int or_check3(const or_cfg_t* c, const void* img0, const void* img1, const void* pool, const void* heads,
              uint64_t* keys_out, uint64_t* n_keys, char* msg, int msglen)
{
    int rc = 0;
    uint64_t nk = 0;
    uint8_t* seen = NULL;
    or_table_t* t = or_new(c);
    if (!t) return -1;
    if (t->l3.on && (!pool || !heads)) { or_free(t); return -1; }
    import_level(t, 0, img0);
    if (t->nlevels == 2) import_level(t, 1, img1);
    if (t->l3.on) {
        import_level(t, 2, pool);
        import_level(t, 3, heads);
    }

    for (int x = 0; x < t->nlevels; ++x) {
        or_level_t* L = &t->lv[x];
        uint64_t nbk = 1ULL << L->nb;
        uint64_t used = L->pbits + L->tbits;
        uint64_t maxtag = c->scheme == OR_CUCKOO ? c->H - 1 : (x == 0 ? 0 : 1);
        for (uint64_t b = 0; b < nbk; ++b) {
            uint64_t* bk = bucket_ptr(L, b);
            int seen_empty = 0;
            for (uint32_t y = 0; y < L->B; ++y) {
                uint64_t v = bk[y];
                if (v == 0) { seen_empty = 1; continue; }
                if (seen_empty && c->scheme != OR_CUCKOO)
                    FAIL("level %d bucket %llu: slot %u filled after an empty slot", x, (unsigned long long)b, y);
                if (v == OR_TOMB) continue;
                if (!(v >> (L->s - 1) & 1)) FAIL("level %d bucket %llu slot %u: occupancy bit clear", x, (unsigned long long)b, y);
                if (used < (uint64_t)L->s - 1 && (v & ~(1ULL << (L->s - 1))) >> used)
                    FAIL("level %d bucket %llu slot %u: stray high bits", x, (unsigned long long)b, y);
                uint64_t tag = tag_of(L, v);
                if (tag > maxtag) FAIL("level %d bucket %llu slot %u: tag %llu out of range", x, (unsigned long long)b, y, (unsigned long long)tag);
                uint32_t pi = c->scheme == OR_CUCKOO ? (uint32_t)tag : (x == 0 ? 0 : 1 + (uint32_t)tag);
                uint64_t k = dec_of(t, L, pi, b, v);
                if (addr_of(t, L, pi, k) != b) FAIL("level %d bucket %llu slot %u: key addresses bucket %llu", x, (unsigned long long)b, y, (unsigned long long)addr_of(t, L, pi, k));
                if (enc_of(t, L, pi, k, tag) != v) FAIL("level %d bucket %llu slot %u: stored form does not re-encode", x, (unsigned long long)b, y);
                keys_out[nk++] = k;
                if (c->scheme == OR_CUCKOO) {
                    if (tag > 0) {
                        uint64_t ap = addr_of(t, L, pi - 1, k);
                        uint64_t* bp = bucket_ptr(L, ap);
                        for (uint32_t u = 0; u < L->B; ++u)
                            if (bp[u] == 0) FAIL("cuckoo key in bucket %llu under hash %llu but bucket %llu of hash %llu is not full", (unsigned long long)b, (unsigned long long)tag, (unsigned long long)ap, (unsigned long long)(tag - 1));
                    }
                } else {
                    or_ice_key_t q;
                    ice_key(t, k, &q);
                    uint32_t sx = x == 0 ? 0 : 1 + (uint32_t)tag;
                    /* order property: every slot before (sx, y) is non-empty and is not k */
                    for (uint32_t xx = 0; xx <= 2; ++xx) {
                        uint32_t By = xx == 0 ? c->B0 : c->B1;
                        for (uint32_t yy = 0; yy < By; ++yy) {
                            if (!or_order_less(xx, yy, sx, y)) continue;
                            uint64_t vv = *ice_slot(t, &q, xx, yy);
                            if (vv == 0) FAIL("order property: key at (%u,%u) but earlier slot (%u,%u) is empty", sx, y, xx, yy);
                            if (vv == q.e[xx]) FAIL("order property: key at (%u,%u) also at earlier slot (%u,%u)", sx, y, xx, yy);
                        }
                    }
                }
            }
        }
    }
    /* level 3: every list is a chain of distinct slabs in which slots fill in
     * order (a slab is followed only once it is full); every stored key
     * decodes to its own list, and its primary and both secondary buckets are
     * full without it (level 3 comes after them in the order of Def. 1);
     * slabs on no list (lost link races) are untouched. */
    if (t->l3.on) {
        or_l3_t* q3 = &t->l3;
        or_level_t* L = &q3->L;
        const uint32_t nslot = L->B - 1;
        seen = (uint8_t*)calloc((size_t)q3->nslabs + 1, 1);
        if (!seen) { rc = -2; goto done; }
        for (uint64_t h = 0; h < q3->nlists; ++h) {
            uint64_t id = q3->head[h];
            int seen_empty = 0;
            while (id) {
                if (id > q3->nslabs) FAIL("level 3 list %llu: slab id %llu out of range", (unsigned long long)h, (unsigned long long)id);
                if (seen[id]) FAIL("level 3 slab %llu linked twice", (unsigned long long)id);
                if (seen_empty) FAIL("level 3 list %llu: slab %llu follows a slab with an empty slot", (unsigned long long)h, (unsigned long long)id);
                seen[id] = 1;
                uint64_t* sb = l3_slab(t, id);
                for (uint32_t y = 0; y < nslot; ++y) {
                    uint64_t v = sb[y];
                    if (v == 0) { seen_empty = 1; continue; }
                    if (seen_empty) FAIL("level 3 slab %llu: slot %u filled after an empty slot", (unsigned long long)id, y);
                    if (v == OR_TOMB) continue;
                    if (!holds_key(L, v)) FAIL("level 3 slab %llu slot %u: occupancy bit clear", (unsigned long long)id, y);
                    if (L->pbits < L->s - 1 && (v & ~(1ULL << (L->s - 1))) >> L->pbits)
                        FAIL("level 3 slab %llu slot %u: stray high bits", (unsigned long long)id, y);
                    uint64_t k = dec_of(t, L, 0, h, v);
                    if (addr_of(t, L, 0, k) != h) FAIL("level 3 slab %llu slot %u: key belongs to another list", (unsigned long long)id, y);
                    if (enc_of(t, L, 0, k, 0) != v) FAIL("level 3 slab %llu slot %u: stored form does not re-encode", (unsigned long long)id, y);
                    or_ice_key_t q;
                    ice_key(t, k, &q);
                    for (uint32_t xx = 0; xx <= 2; ++xx) {
                        uint32_t By = xx == 0 ? c->B0 : c->B1;
                        for (uint32_t yy = 0; yy < By; ++yy) {
                            uint64_t vv = *ice_slot(t, &q, xx, yy);
                            if (vv == 0) FAIL("order property: key in level 3 but slot (%u,%u) of its buckets is empty", xx, yy);
                            if (vv == q.e[xx]) FAIL("key in level 3 also at (%u,%u)", xx, yy);
                        }
                    }
                    keys_out[nk++] = k;
                }
                id = sb[nslot];
            }
        }
        for (uint64_t id = 1; id <= q3->nslabs; ++id) {
            if (seen[id]) continue;
            uint64_t* sb = l3_slab(t, id);
            for (uint32_t y = 0; y < L->B; ++y)
                if (sb[y]) FAIL("level 3 slab %llu is on no list but not empty", (unsigned long long)id);
        }
    }
    qsort(keys_out, nk, sizeof(uint64_t), cmp_u64);
    for (uint64_t i = 1; i < nk; ++i)
        if (keys_out[i] == keys_out[i - 1]) FAIL("key %llu stored twice", (unsigned long long)keys_out[i]);
done:
    *n_keys = nk;
    free(seen);
    or_free(t);
    return rc;
}

int or_check(const or_cfg_t* c, const void* img0, const void* img1, uint64_t* keys_out,
             uint64_t* n_keys, char* msg, int msglen)
{
    return or_check3(c, img0, img1, NULL, NULL, keys_out, n_keys, msg, msglen);
}

/* Bucket of key k under permutation i at level `level` (for tests that build
 * adversarial inputs or check placements). */
uint64_t or_bucket_of(const or_table_t* t, int level, uint32_t i, uint64_t k)
{
    return addr_of(t, &t->lv[level], i, k);
}

/* The stored form r'_i(k) with tag `tag` at level `level`. */
uint64_t or_stored_form(const or_table_t* t, int level, uint32_t i, uint64_t k, uint64_t tag)
{
    return enc_of(t, &t->lv[level], i, k, tag);
}

/* Address and stored form of every key under permutation i at the level the
 * scheme uses it on (cuckoo: level 0, tag i; iceberg: i = 0 primary, tag 0;
 * i = 1, 2 secondary with tag i - 1). */
int or_split_array(const or_table_t* t, uint32_t i, const uint64_t* keys, uint64_t n, uint64_t* addr,
                   uint64_t* stored)
{
    const or_level_t* L;
    uint64_t tag;
    if (t->cfg.scheme == OR_CUCKOO) {
        if (i >= t->cfg.H) return -1;
        L = &t->lv[0];
        tag = i;
    } else {
        if (i > 2) return -1;
        L = &t->lv[i == 0 ? 0 : 1];
        tag = i == 2 ? 1 : 0;
    }
    for (uint64_t q = 0; q < n; ++q) {
        addr[q] = addr_of(t, L, i, keys[q]);
        stored[q] = enc_of(t, L, i, keys[q], tag);
    }
    return 0;
}

/* Theorem 1 (e) on a raw iceberg image: every key reported FULL must be
 * absent from all three of its buckets, and those buckets must be full. */
int or_check_full(const or_cfg_t* c, const void* img0, const void* img1, const uint64_t* keys, uint64_t n,
                  char* msg, int msglen)
{
    int rc = 0;
    if (c->scheme != OR_ICEBERG) return -1;
    or_table_t* t = or_new(c);
    if (!t) return -1;
    import_level(t, 0, img0);
    import_level(t, 1, img1);
    for (uint64_t q = 0; q < n; ++q) {
        or_ice_key_t k;
        ice_key(t, keys[q], &k);
        for (uint32_t x = 0; x <= 2; ++x) {
            uint32_t By = x == 0 ? c->B0 : c->B1;
            for (uint32_t y = 0; y < By; ++y) {
                uint64_t v = *ice_slot(t, &k, x, y);
                if (v == 0) FAIL("FULL key %llu: slot (%u,%u) of its buckets is empty", (unsigned long long)keys[q], x, y);
                if (v == k.e[x]) FAIL("FULL key %llu is stored at (%u,%u)", (unsigned long long)keys[q], x, y);
            }
        }
    }
done:
    or_free(t);
    return rc;
}
