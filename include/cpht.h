/*
 * cpht: compact parallel hash tables for AMD Instinct MI355X (gfx950).
 *
 * Lockless batched insert and find on compact (quotiented) bucketed hash
 * tables, after "Compact Parallel Hash Tables on the GPU" (Hegeman, Woltgens,
 * Wijs, Laarman; arXiv 2406.09255):
 *
 *   - compact bucketed cuckoo hashing (Sec. 2.2, Sec. 4.4 Alg. 4): a static
 *     table, bulk-built from distinct keys and then queried;
 *   - compact two-level iceberg hashing (Sec. 2.3, Sec. 3 Alg. 1, Sec. 4.2
 *     Alg. 2/3): a dynamic table with a concurrent find-or-put returning
 *     PUT / FOUND / FULL, and lookups that may run beside it.
 *
 * Quotienting (Sec. 2.4): a seeded bijection pi_i on w-bit keys; the high
 * log2(#buckets) bits of pi_i(k) select the bucket (the address a_i(k)), and
 * only the remaining bits r_i(k) are stored in the slot.
 *
 * Conventions for every call below
 *   - Keys are device arrays of uint32 words when key_bits <= 32, uint64
 *     words otherwise; a key must be < 2^key_bits (larger values are
 *     undefined behaviour, not checked).
 *   - Result arrays are device arrays of one byte per key.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Batch
 *     calls are asynchronous and stream-ordered: they return once the work is
 *     queued.  The caller keeps key and result buffers alive until the
 *     stream has finished with them.  Calls that return data to the host
 *     (cpht_count, cpht_export) synchronise.
 *   - Argument and configuration errors are reported synchronously and
 *     nothing is launched.  A kernel launch failure returns CPHT_E_DEVICE; a
 *     fault inside a kernel surfaces at the next synchronising call.
 *   - The library owns table memory (device memory of the device current at
 *     cpht_create).  Batch calls allocate nothing.
 *   - n = 0 is valid for every batch call and launches nothing.
 *   - Batch calls, cpht_clear, cpht_sorted_fop and the table-set calls launch
 *     kernels only (no memset or copy nodes), so they can be captured in a
 *     HIP graph.  A captured call keeps the arguments of capture time,
 *     including the permutation constants: a replay uses the seed that was
 *     current when it was captured, whatever an eager cpht_clear set since.
 */
#ifndef CPHT_H
#define CPHT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cpht_table* cpht_table_t;

typedef enum {
    CPHT_OK = 0,
    CPHT_E_ARG = 1,          /* null pointer, bad size or value */
    CPHT_E_NOMEM = 2,        /* device allocation failed */
    CPHT_E_UNSUPPORTED = 3,  /* configuration not representable (e.g. remainder + tag + 1 > slot bits) */
    CPHT_E_KEYRANGE = 4,     /* reserved */
    CPHT_E_DEVICE = 5,       /* HIP runtime error */
    CPHT_E_BUSY = 6,         /* a serving loop's queue is full (cpht_server_submit) */
    CPHT_E_STATE = 7         /* operation not valid for this table (e.g. mixed batch on cuckoo) */
} cpht_status_t;

/* Insert outcomes (one byte per key).  0 = key not processed. */
enum { CPHT_PUT = 1, CPHT_FOUND = 2, CPHT_FULL = 3 };
/* Opcodes of a mixed batch. */
enum { CPHT_OP_FIND = 0, CPHT_OP_INSERT = 1 };
/* Schemes. */
enum { CPHT_CUCKOO = 0, CPHT_ICEBERG = 1 };

typedef struct {
    uint32_t scheme;       /* CPHT_CUCKOO or CPHT_ICEBERG */
    uint32_t key_bits;     /* w, 1..64 */
    uint32_t log2_slots0;  /* cuckoo: log2 of all slots; iceberg: primary level */
    uint32_t log2_slots1;  /* iceberg: secondary ("backyard") level; cuckoo: ignored */
    uint32_t bucket0;      /* slots per bucket (primary); power of two */
    uint32_t bucket1;      /* iceberg: slots per secondary bucket, must be bucket0/2 */
    uint32_t slot_bits0;   /* 16 (iceberg only), 32 or 64 */
    uint32_t slot_bits1;   /* iceberg secondary: 16, 32 or 64 */
    uint32_t n_hash;       /* cuckoo: H, 2 or 3 */
    uint32_t max_chain;    /* cuckoo: eviction rounds C before FULL */
    uint32_t subtile;      /* lanes cooperating on one bucket; 0 = default for the bucket size */
    uint32_t compact;      /* 1 = store remainders (quotienting); 0 = store the full pi_i(k) */
    uint32_t log2_lists;   /* iceberg third level: 2^log2_lists lists (ignored if pool_slabs = 0) */
    uint32_t pool_slabs;   /* iceberg third level: 128-byte slabs in its pool; 0 = two levels only */
    uint32_t value_bytes;  /* iceberg map: 4 or 8 bytes of value per key; 0 = a set */
    uint32_t pad;          /* must be 0 */
    uint64_t seed;         /* seed of the permutations pi_0, pi_1, pi_2 */
} cpht_config_t;

/* Defaults: cuckoo H=2, C=256, 2^20 slots in buckets of 32 x 32-bit slots;
 * iceberg 2^20 + 2^17 slots, 32 x 16-bit primary and 16 x 32-bit secondary
 * slots (the shape of the paper's experiments, Sec. 5.1), key_bits 32,
 * compact, seed 1. */
void cpht_config_default(uint32_t scheme, cpht_config_t* cfg);

/* Check a configuration without allocating anything: CPHT_OK if cpht_create
 * would accept it, and the resolved configuration (subtile filled in) in
 * *resolved when resolved != NULL.  Touches no device. */
cpht_status_t cpht_config_check(const cpht_config_t* cfg, cpht_config_t* resolved);

/* Third iceberg level (pool_slabs > 0; Sec. 2.3: a third level of linked
 * lists outside the table, the list chosen by h_0(k), so that inserts do not
 * fail; Sec. 3 Limitations: slab lists).  A key goes there only when its
 * primary bucket and both secondary buckets are full without it.  List a
 * holds the keys whose pi_0(k) has high log2_lists bits a; it is a chain of
 * 128-byte slabs taken from a pool of pool_slabs slabs allocated at create.
 * A slab has 32-bit slots (64-bit when slot_bits0 = 64) storing the
 * occupancy bit and the remaining w - log2_lists bits of pi_0(k) (all w bits
 * if not compact; w - log2_lists + 1 must fit the slot); its last slot holds
 * the id of the next slab (ids count from 1; 0 = end of list).  Slots of a
 * list fill in list order, as in a bucket; a link is set once (reserved by
 * CAS, then published), so find-or-put keeps one copy per key.  pool_slabs <
 * 2^31 - 1.  Insert answers CPHT_FULL only once
 * the pool is used up.  Lookups and deletes walk the list when both
 * secondary buckets are full.  Not supported for 64-bit primary slots with
 * a 32-lane sub-tile, nor in table sets (CPHT_E_UNSUPPORTED). */

/* Map (value_bytes = 4 or 8; iceberg only): the iceberg table is stable, a
 * key never moves once stored, so its value sits at the same index as its
 * slot in a parallel array per level (Sec. 2.1: a stable table can keep
 * values in a separate array at the key's index; Sec. 6 notes maps as the
 * case where compactness matters more).  Levels 0 and 1 get arrays of
 * 2^log2_slots_x values, the third level pool_slabs * (slots per slab).
 * Only cpht_insert_values writes values and cpht_find_values reads them; the
 * set calls ignore them.  Not supported in table sets. */

/* Create an empty table (synchronous: allocates and zeroes device memory).
 * Level x holds 2^log2_slots_x slots in buckets of bucket_x slots; each
 * bucket is bucket_x*slot_bits_x/8 contiguous bytes.  The stored remainder
 * has key_bits - log2(#buckets) bits (key_bits bits if compact = 0); with
 * its tag (cuckoo: ceil(log2 H) bits; iceberg secondary: 1 bit) and one
 * occupancy bit it must fit the slot, else CPHT_E_UNSUPPORTED. */
cpht_status_t cpht_create(const cpht_config_t* cfg, cpht_table_t* out);

/* Free the table's device memory.  Pending work using it must have finished. */
cpht_status_t cpht_destroy(cpht_table_t t);

/* The resolved configuration (subtile filled in). */
cpht_status_t cpht_get_config(cpht_table_t t, cpht_config_t* cfg);

/* Empty the table and re-derive the permutations from `seed` (stream-ordered;
 * uses a fill kernel, no memset node).  On a table-set view the set's own
 * launches use the new permutations from then on as well: a kernel on the
 * same stream rewrites the set's device copy of the table's description. */
cpht_status_t cpht_clear(cpht_table_t t, uint64_t seed, void* stream);

/* Insert a batch.
 *   Iceberg: find-or-put of every key (Sec. 3 Alg. 1, cooperative form
 *   Alg. 2, batch form Alg. 3).  d_out[i] = CPHT_PUT if this call stored
 *   keys[i], CPHT_FOUND if the key was already present (stored earlier or by
 *   another operation of the batch), CPHT_FULL if its primary bucket and both
 *   secondary buckets are full without it.  Duplicates are allowed; at most
 *   one operation per key returns PUT.  May run concurrently with cpht_find
 *   and other cpht_insert calls on the same table.
 *   Cuckoo: compact cuckoo put (Sec. 4.4 Alg. 4).  Keys must be distinct and
 *   absent from the table, and no find may run concurrently (the table is
 *   static, Sec. 4.4).  d_out[i] = CPHT_PUT, or CPHT_FULL when an eviction
 *   chain exceeded max_chain; the key dropped then is the one being carried,
 *   which need not be keys[i]. */
cpht_status_t cpht_insert(cpht_table_t t, const void* d_keys, uint64_t n, uint8_t* d_out, void* stream);

/* Same as cpht_insert; the name used for the static build of a cuckoo table. */
cpht_status_t cpht_bulk_build(cpht_table_t t, const void* d_keys, uint64_t n, uint8_t* d_out, void* stream);

/* Lookup of a batch: d_found[i] = 1 if keys[i] is in the table, else 0.
 * Cuckoo: buckets a_0(k), a_1(k), ... in order, stopping at the first bucket
 * that is not full (Sec. 4.4 "Lookup").  Iceberg: the primary bucket, and
 * both secondary buckets only when the primary is full (Sec. 2.3 "Lookup"). */
cpht_status_t cpht_find(cpht_table_t t, const void* d_keys, uint64_t n, uint8_t* d_found, void* stream);

/* Delete a batch by tombstones (Sec. 2.2 "Lookup" and Sec. 3 "Limitations"):
 * the slot holding keys[i] gets the tombstone word 1, which is not EMPTY and
 * matches no key, so non-empty slots stay consecutive and lookups keep their
 * early exit.  d_out[i] = 1 if this call removed keys[i], else 0 (absent, or
 * removed by another delete of the same key in the batch: exactly one
 * operation per stored key answers 1).  Tombstones are not reclaimed by
 * find-or-put or by the first-empty claim of the cuckoo put (a cuckoo
 * eviction that picks one as its victim overwrites it); they are counted by
 * neither cpht_count nor the fill factor, but keep their slots until
 * cpht_clear.  Iceberg: may run concurrently with cpht_find and other
 * deletes (a find of a key being deleted may answer either way).  Cuckoo: no
 * put may run concurrently. */
cpht_status_t cpht_delete(cpht_table_t t, const void* d_keys, uint64_t n, uint8_t* d_out, void* stream);

/* Iceberg only: one batch of finds (d_ops[i] = CPHT_OP_FIND, answer 0/1) and
 * find-or-puts (CPHT_OP_INSERT, answer PUT/FOUND/FULL) executed concurrently
 * (dynamic operation, Sec. 1 and Sec. 3).  A find of a key that another
 * operation of the same batch inserts may answer either way. */
cpht_status_t cpht_mixed(cpht_table_t t, const void* d_keys, const uint8_t* d_ops, uint64_t n, uint8_t* d_out,
                         void* stream);

/* Map find-or-put (put if absent): like cpht_insert on an iceberg table, and
 * the operation that stores keys[i] (answer CPHT_PUT) writes d_values[i] (4
 * or 8 bytes each, as value_bytes) as its value; keys already present keep
 * their value (CPHT_FOUND), so with repeats in one batch the stored value is
 * that of the occurrence answered CPHT_PUT.  A concurrent lookup that finds
 * a key stored by this call may read its value before it is written: values
 * are complete for calls that follow in stream order.  CPHT_E_STATE without
 * values. */
cpht_status_t cpht_insert_values(cpht_table_t t, const void* d_keys, const void* d_values, uint64_t n,
                                 uint8_t* d_out, void* stream);

/* Map lookup: d_found[i] = 1 and d_values_out[i] = the value of keys[i] if it
 * is stored, d_found[i] = 0 and d_values_out[i] unchanged otherwise. */
cpht_status_t cpht_find_values(cpht_table_t t, const void* d_keys, uint64_t n, uint8_t* d_found,
                               void* d_values_out, void* stream);

/* Size of, and copy to host memory (synchronous) of, the value array of
 * level 0, 1 or 2 (the third level's pool): value_bytes per slot, at the
 * slot's index in cpht_export's image of that level. */
cpht_status_t cpht_values_bytes(cpht_table_t t, uint32_t level, uint64_t* bytes);
cpht_status_t cpht_export_values(cpht_table_t t, uint32_t level, void* h_dst, uint64_t bytes);
/* The reverse of cpht_export_values (synchronous), for checkpoint / resume. */
cpht_status_t cpht_import_values(cpht_table_t t, uint32_t level, const void* h_src, uint64_t bytes);

/* Cuckoo only: find-or-put by sorting the batch, the baseline of the paper's
 * find-or-put experiment (Sec. 5, find-or-put benchmark): the keys are
 * sorted with their positions to find duplicates, every distinct key is
 * looked up once, and each distinct key that was absent is inserted once
 * with the cuckoo put.  Keys may repeat and may already be stored.
 * d_out[i] = CPHT_FOUND if keys[i] was in the table before the call, else
 * the put's answer at the first occurrence of the key in the batch
 * (CPHT_PUT, or CPHT_FULL when the eviction chain exceeded max_chain; the
 * key dropped then is the carried one, as for cpht_insert) and CPHT_FOUND at
 * its later occurrences (CPHT_FULL if the first got CPHT_FULL).  No other
 * call may use the table concurrently.  n < 2^32.
 * d_workspace: caller-owned device memory of at least
 * cpht_sorted_fop_workspace(t, n) bytes, 256-byte aligned, used as scratch
 * by the call (contents undefined afterwards; not to be shared by calls that
 * overlap).  CPHT_E_STATE on an iceberg table (its insert is already a
 * find-or-put), CPHT_E_ARG if the workspace is too small or misaligned. */
cpht_status_t cpht_sorted_fop(cpht_table_t t, const void* d_keys, uint64_t n, uint8_t* d_out, void* d_workspace,
                              uint64_t workspace_bytes, void* stream);

/* Workspace bytes cpht_sorted_fop needs for n keys on table t (about 40
 * bytes per key with 64-bit key words, 28 with 32-bit ones). */
cpht_status_t cpht_sorted_fop_workspace(cpht_table_t t, uint64_t n, uint64_t* bytes);

/* For callers that cannot allocate device memory (code under stream or graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * find-or-put as cpht_sorted_fop, with the same answers, but its scratch is a
 * fixed 40 MiB array of device memory that the library holds on each GPU it
 * runs on until the process ends (its address is looked up once per device,
 * when the first cuckoo table on that device is created, so the call makes no
 * runtime lookup).  The call allocates nothing and takes no workspace.  n <= 2^20 keys (CPHT_E_ARG above that; CPHT_E_STATE on an
 * iceberg table).  All calls on one GPU share that GPU's array: calls that
 * overlap on one GPU (other streams, other threads, other tables) race and
 * give undefined answers; order them on one stream or synchronise between
 * them.  The array keeps the last call's contents; no step of the pipeline
 * relies on its previous contents. */
cpht_status_t cpht_sorted_fop_noalloc(cpht_table_t t, const void* d_keys, uint64_t n, uint8_t* d_out, void* stream);

/* Slots holding a key (tombstones excluded; third-level slots included) and
 * total slots of the bucket levels (fill factor = occupied / capacity,
 * Sec. 2.1; with a third level it can exceed 1).  Synchronises `stream`. */
cpht_status_t cpht_count(cpht_table_t t, uint64_t* occupied, uint64_t* capacity, void* stream);

/* Third level: slabs taken from the pool so far (synchronous; CPHT_E_STATE
 * without a third level).  A slab is taken only by the insert that reserved
 * the link it goes into, so every slab taken is on a list. */
cpht_status_t cpht_level3_used(cpht_table_t t, uint32_t* slabs);

/* Size in bytes of image `level`: 0 the (primary) bucket level, 1 the iceberg
 * secondary level, and with a third level 2 its slab pool (pool_slabs * 128
 * bytes) and 3 its list heads (2^log2_lists uint32 slab ids). */
cpht_status_t cpht_level_bytes(cpht_table_t t, uint32_t level, uint64_t* bytes);

/* Device pointer to level `level` (for callers that copy it themselves). */
cpht_status_t cpht_level_ptr(cpht_table_t t, uint32_t level, void** d_ptr);

/* Copy image `level` to host memory (synchronous).  Raw layout: bucket b,
 * slot q at byte offset (b*bucket + q)*slot_bits/8, little endian; a slot is 0
 * (EMPTY), 1 (a tombstone) or (1 << (slot_bits-1)) | tag << p | payload, where
 * p is the payload width (key_bits - log2(#buckets), or key_bits if not
 * compact).  The slab pool (level 2) uses the same slot layout with slab id i
 * at byte offset (i - 1)*128; list heads (level 3) are uint32 slab ids. */
cpht_status_t cpht_export(cpht_table_t t, uint32_t level, void* h_dst, uint64_t bytes);

/* Checkpoint / resume: copy a host image (as written by cpht_export, same
 * configuration and seed) into image `level` (synchronous).  Restoring the
 * slab pool (level 2) also restores the count of slabs taken, as the highest
 * slab that holds anything (every slab taken is on a list).  The caller
 * restores every image of the table before using it; no other call may run
 * on the table meanwhile. */
cpht_status_t cpht_import(cpht_table_t t, uint32_t level, const void* h_src, uint64_t bytes);

/* The quotienting split of Sec. 2.4 as the table applies it: for permutation
 * `perm_index` (cuckoo: hash index j < H; iceberg: 0 = primary, 1 and 2 =
 * the two secondary buckets), d_addr[i] = a(keys[i]) and d_stored[i] = the
 * slot value the table stores for keys[i] there (with its tag). */
cpht_status_t cpht_split(cpht_table_t t, uint32_t perm_index, const void* d_keys, uint64_t n, uint64_t* d_addr,
                         uint64_t* d_stored, void* stream);

/* Compiled kernel variants, for tuners: entry i of scheme `scheme` as
 * (key64, slot_bits0, slot_bits1, bucket0, bucket1, subtile).  Returns the
 * number of variants; fills *info (6 values) when info != NULL and i is valid. */
int cpht_variant_info(uint32_t scheme, int i, uint32_t* info);

/* ---- Table sets: many independent tables served by one launch -------------
 * A table set owns one device arena holding every level of n tables whose
 * configurations may differ (they must share the scheme and the key word size:
 * all key_bits <= 32, or all > 32).  Tables are grouped by compiled kernel
 * variant; a batch over the set is planned on the device (its keys cut into
 * chunks of at most 256 keys of one table) and served by one persistent launch
 * per variant group, so plan and launches contain no host step and can be
 * captured in a single graph.  The set keeps device scratch for planning:
 * batch calls on one set must be ordered on one stream (they are not safe to
 * overlap).  Operations are those of cpht_insert / cpht_find, per table. */
typedef struct cpht_multi* cpht_multi_t;

/* Create a set of n_tables empty tables (synchronous).  max_keys bounds the
 * keys of any single batch (it sizes the chunk list: max_keys/256 + n_tables
 * chunks).  Each configuration is checked as by cpht_create. */
cpht_status_t cpht_multi_create(uint32_t n_tables, const cpht_config_t* cfgs, uint64_t max_keys, cpht_multi_t* out);

/* Free the set.  Pending work using it must have finished; views become invalid. */
cpht_status_t cpht_multi_destroy(cpht_multi_t m);

/* A non-owning handle to table i of the set, usable with every single-table
 * call (insert, find, count, export, split, clear); cpht_destroy rejects it
 * with CPHT_E_STATE. */
cpht_status_t cpht_multi_table(cpht_multi_t m, uint32_t i, cpht_table_t* view);

/* Empty every table (fill kernel on `stream`; permutation seeds unchanged). */
cpht_status_t cpht_multi_clear(cpht_multi_t m, void* stream);

/* Insert / find a batch over the set.  d_keys holds the keys of all tables
 * concatenated; d_offsets (device, n_tables + 1 entries) gives table i the
 * keys [d_offsets[i], d_offsets[i+1]); total_keys is the length of d_keys
 * (keys at or past it are ignored; at most max_keys).  d_out has one byte per
 * key at the same index, with the single-table meaning.  If the chunks of a
 * batch exceed the capacity, the excess is skipped and bit 0 of the flags of
 * cpht_multi_error is raised. */
cpht_status_t cpht_multi_insert(cpht_multi_t m, const void* d_keys, const uint64_t* d_offsets, uint64_t total_keys,
                                uint8_t* d_out, void* stream);
cpht_status_t cpht_multi_find(cpht_multi_t m, const void* d_keys, const uint64_t* d_offsets, uint64_t total_keys,
                              uint8_t* d_found, void* stream);

/* Arena size, number of variant groups (= launches per batch), chunk capacity. */
cpht_status_t cpht_multi_info(cpht_multi_t m, uint64_t* arena_bytes, uint32_t* n_groups, uint64_t* max_chunks);

/* Synchronise the device, return and clear the set's error flags. */
cpht_status_t cpht_multi_error(cpht_multi_t m, uint32_t* flags);

/* ---- Serving loop: continuous batching over one resident iceberg table ------
 * A server owns a device staging ring (staging_keys keys with their opcodes and
 * results) and max_inflight streams.  Its dispatcher thread admits queued
 * requests in arrival order whenever a stream is free and the ring has room
 * (admission by free device memory), packs the admitted requests (up to
 * max_batch_keys keys; one request per launch if coalesce = 0) into one
 * cpht_mixed launch, copies each request's results back, and completes the
 * requests when that launch's event fires.  Requests arriving while earlier
 * launches run are admitted into the next free stream, so launches overlap on
 * the device; all of them operate on the same table concurrently (the dynamic
 * operation of Sec. 3).  A find whose key another in-flight request inserts
 * may therefore answer either way; every other answer equals the answer the
 * request gets alone.  Host buffers passed to the server should be pinned
 * (page-locked) for asynchronous copies and must stay valid until the request
 * completes.  Latency = completion time - submission time (steady clock).
 * In zero-copy mode (zero_copy = 1) there is no staging: every request buffer
 * must be pinned host memory mapped for the device (hipHostMalloc, or a torch
 * tensor after pin_memory()), the mixed kernel reads the keys and opcodes and
 * writes the results in place, and a launch covers a run of queued requests
 * that lie back to back in all three buffers (up to max_batch_keys keys).
 * In resident mode (resident = 1, with zero_copy = 1) requests are not
 * launched one by one: a persistent kernel started by the server takes
 * request descriptors from a ring of 1024 in pinned host memory (one per
 * request, or with coalesce = 1 one per run of queued requests that lie back
 * to back in all three buffers, up to max_batch_keys operations), cuts each
 * into chunks of 256 to 2048 operations (small while little work is in
 * flight, so that a lone request is spread over many blocks) that its blocks
 * (two per compute unit, plus one that watches the ring) take in order, and
 * reports every completed descriptor back through the ring; so up to 1024
 * descriptors are in flight and overlap on the device, and an idle request
 * costs no kernel launch.  A request larger than max_batch_keys is refused
 * (CPHT_E_ARG) in this mode.  The kernel ends after idle_us without requests
 * and is started again by the next one.  While it runs it holds part of the device: work
 * that synchronises the whole device (hipDeviceSynchronize) waits until it
 * ends, so stop the server, or let it go idle, before such calls.
 * The server runs set operations (cpht_mixed): on a map table the values are
 * neither written nor returned.  The table must outlive the server, and no
 * other call may clear or import into it while the server runs.  The server
 * keeps a record (about 80 bytes) per ticket until the request has completed
 * and either its ticket was waited on (or polled as done) or 2^20 later
 * tickets exist; poll and wait return CPHT_E_ARG for a ticket whose record is
 * gone.  After a device error every pending and
 * later request completes at once (results undefined) and submit, poll and
 * wait return CPHT_E_DEVICE. */
typedef struct cpht_server* cpht_server_t;

typedef struct {
    uint32_t max_inflight;    /* concurrent launches (streams), 1..64 */
    uint32_t coalesce;        /* 1: pack several requests per launch; 0: one request per launch */
    uint64_t staging_keys;    /* device staging capacity in keys (a request must fit it); 0: sized at
                                 start from the free device memory (a quarter of it, at most 2^28 keys;
                                 CPHT_E_NOMEM if that is below max_batch_keys) */
    uint64_t max_batch_keys;  /* keys per launch when coalescing (<= staging_keys unless zero_copy) */
    uint32_t zero_copy;       /* 1: the device works on the pinned request buffers in place (no staging) */
    uint32_t resident;        /* 1 (requires zero_copy = 1; two-level tables of at most 2^24 primary
                                 slots; max_batch_keys <= 2^17, else CPHT_E_UNSUPPORTED): no launch per
                                 request: one persistent launch takes the requests from a ring in pinned
                                 host memory */
    uint32_t idle_us;         /* resident: the persistent launch ends after this long without requests
                                 (1 .. 10^7; the next request starts it again) */
    uint32_t pad;             /* must be 0 */
} cpht_server_config_t;

/* Defaults: 4 launches in flight, coalescing, 2^24 staging keys, 2^22 keys per
 * launch, staged (zero_copy = 0), not resident (idle_us = 10000). */
void cpht_server_config_default(cpht_server_config_t* cfg);

/* Start a server on an iceberg table (CPHT_E_STATE for cuckoo: static). */
cpht_status_t cpht_server_start(cpht_table_t t, const cpht_server_config_t* cfg, cpht_server_t* out);

/* Queue a request of n operations (h_ops[i]: CPHT_OP_FIND or CPHT_OP_INSERT);
 * results go to h_out (find 0/1, insert PUT/FOUND/FULL).  Returns a ticket.
 * CPHT_E_BUSY if 2^20 requests are already queued; CPHT_E_ARG if n exceeds
 * the staging capacity or, in zero-copy mode, if a buffer is not pinned host
 * memory mapped for the device. */
cpht_status_t cpht_server_submit(cpht_server_t s, const void* h_keys, const uint8_t* h_ops, uint64_t n,
                                 uint8_t* h_out, uint64_t* ticket);

/* Non-blocking completion check; latency in ns once done. */
cpht_status_t cpht_server_poll(cpht_server_t s, uint64_t ticket, int* done, uint64_t* latency_ns);

/* Block until the request completes. */
cpht_status_t cpht_server_wait(cpht_server_t s, uint64_t ticket, uint64_t* latency_ns);

/* Launches issued, requests and operations completed, longest queue seen. */
cpht_status_t cpht_server_stats(cpht_server_t s, uint64_t* launches, uint64_t* requests_done, uint64_t* ops_done,
                                uint64_t* max_queue);

/* Drain queued and in-flight requests, stop the dispatcher, free the server. */
cpht_status_t cpht_server_stop(cpht_server_t s);

/* Replay a request trace from the calling thread: request i (operations
 * [offsets[i], offsets[i+1]) of h_keys / h_ops / h_out) is submitted
 * arrival_ns[i] after the start (non-decreasing), then all are awaited.
 * offsets has n_requests + 1 non-decreasing entries, and the three buffers
 * must hold offsets[n_requests] entries (not checked: the library cannot see
 * their sizes).  latency_ns[i] receives each request's latency; *makespan_ns
 * the time from the start to the last completion.  CPHT_E_ARG for
 * decreasing offsets or arrival times (nothing is submitted then). */
cpht_status_t cpht_server_replay(cpht_server_t s, uint64_t n_requests, const uint64_t* arrival_ns,
                                 const uint64_t* offsets, const void* h_keys, const uint8_t* h_ops, uint8_t* h_out,
                                 uint64_t* latency_ns, uint64_t* makespan_ns);

/* Measurement kernels for the random-access roofline (not table operations).
 * d_buf: device buffer of `bytes` bytes (a power of two, >= 4096), which the
 * CAS kinds modify; d_sink: one device word the kernels may write.
 *   kind 0: random 128-byte line reads, 8 lanes x 16 bytes per line;
 *   kind 1: random 32-bit CAS (expected 0);
 *   kind 2: a random line read followed by a CAS into that line;
 *   kind 3: random 64-bit CAS (expected 0) on 8-byte words;
 *   kind 4: the quotienting split alone (Sec. 2.4): d_buf holds uint64 keys,
 *           read in order (wrapping round), each split under three
 *           permutations of 37-bit keys into a 22-bit address and a stored
 *           form, as the benchmark table does; nothing is written but d_sink
 *           (practically never).  One operation = one key's three splits;
 *   kind 5: random 64-byte reads (half lines), 4 lanes x 16 bytes;
 *   kind 6: random 128-byte line reads as kind 0, with non-temporal loads.
 * `ops` is rounded up to a multiple of 16384; *ops_done receives the count
 * actually issued.  Asynchronous on `stream`. */
cpht_status_t cpht_probe(uint32_t kind, void* d_buf, uint64_t bytes, uint64_t ops, uint64_t seed, uint32_t* d_sink,
                         uint64_t* ops_done, void* stream);

const char* cpht_status_str(cpht_status_t s);

#ifdef __cplusplus
}
#endif

#endif /* CPHT_H */
