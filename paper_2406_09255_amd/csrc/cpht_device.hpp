// Device-side building blocks of the compact hash tables: the quotienting
// permutation (Sec. 2.4), slot encoding, and the wave64 sub-tile primitives
// Any / First / Count / Shuffle of Sec. 4.1 mapped onto CDNA ballots.
//
// A sub-tile is G consecutive lanes of a 64-lane wavefront (G in 2..32, a
// power of two, so a sub-tile never straddles the two 32-lane halves).  A
// bucket is read by one sub-tile with one vector load per lane: lane `rk`
// holds W consecutive 32-bit words of the bucket, i.e. W*32/S slots.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace cpht {

// ---------------------------------------------------------------------------
// Kernel-side table description (filled by the host library)
// ---------------------------------------------------------------------------

struct PermK {             // one permutation pi_i: 3 rounds of constants
  uint64_t m[3];           // odd multipliers mod 2^w
  uint64_t minv[3];        // their inverses mod 2^w
  uint64_t c[3];           // xor constants
};

struct LevelK {
  uint32_t* base;          // bucket array, 2^nb buckets of bucket_words words
  uint64_t pmask;          // payload mask: remainder bits, or all key bits
  uint32_t nb;             // log2 number of buckets
  uint32_t pbits;          // payload bits
  uint32_t bucket_words;   // 32-bit words per bucket
  uint32_t tbits;          // tag bits (cuckoo hash index, iceberg secondary index)
};

// Third iceberg level (Sec. 2.3: lists outside the table chosen by h_0(k)).
// List a = the high nb bits of pi_0(k); each list is a chain of 128-byte
// slabs from a fixed pool; a slab holds 32 / (S3 / 32) slots of S3 bits, the
// last of which holds the id of the next slab (0 = end of the list).  Slab id
// i (1-based) is pool words [(i - 1) * 32, i * 32).  nslabs = 0: no level 3.
struct Level3K {
  LevelK L;                // addressing and encoding (base = pool, bucket_words = 32)
  uint32_t* heads;         // first slab id of each of the 2^L.nb lists
  uint32_t* used;          // slabs handed out so far
  uint32_t nslabs;         // pool capacity
  uint32_t pad;
};

struct TableK {
  LevelK lv[2];
  Level3K l3;
  PermK perm[3];
  uint64_t kmask;          // 2^w - 1
  uint32_t w;              // key bits
  uint32_t h;              // xor-shift distance ceil(w/2)
  uint32_t H;              // cuckoo hash functions
  uint32_t C;              // cuckoo chain bound
  uint32_t compact;        // 1: payload is the remainder
  uint32_t vbytes;         // map values: 0 (a set), 4 or 8 bytes per slot
  // Map values (stable iceberg table: a key's value sits at its slot's index
  // in a parallel array, Sec. 2.1): level 0, level 1, and the slab pool.
  uint8_t* vals[3];
};

struct BatchK {
  const void* keys;        // uint32 words if w <= 32 else uint64 words
  const uint8_t* ops;      // mixed batches: 0 = find, 1 = insert
  uint8_t* out;            // one result byte per key
  uint64_t n;
  const void* vin;         // map inserts: one value per key (vbytes each)
  void* vout;              // map lookups: the value of each key found
};

// Value of slot `index` of a level: map insert writes it (put-if-absent:
// only the operation that stored the key), map lookup reads it.
__device__ __forceinline__ void put_value(const TableK& T, int level, uint64_t index, const BatchK& Bt,
                                          uint64_t idx) {
  if (T.vbytes == 8)
    reinterpret_cast<uint64_t*>(T.vals[level])[index] = static_cast<const uint64_t*>(Bt.vin)[idx];
  else
    reinterpret_cast<uint32_t*>(T.vals[level])[index] = static_cast<const uint32_t*>(Bt.vin)[idx];
}

__device__ __forceinline__ void get_value(const TableK& T, int level, uint64_t index, const BatchK& Bt,
                                          uint64_t idx) {
  if (T.vbytes == 8)
    static_cast<uint64_t*>(Bt.vout)[idx] = reinterpret_cast<const uint64_t*>(T.vals[level])[index];
  else
    static_cast<uint32_t*>(Bt.vout)[idx] = reinterpret_cast<const uint32_t*>(T.vals[level])[index];
}

// A launch over many tables: chunk b = keys [start, start + count) of the
// concatenated key array, all of table `table` (count <= 256).
struct ChunkK {
  uint64_t start;
  uint32_t table;
  uint32_t count;
};

struct MultiK {
  const TableK* descs;     // one description per table (device memory)
  const ChunkK* chunks;    // all chunks, grouped by kernel variant
  const uint64_t* group;   // device pair: first chunk and chunk count of this launch's group
  const void* keys;        // concatenated keys of all tables
  uint8_t* out;            // one result byte per key, same indexing
};

enum : uint8_t { R_NONE = 0, R_PUT = 1, R_FOUND = 2, R_FULL = 3 };

// A deleted key leaves a tombstone: the word 1 in a slot of any width.  It is
// not EMPTY (so the non-empty slots of a bucket stay consecutive and lookups
// keep their early exit, Sec. 2.2 "Lookup", Sec. 3 "Limitations"), and with
// its occupancy bit clear it equals no stored form.
constexpr uint64_t TOMB = 1;

// ---------------------------------------------------------------------------
// Permutation pi_i on w-bit keys and its inverse.  U is uint32_t for w <= 32
// and uint64_t otherwise; all arithmetic is modulo 2^w.
// ---------------------------------------------------------------------------

template <class U>
__device__ __forceinline__ U perm_fwd(const PermK& P, U x, uint32_t h, U mask) {
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    x ^= x >> h;
    x = (x * (U)P.m[q]) & mask;
    x ^= (U)P.c[q];
  }
  x ^= x >> h;
  return x;
}

template <class U>
__device__ __forceinline__ U perm_inv(const PermK& P, U y, uint32_t h, U mask) {
  y ^= y >> h;
#pragma unroll
  for (int q = 2; q >= 0; --q) {
    y ^= (U)P.c[q];
    y = (y * (U)P.minv[q]) & mask;
    y ^= y >> h;
  }
  return y;
}

// Address (high nb bits) and stored form (occupancy | tag | payload) of a key
// under permutation i at level L.
template <class U, int S>
struct Split {
  uint64_t a;
  uint64_t e;
};

template <int S>
__device__ __forceinline__ uint64_t occ_bit() { return 1ull << (S - 1); }

template <class U, int S>
__device__ __forceinline__ Split<U, S> split_key(const TableK& T, const LevelK& L, int i, U k,
                                                 uint32_t tag) {
  const U mask = (U)T.kmask;
  U x = perm_fwd<U>(T.perm[i], k, T.h, mask);
  Split<U, S> r;
  r.a = L.nb ? (uint64_t)(x >> (T.w - L.nb)) : 0ull;
  r.e = occ_bit<S>() | ((uint64_t)tag << L.pbits) | ((uint64_t)x & L.pmask);
  return r;
}

// Key stored as value v in bucket a under permutation i (k = pi^-1(a . r)).
template <class U>
__device__ __forceinline__ U join_key(const TableK& T, const LevelK& L, int i, uint64_t a,
                                      uint64_t v) {
  uint64_t payload = v & L.pmask;
  uint64_t x = payload;
  if (T.compact && L.nb) x |= a << (T.w - L.nb);
  return perm_inv<U>(T.perm[i], (U)x, T.h, (U)T.kmask);
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Cuckoo victim row for carried key k in round c (1-based): low bits of the
// first splitmix64 output for state k ^ (c << 32).
__device__ __forceinline__ uint32_t victim_row(uint64_t k, uint32_t c, uint32_t B) {
  return (uint32_t)(mix64((k ^ ((uint64_t)c << 32)) + 0x9E3779B97F4A7C15ull) & (B - 1));
}

// Slot at which the cuckoo put of carried key k starts looking for an empty
// slot in round c: high bits of the same splitmix64 output.  Concurrent puts
// aimed at one bucket then spread their claims over its empty slots instead
// of all claiming the first one.
__device__ __forceinline__ uint32_t claim_start(uint64_t k, uint32_t c, uint32_t B) {
  return (uint32_t)(mix64((k ^ ((uint64_t)c << 32)) + 0x9E3779B97F4A7C15ull) >> 32) & (B - 1);
}

// ---------------------------------------------------------------------------
// Lane-local slot views.  A lane holds W words = W*32/S slots; the slot index
// within the lane is a compile-time constant wherever registers are indexed.
// ---------------------------------------------------------------------------

template <int S, int W>
struct Lane {
  static constexpr int PER = W * 32 / S;  // slots held by one lane
  static_assert(PER >= 1, "a lane must hold at least one whole slot");
  static_assert(S != 64 || (W % 2) == 0, "64-bit slots need word pairs");
};

template <int S, int W>
__device__ __forceinline__ uint64_t slot_at(const uint32_t (&w)[W], int i) {
  if constexpr (S == 16) return (w[i >> 1] >> ((i & 1) * 16)) & 0xFFFFu;
  else if constexpr (S == 32) return w[i];
  else return (uint64_t)w[2 * i] | ((uint64_t)w[2 * i + 1] << 32);
}

template <int S, int W>
__device__ __forceinline__ bool lane_has(const uint32_t (&w)[W], uint64_t e) {
  bool hit = false;
#pragma unroll
  for (int i = 0; i < Lane<S, W>::PER; ++i) hit |= slot_at<S, W>(w, i) == e;
  return hit;
}

// Index of the slot held by this lane that equals e, or PER if there is none.
template <int S, int W>
__device__ __forceinline__ int lane_match(const uint32_t (&w)[W], uint64_t e) {
  int f = Lane<S, W>::PER;
#pragma unroll
  for (int i = Lane<S, W>::PER - 1; i >= 0; --i)
    if (slot_at<S, W>(w, i) == e) f = i;
  return f;
}

// Index of the first slot held by this lane that is EMPTY in the snapshot
// and not known to be occupied (bit i of `known`), or PER if there is none.
template <int S, int W>
__device__ __forceinline__ int lane_first_empty(const uint32_t (&w)[W], uint32_t known) {
  int f = Lane<S, W>::PER;
#pragma unroll
  for (int i = Lane<S, W>::PER - 1; i >= 0; --i)
    if (slot_at<S, W>(w, i) == 0 && !((known >> i) & 1u)) f = i;
  return f;
}

// Word idx (a run-time value) of the lane's registers, selected with masks so
// the register array is never indexed dynamically (which would spill it).
template <int W>
__device__ __forceinline__ uint32_t get_word(const uint32_t (&w)[W], int idx) {
  uint32_t v = 0;
#pragma unroll
  for (int i = 0; i < W; ++i) v |= w[i] & (0u - (uint32_t)(i == idx));
  return v;
}

// Vector load of the lane's W words (16-byte pieces where possible).
template <int W>
__device__ __forceinline__ void load_words(uint32_t (&w)[W], const uint32_t* p) {
  if constexpr (W % 4 == 0) {
#pragma unroll
    for (int i = 0; i < W; i += 4) {
      uint4 v = *reinterpret_cast<const uint4*>(p + i);
      w[i] = v.x; w[i + 1] = v.y; w[i + 2] = v.z; w[i + 3] = v.w;
    }
  } else if constexpr (W == 2) {
    uint2 v = *reinterpret_cast<const uint2*>(p);
    w[0] = v.x; w[1] = v.y;
  } else {
#pragma unroll
    for (int i = 0; i < W; ++i) w[i] = p[i];
  }
}

// ---------------------------------------------------------------------------
// Atomics (agent scope: visible across all XCDs of the device)
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t cas32(uint32_t* p, uint32_t expect, uint32_t desired) {
  __hip_atomic_compare_exchange_strong(p, &expect, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return expect;  // the value found in memory
}

__device__ __forceinline__ uint64_t cas64(uint64_t* p, uint64_t expect, uint64_t desired) {
  __hip_atomic_compare_exchange_strong(p, &expect, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return expect;
}

__device__ __forceinline__ uint32_t xchg32(uint32_t* p, uint32_t v) {
  return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t xchg64(uint64_t* p, uint64_t v) {
  return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

enum : int { CLAIM_LOST = 0, CLAIM_WON = 1, CLAIM_SAME = 2 };

// Claim slot q of the bucket starting at `bucket` for value e, by a single
// lane on behalf of its own key (the pipelined paths let every key's owner
// lane claim at once).  `word` is the snapshot of the 32-bit word holding the
// slot (used by 16-bit slots only).  Returns CLAIM_WON if this call stored e,
// CLAIM_SAME if the slot already holds e (another operation stored the same
// key: the CAS result stands in for a re-read, Sec. 4.2 implementation
// notes), CLAIM_LOST otherwise.  16-bit slots have no native CAS: the
// containing 32-bit word is compare-and-swapped, and the attempt repeats only
// while the other half of the word is what changed (a bounded number of
// times: a slot goes from EMPTY to a key, and at most on to a tombstone).
template <int S>
__device__ __forceinline__ int claim_at(uint32_t* bucket, uint32_t q, uint32_t word, uint64_t e) {
  uint64_t got;
  if constexpr (S == 32) {
    got = cas32(bucket + q, 0u, (uint32_t)e);
  } else if constexpr (S == 64) {
    got = cas64(reinterpret_cast<uint64_t*>(bucket + 2 * q), 0ull, e);
  } else {
    const uint32_t wi = q >> 1;
    const int sh = (int)(q & 1u) * 16;
    const uint32_t mine = (uint32_t)e << sh;
    uint32_t cur = word & ~(0xFFFFu << sh);
    for (;;) {
      const uint32_t old = cas32(bucket + wi, cur, cur | mine);
      if (old == cur) { got = 0; break; }
      got = (old >> sh) & 0xFFFFu;
      if (got) break;
      cur = old;
    }
  }
  if (got == 0) return CLAIM_WON;
  return got == e ? CLAIM_SAME : CLAIM_LOST;
}

// Delete: replace the stored form e in slot q by the tombstone.  True if
// this call did it, false if the slot no longer holds e (a concurrent delete
// of the same key won).  16-bit slots compare-and-swap the containing word,
// repeating only while the other half of the word is what changed.
template <int S>
__device__ __forceinline__ bool erase_at(uint32_t* bucket, uint32_t q, uint32_t word, uint64_t e) {
  if constexpr (S == 32) {
    return cas32(bucket + q, (uint32_t)e, (uint32_t)TOMB) == (uint32_t)e;
  } else if constexpr (S == 64) {
    return cas64(reinterpret_cast<uint64_t*>(bucket + 2 * q), e, TOMB) == e;
  } else {
    const uint32_t wi = q >> 1;
    const int sh = (int)(q & 1u) * 16;
    const uint32_t keep = ~(0xFFFFu << sh);
    uint32_t cur = (word & keep) | ((uint32_t)e << sh);
    for (;;) {
      const uint32_t old = cas32(bucket + wi, cur, (cur & keep) | ((uint32_t)TOMB << sh));
      if (old == cur) return true;
      if (((old >> sh) & 0xFFFFu) != (uint32_t)e) return false;
      cur = old;
    }
  }
}

// Swap bucket slot q with value e (cuckoo eviction); returns the old value.
template <int S>
__device__ __forceinline__ uint64_t swap_at(uint32_t* bucket, uint32_t q, uint64_t e) {
  static_assert(S == 32 || S == 64, "swap needs a native atomic exchange");
  if constexpr (S == 32) return xchg32(bucket + q, (uint32_t)e);
  else return xchg64(reinterpret_cast<uint64_t*>(bucket + 2 * q), e);
}

// Known-occupied mask of a bucket (one bit per slot), as broadcast within a
// sub-tile: 32 bits for buckets of up to 32 slots, 64 bits otherwise.
template <int B>
using KnownMask = typename std::conditional<(B <= 32), uint32_t, uint64_t>::type;

// The bits of a bucket mask that belong to the lane holding slots
// [first, first + PER).
template <int PER, class M>
__device__ __forceinline__ uint32_t lane_bits(M mask, int first) {
  const uint64_t m = (uint64_t)mask >> first;
  return PER >= 32 ? (uint32_t)m : (uint32_t)(m & ((1ull << PER) - 1ull));
}

// ---------------------------------------------------------------------------
// Sub-tile collectives over a 64-lane wavefront.  Every lane of a sub-tile
// executes them together (control flow is uniform per sub-tile).
// ---------------------------------------------------------------------------

template <int G>
struct SubTile {
  static_assert(G >= 2 && G <= 32 && (G & (G - 1)) == 0, "sub-tile width");
  int lane;   // lane in the wavefront
  int rk;     // rank in the sub-tile
  int base;   // first lane of the sub-tile
  __device__ __forceinline__ SubTile() {
    lane = (int)(threadIdx.x & 63u);
    rk = lane & (G - 1);
    base = lane & ~(G - 1);
  }
  static constexpr uint32_t full_mask() { return G == 32 ? 0xFFFFFFFFu : ((1u << G) - 1u); }
  // Ballot restricted to this sub-tile: bit r set iff predicate holds at rank r.
  __device__ __forceinline__ uint32_t ballot(bool p) const {
    uint64_t m = __ballot(p);
    return (uint32_t)(m >> base) & full_mask();
  }
  // Shuffle: the value v of rank src_rank, to every lane of the sub-tile.
  __device__ __forceinline__ uint32_t bcast(uint32_t v, int src_rank) const {
    return (uint32_t)__builtin_amdgcn_ds_bpermute((base + src_rank) << 2, (int)v);
  }
  __device__ __forceinline__ uint64_t bcast64(uint64_t v, int src_rank) const {
    uint32_t lo = bcast((uint32_t)v, src_rank);
    uint32_t hi = bcast((uint32_t)(v >> 32), src_rank);
    return (uint64_t)lo | ((uint64_t)hi << 32);
  }
  __device__ __forceinline__ bool bcast_bool(bool v, int src_rank) const {
    return bcast((uint32_t)v, src_rank) != 0u;
  }
  template <class M>
  __device__ __forceinline__ M bcast_mask(M v, int src_rank) const {
    if constexpr (sizeof(M) == 8) return (M)bcast64((uint64_t)v, src_rank);
    else return (M)bcast((uint32_t)v, src_rank);
  }
  template <int S>
  __device__ __forceinline__ uint64_t bcast_slot(uint64_t v, int src_rank) const {
    if constexpr (S == 64) return bcast64(v, src_rank);
    else return bcast((uint32_t)v, src_rank);
  }
};

__device__ __forceinline__ int ctz32(uint32_t m) { return __builtin_ctz(m); }

}  // namespace cpht
