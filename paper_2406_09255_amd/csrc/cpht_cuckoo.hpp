// Compact bucketed cuckoo table: parallel put (Sec. 4.4, Alg. 4) and lookup
// (Sec. 4.4 "Lookup"), with the sub-tile work sharing of Sec. 4.2.
//
// One sub-tile of G lanes reads a bucket of B = G*W*32/S slots, W words per
// lane.  Each slot holds (r_j(k), j): occupancy bit, hash index j, and the
// remainder of pi_j(k) (or all of pi_j(k) for the non-compact table).
//
// Execution is organised in supersteps.  In every superstep each sub-tile
// first issues the bucket loads of all its pending keys (so a wave keeps up
// to 64 bucket reads in flight), then resolves each key with sub-tile
// ballots, and finally every pending key's own lane performs that key's
// atomic (CAS into the first empty slot, or the eviction swap) at the same
// time as all other owner lanes.  A key therefore advances exactly one round
// of Alg. 4 per superstep.
#pragma once
#include "cpht_device.hpp"

namespace cpht {

template <int S, int B, int G>
struct CkShape {
  static constexpr int W = B * S / (32 * G);
  static constexpr int PER = W * 32 / S;
  static_assert(S == 32 || S == 64, "cuckoo slots are 32 or 64 bits (native CAS and swap)");
  static_assert(W >= 1 && W * 32 * G == B * S && PER * G == B, "bucket must split into whole words per lane");
};

// Keys whose buckets one sub-tile loads together: every key of the sub-tile,
// as long as the buffers stay within 32 registers per lane.
template <int G, int W>
struct Depth {
  static constexpr int D = G * W <= 32 ? G : (32 / W > 0 ? 32 / W : 1);
  static_assert(G % D == 0, "prefetch depth must divide the sub-tile");
};

enum : int { CK_FIND = 0, CK_PUT = 1, CK_ERASE = 2 };

// Batch kernel, one operation per key:
//   CK_FIND: buckets a_0(k), a_1(k), ... in order; a hit answers 1, a bucket
//     that is not full and lacks (r_j(k), j) answers 0 (keys are only pushed
//     to hash j+1 out of a full bucket, so k cannot be further on; tombstones
//     count as occupied, so deletes keep this true).
//   CK_PUT: Alg. 4.  Per round, the bucket T[a_j(k)] of the carried key k is
//     snapshotted; with an empty slot, one is claimed with CAS: the first
//     empty slot at or after a start slot drawn from (k, round), else the
//     first empty slot (Alg. 4 asks for some empty slot; spreading the claims
//     of keys that share a bucket lets several of them win in one round).  A
//     lost claim uses up the round and marks the slot known-occupied, so a
//     stale re-read cannot offer it again.  Buckets therefore need not fill as
//     a prefix, which the lookup does not rely on: it asks whether the bucket
//     holds the key and whether any slot is empty.  With no empty slot, the victim row
//     chosen from (k, round) is swapped with (r_j(k), j) and the evicted pair
//     (r', j') continues as key pi_{j'}^{-1}(a . r') with hash index j'+1 mod
//     H; a tombstone as victim ends the chain (nothing is carried).  After C
//     rounds the carried key is dropped and the result is FULL.
//   CK_ERASE: the lookup's probe sequence; the slot holding (r_j(k), j) is
//     replaced by the tombstone with CAS; answers 1 if this operation did it.
template <class KeyT, int S, int B, int G, int OP>
__device__ __forceinline__ void cuckoo_body(const TableK& T, const BatchK& Bt, uint64_t idx) {
  constexpr bool PUT = OP == CK_PUT;
  using U = KeyT;
  using Sh = CkShape<S, B, G>;
  using KM = KnownMask<B>;
  constexpr int W = Sh::W, PER = Sh::PER, D = Depth<G, W>::D;
  const SubTile<G> st;
  const LevelK& L = T.lv[0];
  const bool act = idx < Bt.n;
  U k = act ? static_cast<const U*>(Bt.keys)[idx] : (U)0;
  Split<U, S> s = split_key<U, S>(T, L, 0, k, 0u);
  uint8_t result = 0;
  bool pend = act;   // this lane's key still needs work
  uint32_t j = 0;    // hash index of the (carried) key
  uint32_t c = 1;    // Alg. 4 round
  KM known = 0;      // slots of bucket s.a known to be occupied

#pragma unroll 1
  while (__ballot(pend) != 0ull) {
    bool claim = false, evict = false, erase = false;
    uint32_t q = 0;
    uint32_t start = 0;  // first slot the claim of this round looks at
    if constexpr (PUT) start = claim_start((uint64_t)k, c, (uint32_t)B);
#pragma unroll 1
    for (int t0 = 0; t0 < G; t0 += D) {
      uint32_t buf[D][W];
      uint64_t ev[D];
      KM kn[D];
      uint32_t p0[D];
      bool live[D];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        live[d] = st.bcast_bool(pend, t0 + d);
        const uint32_t a = st.bcast((uint32_t)s.a, t0 + d);
        if constexpr (!PUT) {
          ev[d] = st.template bcast_slot<S>(s.e, t0 + d);
        } else {
          kn[d] = st.bcast_mask(known, t0 + d);
          p0[d] = st.bcast(start, t0 + d);
        }
        if (live[d]) load_words<W>(buf[d], L.base + (uint64_t)a * L.bucket_words + (uint32_t)(st.rk * W));
      }
#pragma unroll
      for (int d = 0; d < D; ++d) {
        if (!live[d]) continue;
        const bool mine = st.rk == t0 + d;
        if constexpr (!PUT) {
          const uint32_t hits = st.ballot(lane_has<S, W>(buf[d], ev[d]));
          const bool room = st.ballot(lane_first_empty<S, W>(buf[d], 0u) < PER) != 0u;
          if constexpr (OP == CK_ERASE) {
            if (hits) {
              const int f = ctz32(hits);
              const uint32_t qq = (uint32_t)(f * PER) + st.bcast((uint32_t)lane_match<S, W>(buf[d], ev[d]), f);
              if (mine) { erase = true; q = qq; pend = false; }
              continue;
            }
          }
          if (mine && (hits || room)) {
            result = hits ? 1 : 0;
            pend = false;
          }
        } else {
          const uint32_t kb = lane_bits<PER>(kn[d], st.rk * PER);
          // this lane's slots that lie before the start slot
          const int before = min(max((int)p0[d] - st.rk * PER, 0), PER);
          const uint32_t skip = before >= 32 ? 0xFFFFFFFFu : ((1u << before) - 1u);
          const int le_from = lane_first_empty<S, W>(buf[d], kb | skip);
          const int le_any = lane_first_empty<S, W>(buf[d], kb);
          const uint32_t em_from = st.ballot(le_from < PER);
          const uint32_t em = st.ballot(le_any < PER);
          if (em) {
            const int f = ctz32(em_from ? em_from : em);
            const uint32_t qq = (uint32_t)(f * PER) + st.bcast((uint32_t)(em_from ? le_from : le_any), f);
            if (mine) { claim = true; q = qq; }
          } else if (mine) {
            evict = true;
          }
        }
      }
    }
    if constexpr (!PUT) {
      if constexpr (OP == CK_ERASE) {
        if (erase) result = erase_at<S>(L.base + s.a * L.bucket_words, q, 0u, s.e) ? 1 : 0;
      }
      if (pend) {  // the bucket was full without k: next hash function
        if (++j == T.H) { result = 0; pend = false; }
        else s = split_key<U, S>(T, L, (int)j, k, j);
      }
    } else {
      uint32_t* bucket = L.base + s.a * L.bucket_words;
      if (claim) {
        if (claim_at<S>(bucket, q, 0u, s.e) == CLAIM_WON) {
          result = R_PUT;
          pend = false;
        } else {
          known |= (KM)1 << q;
        }
      } else if (evict) {
        const uint32_t v = victim_row((uint64_t)k, c, (uint32_t)B);
        const uint64_t old = swap_at<S>(bucket, v, s.e);
        if (((old >> (S - 1)) & 1ull) == 0ull) {  // a tombstone: the chain ends here
          result = R_PUT;
          pend = false;
        } else {
          const uint32_t jj = (uint32_t)((old >> L.pbits) & ((1ull << L.tbits) - 1ull));
          k = join_key<U>(T, L, (int)jj, s.a, old);
          j = jj + 1 == T.H ? 0u : jj + 1;
          s = split_key<U, S>(T, L, (int)j, k, j);
          known = 0;
        }
      }
      if (pend && ++c > T.C) {
        result = R_FULL;
        pend = false;
      }
    }
  }
  if (act) Bt.out[idx] = result;
}

// One table: key i of the batch is handled by global thread i.
template <class KeyT, int S, int B, int G, int OP>
__global__ __launch_bounds__(256) void cuckoo_kernel(TableK T, BatchK Bt) {
  cuckoo_body<KeyT, S, B, G, OP>(T, Bt, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Many tables in one persistent launch (see iceberg_multi_kernel).
template <class KeyT, int S, int B, int G, int OP>
__global__ __launch_bounds__(256) void cuckoo_multi_kernel(MultiK M) {
  const uint64_t first = M.group[0], count = M.group[1];
#pragma unroll 1
  for (uint64_t c = blockIdx.x; c < count; c += gridDim.x) {
    const ChunkK ch = M.chunks[first + c];
    const TableK& T = M.descs[ch.table];
    BatchK Bt;
    Bt.keys = static_cast<const KeyT*>(M.keys) + ch.start;
    Bt.ops = nullptr;
    Bt.out = M.out + ch.start;
    Bt.n = ch.count;
    cuckoo_body<KeyT, S, B, G, OP>(T, Bt, threadIdx.x);
  }
}

}  // namespace cpht
