// Compact two-level iceberg table: lockless find-or-put (Sec. 3 Alg. 1; its
// cooperative form Sec. 4.2 Alg. 2), lookup (Sec. 2.3), and the batch work
// sharing of Sec. 4.2 Alg. 3 for batches of any size.
//
// Sub-tile layout: G lanes read the primary bucket T0[a_0(k)] (W0 words per
// lane, so B0 = G*W0*32/S0).  On the second level the sub-tile splits into two
// contiguous halves; half h reads secondary bucket T1[a_{1+h}(k)] (W1 words
// per lane, B1 = (G/2)*W1*32/S1).  The paper splits by even/odd rank; which
// lanes serve which bucket does not change what is computed.
//
// Execution is organised in supersteps.  Each superstep has a level-1 part
// and a level-2 part; in each part a sub-tile first issues the bucket loads of
// all its keys that are at that level, then decides every key with sub-tile
// ballots, and finally each key that needs a claim has its own lane CAS the
// chosen slot, all owner lanes at once.  A lost claim marks that slot
// known-occupied for the key and the key stays pending, so every superstep
// either decides a key or learns one more occupied slot of its buckets; that
// bounds a key to B0 + 2*B1 lost claims (the termination argument of the
// proof in Appendix A), also when a re-read returns stale data.
#pragma once
#include "cpht_device.hpp"

namespace cpht {

enum : int { MODE_FIND = 0, MODE_INSERT = 1, MODE_MIXED = 2, MODE_ERASE = 3, MODE_FIND_V = 4, MODE_INSERT_V = 5 };

template <int S0, int S1, int B0, int B1, int G>
struct IceShape {
  static constexpr int W0 = B0 * S0 / (32 * G);
  static constexpr int W1 = 2 * B1 * S1 / (32 * G);
  static constexpr int HG = G / 2;
  static constexpr int PER0 = W0 * 32 / S0;
  static constexpr int PER1 = W1 * 32 / S1;
  static_assert(W0 >= 1 && W0 * 32 * G == B0 * S0, "primary bucket must split into whole words per lane");
  static_assert(W1 >= 1 && W1 * 32 * HG == B1 * S1, "secondary bucket must split into whole words per lane");
  static_assert(PER0 * G == B0 && PER1 * HG == B1, "slots per lane");
};

// Third level: a 128-byte slab read by the whole sub-tile, W3 words per
// lane; slots of S3 = 32 bits (64 for 64-bit primary slots), the last slot of
// a slab holding the next slab id.  Compiled only where every lane holds whole
// slots (not for 64-bit slots with 32 lanes).
template <int S0, int G>
struct L3Shape {
  static constexpr int S3 = S0 == 64 ? 64 : 32;
  static constexpr int W3 = 32 / G;
  static constexpr bool OK = W3 * 32 >= S3;
  static constexpr int PER3 = OK ? W3 * 32 / S3 : 1;
  static constexpr int B3 = 1024 / S3;
  static constexpr int LINK = B3 - 1;             // slot index of the link
  static constexpr int LINK_WORD = S3 == 32 ? 31 : 30;  // its word in the slab
  static constexpr int LINK_LANE_WORD = OK ? LINK_WORD - (G - 1) * W3 : 0;  // in the last lane
};

// A list head or slab link being set: the value a key writes (by CAS from 0)
// before it takes a slab from the pool and publishes the slab's id there.
// Never a slab id (the pool has fewer than 2^31 - 1 slabs) and, with its top
// bit clear, never a stored form.
constexpr uint32_t LINK_BUSY = 0x7FFFFFFFu;

// A fresh slab id from the pool, or 0 when the pool is used up.
__device__ __forceinline__ uint32_t alloc_slab(const Level3K& L3) {
  if (__hip_atomic_load(L3.used, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= L3.nslabs) return 0u;
  const uint32_t id = __hip_atomic_fetch_add(L3.used, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
  return id <= L3.nslabs ? id : 0u;
}

// Keys whose buckets one sub-tile loads together, within a budget of REGS
// registers per lane for the buffers.  Level 1 gets 32.  Levels 2 and 3 get
// 16: only keys whose primary bucket is full reach them, yet their buffers
// set the kernel's peak register count; with 32 they held the 16/32-bit,
// 32-slot kernels at 4 waves per SIMD instead of 5 (3 instead of 4 with the
// third level).
template <int G, int W, int REGS = 32>
struct IceDepth {
  static constexpr int D = G * W <= REGS ? G : (REGS / W > 0 ? REGS / W : 1);
  static_assert(G % D == 0, "prefetch depth must divide the sub-tile");
};

// Batch kernel.  Lane i owns key i (coalesced load) and its result byte.
//   Level 1 (Alg. 1, first loop): k's remainder in the primary snapshot ->
//     FOUND (lookup: 1); an empty slot -> lookup answers 0, find-or-put claims
//     the first empty slot; primary full -> level 2.
//   Level 2 (Alg. 1, second loop): k's tagged remainder in either secondary
//     snapshot -> FOUND (lookup: 1; lookup otherwise 0); else the target is
//     the first empty slot of bucket 1 if bucket 1 is strictly less full than
//     bucket 2, else of bucket 2 (the least empty slot under the order of
//     Appendix A, Def. 1); FULL if the target bucket has no empty slot.
//   A claim that finds k's own stored form in the slot answers FOUND.
// MODE_MIXED reads a per-key opcode (0 = find, 1 = find-or-put).
// MODE_ERASE follows the lookup and replaces the slot holding k's stored form
// by the tombstone with CAS (answer 1 if this operation did it, else 0).
// Tombstones count as occupied everywhere and are never claimed, so the
// order property and the lookup's early exit hold with deletes.
// L3ON compiles the third level in (tables with a slab pool); without it the
// two-level kernels carry none of its registers.
// MODE_FIND_V / MODE_INSERT_V are lookup / find-or-put of a map: the value of
// a key sits at its slot's index in a parallel array (the table is stable);
// the insert that stores a key writes its value, a lookup that finds the key
// returns it.
template <class KeyT, int S0, int S1, int B0, int B1, int G, int MODE_, bool L3ON>
__device__ __forceinline__ void iceberg_body(const TableK& T, const BatchK& Bt, uint64_t idx) {
  constexpr bool VALS = MODE_ == MODE_FIND_V || MODE_ == MODE_INSERT_V;
  constexpr int MODE = MODE_ == MODE_FIND_V ? MODE_FIND : MODE_ == MODE_INSERT_V ? MODE_INSERT : MODE_;
  constexpr bool WRITES = MODE == MODE_INSERT || MODE == MODE_MIXED;  // find-or-put claims
  using U = KeyT;
  using Sh = IceShape<S0, S1, B0, B1, G>;
  using KM0 = KnownMask<B0>;
  using KM1 = KnownMask<B1>;
  constexpr int W0 = Sh::W0, W1 = Sh::W1, PER0 = Sh::PER0, PER1 = Sh::PER1, HG = Sh::HG;
  constexpr int D0 = IceDepth<G, W0>::D, D1 = IceDepth<G, W1, 16>::D;
  const SubTile<G> st;
  const LevelK& L0 = T.lv[0];
  const LevelK& L1 = T.lv[1];
  const bool act = idx < Bt.n;
  const U k = act ? static_cast<const U*>(Bt.keys)[idx] : (U)0;
  bool ins = MODE == MODE_INSERT;
  if constexpr (MODE == MODE_MIXED) ins = act && Bt.ops[idx] != 0;
  const Split<U, S0> s0 = split_key<U, S0>(T, L0, 0, k, 0u);
  Split<U, S1> s1{0, 0}, s2{0, 0};
  bool have12 = false;
  uint8_t result = 0;
  uint32_t stage = act ? 1u : 0u;  // 0 decided, 1 at level 1, 2 at level 2
  KM0 known0 = 0;                  // primary slots known to be occupied
  KM1 known1 = 0, known2 = 0;      // same for the two secondary buckets
  const int half = st.rk >= HG ? 1 : 0;
  const int hr = st.rk & (HG - 1);
  const uint32_t hmask = HG == 32 ? 0xFFFFFFFFu : ((1u << HG) - 1u);
  // level 3 (stage 3): the key's list and stored form, the slab being read
  // (0 = list head not read yet), and slab slots known to be occupied (the
  // link slot always)
  using L3 = L3Shape<S0, G>;
  constexpr int S3 = L3::S3, W3 = L3::W3, PER3 = L3::PER3;
  constexpr uint32_t LINKBIT = 1u << L3::LINK;
  constexpr bool L3C = L3ON && L3::OK;  // level-3 code compiled in
  const bool l3on = L3C && T.l3.nslabs != 0u;
  Split<U, S3> s3{0, 0};
  uint32_t cur = 0, known3 = 0;

#pragma unroll 1
  while (__ballot(stage != 0u) != 0ull) {
    // ------------------------------------------------------------ level 1
    if (__ballot(stage == 1u) != 0ull) {
      bool claim = false, erase = false;
      uint32_t q = 0, word = 0;
#pragma unroll 1
      for (int t0 = 0; t0 < G; t0 += D0) {
        uint32_t buf[D0][W0];
        uint64_t ev[D0];
        KM0 kn[D0];
        bool live[D0];
#pragma unroll
        for (int d = 0; d < D0; ++d) {
          live[d] = st.bcast(stage, t0 + d) == 1u;
          const uint32_t a = st.bcast((uint32_t)s0.a, t0 + d);
          ev[d] = st.template bcast_slot<S0>(s0.e, t0 + d);
          if constexpr (WRITES) kn[d] = st.bcast_mask(known0, t0 + d);
          if (live[d]) load_words<W0>(buf[d], L0.base + (uint64_t)a * L0.bucket_words + (uint32_t)(st.rk * W0));
        }
#pragma unroll
        for (int d = 0; d < D0; ++d) {
          if (!live[d]) continue;
          const bool mine = st.rk == t0 + d;
          const bool ins_t = MODE == MODE_MIXED ? st.bcast_bool(ins, t0 + d) : MODE == MODE_INSERT;
          const uint32_t hits = st.ballot(lane_has<S0, W0>(buf[d], ev[d]));
          if (hits) {
            if constexpr (MODE == MODE_ERASE) {
              const int f = ctz32(hits);
              const uint32_t i = st.bcast((uint32_t)lane_match<S0, W0>(buf[d], ev[d]), f);
              uint32_t wf = 0;
              if constexpr (S0 == 16) wf = st.bcast(get_word<W0>(buf[d], (int)(i >> 1)), f);
              if (mine) { erase = true; q = (uint32_t)(f * PER0) + i; word = wf; stage = 0; }
            } else if constexpr (VALS && MODE == MODE_FIND) {
              const int f = ctz32(hits);
              const uint32_t i = st.bcast((uint32_t)lane_match<S0, W0>(buf[d], ev[d]), f);
              if (mine) {
                result = 1;
                stage = 0;
                get_value(T, 0, s0.a * B0 + (uint64_t)(f * PER0) + i, Bt, idx);
              }
            } else {
              if (mine) { result = ins_t ? R_FOUND : 1; stage = 0; }
            }
            continue;
          }
          KM0 knd = 0;
          if constexpr (WRITES) knd = kn[d];
          const int le = lane_first_empty<S0, W0>(buf[d], ins_t ? lane_bits<PER0>(knd, st.rk * PER0) : 0u);
          const uint32_t em = st.ballot(le < PER0);
          if (!em) {
            if (mine) stage = 2;  // primary full
            continue;
          }
          if (!ins_t) {
            if (mine) { result = 0; stage = 0; }
            continue;
          }
          const int f = ctz32(em);
          const uint32_t lef = st.bcast((uint32_t)le, f);
          uint32_t wf = 0;
          if constexpr (S0 == 16) wf = st.bcast(get_word<W0>(buf[d], (int)(lef >> 1)), f);
          if (mine) { claim = true; q = (uint32_t)(f * PER0) + lef; word = wf; }
        }
      }
      if constexpr (WRITES) {
        if (claim) {
          const int r = claim_at<S0>(L0.base + s0.a * L0.bucket_words, q, word, s0.e);
          if (r == CLAIM_WON) {
            result = R_PUT;
            stage = 0;
            if constexpr (VALS) put_value(T, 0, s0.a * B0 + q, Bt, idx);
          }
          else if (r == CLAIM_SAME) { result = R_FOUND; stage = 0; }
          else known0 |= (KM0)1 << q;
        }
      }
      if constexpr (MODE == MODE_ERASE) {
        if (erase) result = erase_at<S0>(L0.base + s0.a * L0.bucket_words, q, word, s0.e) ? 1 : 0;
      }
    }
    // ------------------------------------------------------------ level 2
    if (__ballot(stage == 2u) != 0ull) {
      if (stage == 2u && !have12) {
        s1 = split_key<U, S1>(T, L1, 1, k, 0u);
        s2 = split_key<U, S1>(T, L1, 2, k, 1u);
        have12 = true;
      }
      bool claim = false, erase = false;
      uint32_t q = 0, word = 0, pick2 = 0;
#pragma unroll 1
      for (int t0 = 0; t0 < G; t0 += D1) {
        uint32_t buf[D1][W1];
        uint64_t ev[D1];
        KM1 kn[D1];
        bool live[D1];
#pragma unroll
        for (int d = 0; d < D1; ++d) {
          live[d] = st.bcast(stage, t0 + d) == 2u;
          const uint32_t a1 = st.bcast((uint32_t)s1.a, t0 + d);
          const uint32_t a2 = st.bcast((uint32_t)s2.a, t0 + d);
          const uint64_t e1 = st.template bcast_slot<S1>(s1.e, t0 + d);
          const uint64_t e2 = st.template bcast_slot<S1>(s2.e, t0 + d);
          if constexpr (WRITES) {
            const KM1 k1 = st.bcast_mask(known1, t0 + d);
            const KM1 k2 = st.bcast_mask(known2, t0 + d);
            kn[d] = half ? k2 : k1;
          }
          ev[d] = half ? e2 : e1;
          const uint32_t a = half ? a2 : a1;
          if (live[d]) load_words<W1>(buf[d], L1.base + (uint64_t)a * L1.bucket_words + (uint32_t)(hr * W1));
        }
#pragma unroll
        for (int d = 0; d < D1; ++d) {
          if (!live[d]) continue;
          const bool mine = st.rk == t0 + d;
          const bool ins_t = MODE == MODE_MIXED ? st.bcast_bool(ins, t0 + d) : MODE == MODE_INSERT;
          const uint32_t hits = st.ballot(lane_has<S1, W1>(buf[d], ev[d]));
          if (hits) {
            if constexpr (MODE == MODE_ERASE) {
              // lanes [0, HG) read secondary bucket 1, lanes [HG, G) bucket 2
              const int f = ctz32(hits);
              const uint32_t i = st.bcast((uint32_t)lane_match<S1, W1>(buf[d], ev[d]), f);
              uint32_t wf = 0;
              if constexpr (S1 == 16) wf = st.bcast(get_word<W1>(buf[d], (int)(i >> 1)), f);
              if (mine) {
                erase = true;
                pick2 = f >= HG ? 1u : 0u;
                q = (uint32_t)((f & (HG - 1)) * PER1) + i;
                word = wf;
                stage = 0;
              }
            } else if constexpr (VALS && MODE == MODE_FIND) {
              const int f = ctz32(hits);
              const uint32_t i = st.bcast((uint32_t)lane_match<S1, W1>(buf[d], ev[d]), f);
              if (mine) {
                result = 1;
                stage = 0;
                const uint64_t ab = f >= HG ? s2.a : s1.a;
                get_value(T, 1, ab * B1 + (uint64_t)((f & (HG - 1)) * PER1) + i, Bt, idx);
              }
            } else {
              if (mine) { result = ins_t ? R_FOUND : 1; stage = 0; }
            }
            continue;
          }
          if (!ins_t) {
            // k can only be on level 3 if both secondary buckets are full
            bool to3 = false;
            if (l3on) to3 = st.ballot(lane_first_empty<S1, W1>(buf[d], 0u) < PER1) == 0u;
            if (mine) {
              if (to3) { stage = 3; s3 = split_key<U, S3>(T, T.l3.L, 0, k, 0u); cur = 0; known3 = LINKBIT; }
              else { result = 0; stage = 0; }
            }
            continue;
          }
          KM1 knd = 0;
          if constexpr (WRITES) knd = kn[d];
          const int le = lane_first_empty<S1, W1>(buf[d], lane_bits<PER1>(knd, hr * PER1));
          const uint32_t em = st.ballot(le < PER1);
          const uint32_t em1 = em & hmask, em2 = em >> HG;
          uint32_t l1 = B1, l2 = B1;
          int f1 = 0, f2 = HG;
          if (em1) { f1 = ctz32(em1); l1 = (uint32_t)(f1 * PER1) + st.bcast((uint32_t)le, f1); }
          if (em2) { f2 = HG + ctz32(em2); l2 = (uint32_t)((f2 - HG) * PER1) + st.bcast((uint32_t)le, f2); }
          const bool p1 = l1 < l2;  // bucket 1 only if strictly less full (ties go to bucket 2)
          const uint32_t lp = p1 ? l1 : l2;
          if (lp == (uint32_t)B1) {  // both secondary buckets full
            if (mine) {
              if (l3on) { stage = 3; s3 = split_key<U, S3>(T, T.l3.L, 0, k, 0u); cur = 0; known3 = LINKBIT; }
              else { result = R_FULL; stage = 0; }
            }
            continue;
          }
          uint32_t wf = 0;
          if constexpr (S1 == 16) wf = st.bcast(get_word<W1>(buf[d], (int)((lp % PER1) >> 1)), p1 ? f1 : f2);
          if (mine) { claim = true; q = lp; word = wf; pick2 = p1 ? 0u : 1u; }
        }
      }
      if constexpr (MODE == MODE_ERASE) {
        if (erase) {
          const uint64_t ab = pick2 ? s2.a : s1.a;
          const uint64_t e = pick2 ? s2.e : s1.e;
          result = erase_at<S1>(L1.base + ab * L1.bucket_words, q, word, e) ? 1 : 0;
        }
      }
      if constexpr (WRITES) {
        if (claim) {
          const uint64_t ab = pick2 ? s2.a : s1.a;
          const uint64_t e = pick2 ? s2.e : s1.e;
          const int r = claim_at<S1>(L1.base + ab * L1.bucket_words, q, word, e);
          if (r == CLAIM_WON) {
            result = R_PUT;
            stage = 0;
            if constexpr (VALS) put_value(T, 1, ab * B1 + q, Bt, idx);
          }
          else if (r == CLAIM_SAME) { result = R_FOUND; stage = 0; }
          else if (pick2) known2 |= (KM1)1 << q;
          else known1 |= (KM1)1 << q;
        }
      }
    }
    // ------------------------------------------------------------ level 3
    // The list of k, slab by slab in list order: k's stored form before the
    // first empty slot -> FOUND (lookup 1); else an insert claims the first
    // empty slot (a lookup answers 0); a full slab is followed through its
    // link.  An insert at an empty list or a full last slab sets the link:
    // CAS 0 -> LINK_BUSY, and only the key that wins takes a slab from the
    // pool and publishes its id (or 0 again, and FULL, when the pool is used
    // up); a key that finds the link busy keeps its place and retries the CAS
    // next superstep (a CAS result is never stale), so no slab is taken
    // twice and every list is a chain set once per link, filling in one
    // order as a bucket does.  A lookup treats a busy or empty link as the
    // end of the list.
    if constexpr (L3C) {
      if (__ballot(stage == 3u) != 0ull) {
        bool link = false, claim = false, erase = false;
        uint32_t q = 0;
        if (stage == 3u && cur == 0u) {  // read the list head
          const uint32_t h = T.l3.heads[s3.a];
          if (h != 0u && h != LINK_BUSY) cur = h;
          else if (ins) link = true;
          else { result = 0; stage = 0; }
        }
        constexpr int D3 = IceDepth<G, W3, 16>::D;
#pragma unroll 1
        for (int t0 = 0; t0 < G; t0 += D3) {
          uint32_t buf[D3][W3];
          uint64_t ev[D3];
          uint32_t kn[D3];
          bool live[D3];
#pragma unroll
          for (int d = 0; d < D3; ++d) {
            live[d] = st.bcast_bool(stage == 3u && cur != 0u && !link, t0 + d);
            const uint32_t id = st.bcast(cur, t0 + d);
            ev[d] = st.template bcast_slot<S3>(s3.e, t0 + d);
            kn[d] = st.bcast(known3, t0 + d);
            if (live[d]) load_words<W3>(buf[d], T.l3.L.base + (uint64_t)(id - 1u) * 32u + (uint32_t)(st.rk * W3));
          }
#pragma unroll
          for (int d = 0; d < D3; ++d) {
            if (!live[d]) continue;
            const bool mine = st.rk == t0 + d;
            const bool ins_t = MODE == MODE_MIXED ? st.bcast_bool(ins, t0 + d) : MODE == MODE_INSERT;
            const uint32_t hits = st.ballot(lane_has<S3, W3>(buf[d], ev[d]));
            if (hits) {
              if constexpr (MODE == MODE_ERASE) {
                const int f = ctz32(hits);
                const uint32_t i = st.bcast((uint32_t)lane_match<S3, W3>(buf[d], ev[d]), f);
                if (mine) { erase = true; q = (uint32_t)(f * PER3) + i; stage = 0; }
              } else if constexpr (VALS && MODE == MODE_FIND) {
                const int f = ctz32(hits);
                const uint32_t i = st.bcast((uint32_t)lane_match<S3, W3>(buf[d], ev[d]), f);
                if (mine) {
                  result = 1;
                  stage = 0;
                  get_value(T, 2, (uint64_t)(cur - 1u) * L3::B3 + (uint64_t)(f * PER3) + i, Bt, idx);
                }
              } else {
                if (mine) { result = ins_t ? R_FOUND : 1; stage = 0; }
              }
              continue;
            }
            const uint32_t knd = ins_t ? kn[d] : LINKBIT;
            const int le = lane_first_empty<S3, W3>(buf[d], lane_bits<PER3>(knd, st.rk * PER3));
            const uint32_t em = st.ballot(le < PER3);
            if (em) {
              if (!ins_t) {
                if (mine) { result = 0; stage = 0; }
                continue;
              }
              const int f = ctz32(em);
              const uint32_t lef = st.bcast((uint32_t)le, f);
              if (mine) { claim = true; q = (uint32_t)(f * PER3) + lef; }
              continue;
            }
            // slab full: its link
            const uint32_t nx = st.bcast(buf[d][L3::LINK_LANE_WORD], G - 1);
            if (mine) {
              if (nx != 0u && nx != LINK_BUSY) { cur = nx; known3 = LINKBIT; }
              else if (ins_t) link = true;
              else { result = 0; stage = 0; }
            }
          }
        }
        uint32_t* slab = T.l3.L.base + (uint64_t)(cur - 1u) * 32u;
        if constexpr (MODE == MODE_ERASE) {
          if (erase) result = erase_at<S3>(slab, q, 0u, s3.e) ? 1 : 0;
        }
        if constexpr (WRITES) {
          if (claim) {
            const int r = claim_at<S3>(slab, q, 0u, s3.e);
            if (r == CLAIM_WON) {
              result = R_PUT;
              stage = 0;
              if constexpr (VALS) put_value(T, 2, (uint64_t)(cur - 1u) * L3::B3 + q, Bt, idx);
            }
            else if (r == CLAIM_SAME) { result = R_FOUND; stage = 0; }
            else known3 |= 1u << q;
          }
          if (link) {  // a new slab at the list head or after the full last slab
            uint32_t* at = cur ? slab + L3::LINK_WORD : T.l3.heads + s3.a;
            const uint32_t old = cas32(at, 0u, LINK_BUSY);
            if (old == 0u) {
              const uint32_t sl = alloc_slab(T.l3);
              xchg32(at, sl);  // publish the slab, or release the link when the pool is used up
              if (sl == 0u) { result = R_FULL; stage = 0; }
              else { cur = sl; known3 = LINKBIT; }
            } else if (old != LINK_BUSY) {  // linked by another key meanwhile
              cur = old;
              known3 = LINKBIT;
            }
          }
        }
      }
    }
  }
  if (act) Bt.out[idx] = result;
}

// One table: key i of the batch is handled by global thread i.
template <class KeyT, int S0, int S1, int B0, int B1, int G, int MODE, bool L3ON>
__global__ __launch_bounds__(256) void iceberg_kernel(TableK T, BatchK Bt) {
  iceberg_body<KeyT, S0, S1, B0, B1, G, MODE, L3ON>(T, Bt, (uint64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Many tables in one persistent launch: a fixed grid of blocks walks the
// chunks of its variant group (each chunk = up to 256 consecutive keys of one
// table), reading that table's description from device memory.
template <class KeyT, int S0, int S1, int B0, int B1, int G, int MODE>
__global__ __launch_bounds__(256) void iceberg_multi_kernel(MultiK M) {
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
    iceberg_body<KeyT, S0, S1, B0, B1, G, MODE, false>(T, Bt, threadIdx.x);
  }
}

}  // namespace cpht
