// Compact two-level iceberg table: cooperative find-or-put (Sec. 3 Alg. 1 in
// its cooperative form, Sec. 4.2 Alg. 2), lookup (Sec. 2.3), and the batch
// work sharing of Sec. 4.2 Alg. 3 generalised to any batch size.
//
// Sub-tile layout: G lanes read the primary bucket T0[a_0(k)] (W0 words per
// lane, so B0 = G*W0*32/S0).  On the second level the sub-tile splits into two
// contiguous halves; half h reads secondary bucket T1[a_{1+h}(k)] (W1 words
// per lane, B1 = (G/2)*W1*32/S1).  The paper splits by even/odd rank; which
// lanes serve which bucket does not change what is computed.
#pragma once
#include "cpht_device.hpp"

namespace cpht {

enum : int { MODE_FIND = 0, MODE_INSERT = 1, MODE_MIXED = 2 };

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

// Second-level part of find-or-put (the level-2 loop of Alg. 1 / Alg. 2).
// Both secondary buckets are snapshotted, one per half sub-tile.  FOUND if
// either holds k's tagged remainder; otherwise the target is the first empty
// slot of bucket 1 if that bucket is strictly less full than bucket 2, else
// of bucket 2 (the least empty slot under the order of Appendix A, Def. 1);
// FULL if the target bucket has no empty slot.  A lost claim merges the value
// that won into the snapshot and the loop repeats.
template <class U, int S0, int S1, int B0, int B1, int G>
__device__ __forceinline__ uint8_t ice_level2(const TableK& T, const SubTile<G>& st, U k, bool insert) {
  using Sh = IceShape<S0, S1, B0, B1, G>;
  constexpr int HG = Sh::HG, W1 = Sh::W1, PER1 = Sh::PER1;
  const int half = st.rk >= HG ? 1 : 0;
  const int hr = st.rk & (HG - 1);
  const LevelK& L = T.lv[1];
  Split<U, S1> s = split_key<U, S1>(T, L, 1 + half, k, (uint32_t)half);
  uint32_t* p = L.base + s.a * L.bucket_words + (uint32_t)(hr * W1);
  uint32_t v[W1];
  uint32_t known = 0;
  load_words<W1>(v, p);
  const uint32_t hmask = HG == 32 ? 0xFFFFFFFFu : ((1u << HG) - 1u);
  for (;;) {
    if (st.ballot(lane_has<S1, W1>(v, s.e))) return R_FOUND;
    if (!insert) return 0;  // lookup: k is in neither secondary bucket
    const int le = lane_first_empty<S1, W1>(v, known);
    const uint32_t em = st.ballot(le < PER1);
    const uint32_t em1 = em & hmask, em2 = em >> HG;
    uint32_t l1 = B1, l2 = B1;
    int f1 = 0, f2 = HG;
    if (em1) { f1 = ctz32(em1); l1 = (uint32_t)(f1 * PER1) + st.bcast((uint32_t)le, f1); }
    if (em2) { f2 = HG + ctz32(em2); l2 = (uint32_t)((f2 - HG) * PER1) + st.bcast((uint32_t)le, f2); }
    const bool pick1 = l1 < l2;
    if ((pick1 ? l1 : l2) == (uint32_t)B1) return R_FULL;
    const int f = pick1 ? f1 : f2;
    int claim = CLAIM_LOST;
    if (st.rk == f) claim = claim_slot<S1, W1>(p, v, known, le, s.e);
    claim = (int)st.bcast((uint32_t)claim, f);
    if (claim == CLAIM_WON) return R_PUT;
    if (claim == CLAIM_SAME) return R_FOUND;
    uint32_t fr[W1];
    load_words<W1>(fr, p);
    merge_words<W1>(v, fr);
  }
}

// Find-or-put (insert = true) or lookup (insert = false) of key k by the whole
// sub-tile.  a0/e0 are k's primary bucket and stored form r_0(k).  The key
// itself is only needed (for pi_1, pi_2) once the primary bucket is full.
template <class U, int S0, int S1, int B0, int B1, int G>
__device__ __forceinline__ uint8_t ice_op(const TableK& T, const SubTile<G>& st, U k_own, int t,
                                          uint32_t a0, uint64_t e0, bool insert) {
  using Sh = IceShape<S0, S1, B0, B1, G>;
  constexpr int W0 = Sh::W0, PER0 = Sh::PER0;
  const LevelK& L = T.lv[0];
  uint32_t* p = L.base + (uint64_t)a0 * L.bucket_words + (uint32_t)(st.rk * W0);
  uint32_t w[W0];
  uint32_t known = 0;
  load_words<W0>(w, p);
  for (;;) {
    if (st.ballot(lane_has<S0, W0>(w, e0))) return insert ? R_FOUND : 1;
    const int le = lane_first_empty<S0, W0>(w, known);
    const uint32_t em = st.ballot(le < PER0);
    if (!em) break;           // primary full: go to level 2
    if (!insert) return 0;    // lookup: a non-full primary bucket without k decides
    const int f = ctz32(em);  // the lane holding the first empty slot
    int claim = CLAIM_LOST;
    if (st.rk == f) claim = claim_slot<S0, W0>(p, w, known, le, e0);
    claim = (int)st.bcast((uint32_t)claim, f);
    if (claim == CLAIM_WON) return R_PUT;
    if (claim == CLAIM_SAME) return R_FOUND;
    uint32_t fr[W0];
    load_words<W0>(fr, p);
    merge_words<W0>(w, fr);
  }
  U k;
  if constexpr (sizeof(U) == 8) k = (U)st.bcast64((uint64_t)k_own, t);
  else k = (U)st.bcast((uint32_t)k_own, t);
  const uint8_t r = ice_level2<U, S0, S1, B0, B1, G>(T, st, k, insert);
  return insert ? r : (r == R_FOUND ? 1 : 0);
}

// Batch kernel (Alg. 3): lane i owns key i (coalesced load) and its result
// byte; each sub-tile serves the keys of its G lanes one after another.
// MODE_MIXED reads a per-key opcode (0 = find, 1 = find-or-put).
template <class KeyT, int S0, int S1, int B0, int B1, int G, int MODE>
__global__ __launch_bounds__(256) void iceberg_kernel(TableK T, BatchK Bt) {
  using U = KeyT;
  const SubTile<G> st;
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = idx < Bt.n;
  const U k = act ? static_cast<const U*>(Bt.keys)[idx] : (U)0;
  uint32_t op = (uint32_t)MODE;
  if constexpr (MODE == MODE_MIXED) op = act ? (uint32_t)Bt.ops[idx] : 0u;
  const Split<U, S0> s0 = split_key<U, S0>(T, T.lv[0], 0, k, 0u);
  uint8_t result = 0;
#pragma unroll 1
  for (int t = 0; t < G; ++t) {
    if (!st.bcast_bool(act, t)) break;  // inactive lanes form the tail of the batch
    const uint32_t a0 = st.bcast((uint32_t)s0.a, t);
    uint64_t e0;
    if constexpr (S0 == 64) e0 = st.bcast64(s0.e, t);
    else e0 = st.bcast((uint32_t)s0.e, t);
    bool ins = MODE == MODE_INSERT;
    if constexpr (MODE == MODE_MIXED) ins = st.bcast(op, t) != 0u;
    const uint8_t r = ice_op<U, S0, S1, B0, B1, G>(T, st, k, t, a0, e0, ins);
    if (st.rk == t) result = r;
  }
  if (act) Bt.out[idx] = result;
}

}  // namespace cpht
