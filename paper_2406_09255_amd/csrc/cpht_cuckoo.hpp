// Compact bucketed cuckoo table: parallel put (Sec. 4.4, Alg. 4) and lookup
// (Sec. 4.4 "Lookup"), both with the sub-tile work sharing of Sec. 4.2.
//
// One sub-tile of G lanes reads a bucket of B = G*W*32/S slots, W words per
// lane.  Each slot holds (r_j(k), j): occupancy bit, hash index j, and the
// remainder of pi_j(k) (or all of pi_j(k) for the non-compact table).
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

// Atomic swap of lane-local slot i with value e; returns the evicted value.
template <int S, int W>
__device__ __forceinline__ uint64_t swap_slot(uint32_t* lane_ptr, int i, uint64_t e) {
  if constexpr (S == 32) return xchg32(lane_ptr + i, (uint32_t)e);
  else return xchg64(reinterpret_cast<uint64_t*>(lane_ptr + 2 * i), e);
}

// Alg. 4 for the key k (same in every lane of the sub-tile), starting with
// hash index 0 at bucket a with stored form e.  Each of the C rounds
// snapshots the bucket of the carried key; if it has an empty slot the first
// one is claimed with CAS (a lost claim uses up the round, as in Alg. 4, and
// marks the slot known-occupied); otherwise a victim row is swapped
// with the carried pair, and the evicted pair (r', j') continues as key
// pi_{j'}^{-1}(a . r') with hash index j'+1 mod H.  After C rounds the carried
// key is dropped and the result is FULL.
template <class U, int S, int B, int G>
__device__ __forceinline__ uint8_t ck_put(const TableK& T, const SubTile<G>& st, U k, uint32_t a, uint64_t e) {
  using Sh = CkShape<S, B, G>;
  constexpr int W = Sh::W, PER = Sh::PER;
  const LevelK& L = T.lv[0];
  const uint64_t tmask = (1ull << L.tbits) - 1ull;
  uint64_t ab = a;
  uint32_t* p = L.base + ab * L.bucket_words + (uint32_t)(st.rk * W);
  uint32_t w[W];
  uint32_t known = 0;
  load_words<W>(w, p);
#pragma unroll 1
  for (uint32_t c = 1; c <= T.C; ++c) {
    const int le = lane_first_empty<S, W>(w, known);
    const uint32_t em = st.ballot(le < PER);
    if (em) {
      const int f = ctz32(em);
      int claim = CLAIM_LOST;
      if (st.rk == f) claim = claim_slot<S, W>(p, w, known, le, e);
      if (st.bcast((uint32_t)claim, f) == (uint32_t)CLAIM_WON) return R_PUT;
      uint32_t fr[W];
      load_words<W>(fr, p);
      merge_words<W>(w, fr);
      continue;
    }
    const uint32_t v = victim_row((uint64_t)k, c, (uint32_t)B);
    const int vl = (int)(v / PER), vi = (int)(v % PER);
    uint64_t old = 0;
    if (st.rk == vl) old = swap_slot<S, W>(p, vi, e);
    if constexpr (S == 64) old = st.bcast64(old, vl);
    else old = st.bcast((uint32_t)old, vl);
    const uint32_t jj = (uint32_t)((old >> L.pbits) & tmask);
    k = join_key<U>(T, L, (int)jj, ab, old);
    const uint32_t j = jj + 1 == T.H ? 0u : jj + 1;
    const Split<U, S> sp = split_key<U, S>(T, L, (int)j, k, j);
    ab = sp.a;
    e = sp.e;
    p = L.base + ab * L.bucket_words + (uint32_t)(st.rk * W);
    known = 0;
    load_words<W>(w, p);
  }
  return R_FULL;
}

// Lookup: buckets a_0(k), a_1(k), ... in order; a hit answers 1, a bucket
// that is not full and lacks (r_j(k), j) answers 0.
template <class U, int S, int B, int G>
__device__ __forceinline__ uint8_t ck_find(const TableK& T, const SubTile<G>& st, U k, uint32_t a, uint64_t e) {
  using Sh = CkShape<S, B, G>;
  constexpr int W = Sh::W, PER = Sh::PER;
  const LevelK& L = T.lv[0];
  uint64_t ab = a;
#pragma unroll 1
  for (uint32_t j = 0;;) {
    const uint32_t* p = L.base + ab * L.bucket_words + (uint32_t)(st.rk * W);
    uint32_t w[W];
    load_words<W>(w, p);
    if (st.ballot(lane_has<S, W>(w, e))) return 1;
    if (st.ballot(lane_first_empty<S, W>(w, 0u) < PER)) return 0;
    if (++j == T.H) return 0;
    const Split<U, S> sp = split_key<U, S>(T, L, (int)j, k, j);
    ab = sp.a;
    e = sp.e;
  }
}

template <class KeyT, int S, int B, int G, bool PUT>
__global__ __launch_bounds__(256) void cuckoo_kernel(TableK T, BatchK Bt) {
  using U = KeyT;
  const SubTile<G> st;
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = idx < Bt.n;
  const U k = act ? static_cast<const U*>(Bt.keys)[idx] : (U)0;
  const Split<U, S> s0 = split_key<U, S>(T, T.lv[0], 0, k, 0u);
  uint8_t result = 0;
#pragma unroll 1
  for (int t = 0; t < G; ++t) {
    if (!st.bcast_bool(act, t)) break;
    U kt;
    if constexpr (sizeof(U) == 8) kt = (U)st.bcast64((uint64_t)k, t);
    else kt = (U)st.bcast((uint32_t)k, t);
    const uint32_t a0 = st.bcast((uint32_t)s0.a, t);
    uint64_t e0;
    if constexpr (S == 64) e0 = st.bcast64(s0.e, t);
    else e0 = st.bcast((uint32_t)s0.e, t);
    uint8_t r;
    if constexpr (PUT) r = ck_put<U, S, B, G>(T, st, kt, a0, e0);
    else r = ck_find<U, S, B, G>(T, st, kt, a0, e0);
    if (st.rk == t) result = r;
  }
  if (act) Bt.out[idx] = result;
}

}  // namespace cpht
