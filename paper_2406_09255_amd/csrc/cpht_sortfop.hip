// Find-or-put for the static cuckoo table by sorting the batch: the baseline
// the paper measures its iceberg find-or-put against (Sec. 5, find-or-put
// benchmark).  A cuckoo put must not see a key twice or a key already stored,
// so the batch is first reduced to its distinct keys:
//
//   1. sort (key, input position) pairs by key: stable LSD radix sort over
//      the w key bits, 8-bit digits, one histogram / offset scan / scatter
//      round per digit;
//   2. a sorted key that differs from its left neighbour starts a run of
//      equal keys; an exclusive scan of these run heads numbers the distinct
//      keys and packs them into an array U (the head is the run's first input
//      position, since the sort is stable);
//   3. one lookup per distinct key (the cuckoo find kernel over U);
//   4. the distinct keys the lookup missed are packed again and inserted with
//      the cuckoo put kernel;
//   5. every input position gets its answer: FOUND for keys already stored,
//      and for a missing key the put's PUT or FULL at its first occurrence and
//      FOUND (or FULL) at the later ones.  The answers are produced in sorted
//      order; rather than scattering single bytes over the whole output, they
//      are packed with their positions, partitioned by the positions' high
//      bits (one more radix round) and written one output window at a time.
//
// Counts that only the device knows (distinct keys, missing keys) stay on the
// device: the lookup and put run as persistent launches over chunk lists that
// a small kernel builds from those counts, so the call makes no host round
// trip.
#include "cpht_sortfop.hpp"

#include <algorithm>
#include <mutex>

// Device scratch of the allocation-free variant of the pipeline: one copy of
// this array per GPU, loaded with the library's code and kept until the
// process ends.  Host code never passes the array's name to a kernel (on the
// host it is only a stand-in for the symbol); it uses the per-device address
// that sorted_fop_scratch() obtains from the runtime.
static __device__ __align__(256) uint8_t scratch[cpht::NOALLOC_SCRATCH_BYTES];

namespace cpht {
namespace {

constexpr int TPB = 256;            // threads per block (four waves)
constexpr int IPT = 16;             // items per thread
constexpr int TILE = TPB * IPT;     // items per tile
constexpr int RADIX = 256;          // 8-bit digits
constexpr int WAVES = TPB / 64;
constexpr int SEG = TILE / WAVES;   // items per wave within a tile

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63u; }

// Blocks are handed to the 8 XCDs in turn (block b runs on XCD b mod 8).
// Consecutive sort tiles write adjacent runs of every digit, so they are given
// to blocks of the same XCD, where the partial cache lines at the run ends
// merge in that XCD's L2 instead of going to memory separately.  The grid has
// XCDS * ceil(ntiles / XCDS) blocks; the surplus ones exit.
constexpr uint32_t XCDS = 8;

__host__ __device__ inline uint32_t tile_grid(uint64_t ntiles) {
  return (uint32_t)(((ntiles + XCDS - 1) / XCDS) * XCDS);
}

__device__ __forceinline__ uint64_t tile_of_block(uint64_t ntiles) {
  const uint64_t per = (ntiles + XCDS - 1) / XCDS;
  return (uint64_t)(blockIdx.x % XCDS) * per + blockIdx.x / XCDS;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(v, (unsigned)o, 64);
    if (lane >= (uint32_t)o) v += t;
  }
  return v;
}

// Exclusive scan of one value per thread over the block; *total gets the sum.
// `tmp` holds WAVES + 1 words of shared memory.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* tmp, uint32_t* total) {
  const uint32_t lane = lane_id(), wv = threadIdx.x >> 6;
  const uint32_t inc = wave_incl_scan(v);
  if (lane == 63) tmp[wv] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int w = 0; w < WAVES; ++w) {
      const uint32_t t = tmp[w];
      tmp[w] = run;
      run += t;
    }
    tmp[WAVES] = run;
  }
  __syncthreads();
  const uint32_t r = tmp[wv] + inc - v;
  *total = tmp[WAVES];
  __syncthreads();  // tmp may be reused by the caller
  return r;
}

// Lanes (of `valid`) whose digit equals this lane's digit.
__device__ __forceinline__ uint64_t same_digit(uint32_t d, uint64_t valid) {
  uint64_t m = valid;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const uint32_t bit = (d >> b) & 1u;
    const uint64_t bl = __ballot(bit);
    m &= bit ? bl : ~bl;
  }
  return m;
}

// ---------------------------------------------------------------------------
// Radix sort rounds
// ---------------------------------------------------------------------------

// counts[d * ntiles + tile] = number of keys of the tile whose digit is d.
template <class K>
__global__ __launch_bounds__(TPB) void sort_hist(const K* __restrict__ keys, uint64_t n, uint32_t shift,
                                                 uint32_t* __restrict__ counts, uint32_t ntiles) {
  __shared__ uint32_t h[WAVES][RADIX];
  const uint64_t tile = tile_of_block(ntiles);
  if (tile >= ntiles) return;
  const uint32_t wv = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < WAVES * RADIX; i += TPB) (&h[0][0])[i] = 0u;
  __syncthreads();
  const uint64_t base = tile * TILE;
#pragma unroll 4
  for (int r = 0; r < IPT; ++r) {
    const uint64_t i = base + (uint64_t)r * TPB + threadIdx.x;
    if (i < n) atomicAdd(&h[wv][(uint32_t)(keys[i] >> shift) & (RADIX - 1u)], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < RADIX; d += TPB) {
    uint32_t c = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) c += h[w][d];
    counts[(uint64_t)d * ntiles + tile] = c;
  }
}

// Stable scatter of one tile by digit.  offs[d * ntiles + tile] is where the
// tile's keys with digit d start in the output (exclusive scan of the counts
// in digit-major order).  Within the tile, wave w ranks items
// [w * SEG, (w + 1) * SEG) in order, 64 at a time: lanes with equal digits
// rank by lane, and a per-wave counter per digit carries the rank across
// rounds.  The tile is then laid out by digit in shared memory and written
// out in order, so consecutive threads write consecutive output words: keys
// first, then the positions through the same buffer (one buffer of keys and
// a byte of digit per slot keep shared memory at 42 KB, three blocks per CU).
template <class K>
__global__ __launch_bounds__(TPB, 3) void sort_scatter(const K* __restrict__ kin, const uint32_t* __restrict__ iin,
                                                    K* __restrict__ kout, uint32_t* __restrict__ iout, uint64_t n,
                                                    uint32_t shift, const uint32_t* __restrict__ offs,
                                                    uint32_t ntiles) {
  __shared__ uint32_t wc[WAVES][RADIX];
  __shared__ uint32_t dstart[RADIX];
  __shared__ uint32_t obase[RADIX];  // output index of staged slot p with digit d: obase[d] + p
  __shared__ uint32_t tmp[WAVES + 1];
  __shared__ K stage[TILE];        // keys by digit, then (as uint32) their input positions
  __shared__ uint8_t sdig[TILE];   // digit of each staged slot
  const uint64_t tile = tile_of_block(ntiles);
  if (tile >= ntiles) return;
  const uint32_t lane = lane_id(), wv = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < WAVES * RADIX; i += TPB) (&wc[0][0])[i] = 0u;
  __syncthreads();

  const uint64_t tbase = tile * TILE;
  const uint64_t seg = tbase + (uint64_t)wv * SEG;
  const uint64_t below = (1ull << lane) - 1ull;
  K key[IPT];
  uint32_t src[IPT];  // input position carried with each key (absent in keys-only rounds)
  uint32_t pos[IPT];  // rank among the wave's keys of the same digit, then slot in the tile
  // all of the tile's loads first, so they are in flight together (the
  // ranking below is serialised by its shared-memory counters)
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const uint64_t i = seg + (uint64_t)r * 64 + lane;
    key[r] = i < n ? kin[i] : (K)0;
    src[r] = iin && i < n ? iin[i] : (uint32_t)i;
  }
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const uint64_t i = seg + (uint64_t)r * 64 + lane;
    const bool valid = i < n;
    const K k = key[r];
    const uint32_t d = (uint32_t)(k >> shift) & (RADIX - 1u);
    const uint64_t vm = __ballot(valid);
    const uint64_t peers = same_digit(d, vm);
    // The wave reads the counter of its digit, then the group's lowest lane
    // advances it; shared-memory accesses of one wave complete in issue
    // order, and the volatile accesses keep that order in the code.
    volatile uint32_t* ctr = &wc[wv][d];
    const uint32_t b = valid ? *ctr : 0u;
    if (valid && (peers & below) == 0ull) *ctr = b + (uint32_t)__popcll(peers);
    pos[r] = b + (uint32_t)__popcll(peers & below);
  }
  __syncthreads();

  // per digit: exclusive prefix over the waves, and the tile's total
  static_assert(TPB == RADIX, "one thread per digit");
  uint32_t tot = 0;
  {
    const uint32_t d = threadIdx.x;  // TPB == RADIX
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
      const uint32_t c = wc[w][d];
      wc[w][d] = run;
      run += c;
    }
    tot = run;
  }
  uint32_t all;
  const uint32_t ds = block_excl_scan(tot, tmp, &all);
  dstart[threadIdx.x] = ds;
  // the tile's run of digit d starts at offs[d][tile] >= ds (it follows every
  // key of a smaller digit), so the difference fits the index type
  obase[threadIdx.x] = offs[(uint64_t)threadIdx.x * ntiles + tile] - ds;
  __syncthreads();

  const uint32_t tile_n = (uint32_t)(n - tbase < (uint64_t)TILE ? n - tbase : (uint64_t)TILE);
  // keys
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const uint64_t i = seg + (uint64_t)r * 64 + lane;
    if (i < n) {
      const uint32_t d = (uint32_t)(key[r] >> shift) & (RADIX - 1u);
      pos[r] += dstart[d] + wc[wv][d];
      stage[pos[r]] = key[r];
      sdig[pos[r]] = (uint8_t)d;
    }
  }
  __syncthreads();
  for (uint32_t p = threadIdx.x; p < tile_n; p += TPB) kout[(uint64_t)obase[sdig[p]] + p] = stage[p];
  if (iout == nullptr) return;  // keys only (uniform across the block)
  __syncthreads();
  // input positions, through the same buffer
  uint32_t* sidx = reinterpret_cast<uint32_t*>(stage);
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const uint64_t i = seg + (uint64_t)r * 64 + lane;
    if (i < n) sidx[pos[r]] = src[r];
  }
  __syncthreads();
  for (uint32_t p = threadIdx.x; p < tile_n; p += TPB) iout[(uint64_t)obase[sdig[p]] + p] = sidx[p];
}

// ---------------------------------------------------------------------------
// Tile scans: exclusive scan of per-item values with a caller-defined emit.
// A policy P provides count() (items; may read device memory), value(i) and
// emit(i, exclusive prefix, value).
// ---------------------------------------------------------------------------

// Items are striped over the block (item base + r * TPB + thread, so every
// load and store of a wave is contiguous); the exclusive prefix in item order
// combines a wave scan per round with one serial pass over the per-round,
// per-wave totals.
template <class P>
__global__ __launch_bounds__(TPB) void tile_reduce(P p, uint32_t* __restrict__ psum) {
  __shared__ uint32_t tmp[WAVES + 1];
  const uint64_t n = p.count();
  const uint64_t base = (uint64_t)blockIdx.x * TILE + threadIdx.x;
  uint32_t s = 0;
#pragma unroll 4
  for (int r = 0; r < IPT; ++r) {
    const uint64_t i = base + (uint64_t)r * TPB;
    if (i < n) s += p.value(i);
  }
  uint32_t total;
  block_excl_scan(s, tmp, &total);
  if (threadIdx.x == 0) psum[blockIdx.x] = total;
}

// One block: exclusive scan of psum[0 .. np) in place; *grand = the sum.
__global__ __launch_bounds__(TPB) void scan_top(uint32_t* __restrict__ psum, uint64_t np,
                                                uint64_t* __restrict__ grand) {
  __shared__ uint32_t tmp[WAVES + 1];
  uint64_t carry = 0;
  for (uint64_t base = 0; base < np; base += TILE) {
    const uint64_t b = base + (uint64_t)threadIdx.x * IPT;
    uint32_t v[IPT];
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      v[r] = b + r < np ? psum[b + r] : 0u;
      s += v[r];
    }
    uint32_t total;
    uint32_t e = block_excl_scan(s, tmp, &total);
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
      if (b + r < np) psum[b + r] = (uint32_t)carry + e;
      e += v[r];
    }
    carry += total;
  }
  if (threadIdx.x == 0 && grand) *grand = carry;
}

template <class P>
__global__ __launch_bounds__(TPB) void tile_apply(P p, const uint32_t* __restrict__ pexcl) {
  __shared__ uint32_t tot[IPT][WAVES];
  const uint32_t lane = lane_id(), wv = threadIdx.x >> 6;
  const uint64_t n = p.count();
  const uint64_t base = (uint64_t)blockIdx.x * TILE + threadIdx.x;
  uint32_t v[IPT], inc[IPT];
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const uint64_t i = base + (uint64_t)r * TPB;
    v[r] = i < n ? p.value(i) : 0u;
    inc[r] = wave_incl_scan(v[r]);
    if (lane == 63) tot[r][wv] = inc[r];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = pexcl[blockIdx.x];
    for (int r = 0; r < IPT; ++r)
      for (int w = 0; w < WAVES; ++w) {
        const uint32_t t = tot[r][w];
        tot[r][w] = run;
        run += t;
      }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < IPT; ++r) {
    const uint64_t i = base + (uint64_t)r * TPB;
    if (i < n) p.emit(i, tot[r][wv] + inc[r] - v[r], v[r]);
  }
}

// Radix offsets: counts scanned in place.
struct CountsScan {
  uint32_t* c;
  uint64_t n;
  __device__ uint64_t count() const { return n; }
  __device__ uint32_t value(uint64_t i) const { return c[i]; }
  __device__ void emit(uint64_t i, uint32_t e, uint32_t) const { c[i] = e; }
};

// Run heads of the sorted keys: U[e] = key of the e-th distinct key,
// uniq[i] = number of the distinct key at sorted position i.
template <class K>
struct Heads {
  const K* key;
  K* U;
  uint32_t* uniq;
  uint64_t n;
  __device__ uint64_t count() const { return n; }
  __device__ uint32_t value(uint64_t i) const { return i == 0 || key[i] != key[i - 1] ? 1u : 0u; }
  __device__ void emit(uint64_t i, uint32_t e, uint32_t v) const {
    uniq[i] = e + v - 1u;
    if (v) U[e] = key[i];
  }
};

// Distinct keys the lookup missed: P[e] = U[u], pidx[e] = u; answers of
// the found ones are final (FOUND), the others wait for the put.
template <class K>
struct Missing {
  const K* U;
  const uint8_t* found;
  const uint64_t* m;
  K* P;
  uint32_t* pidx;
  uint8_t* uo;
  __device__ uint64_t count() const { return *m; }
  __device__ uint32_t value(uint64_t u) const { return found[u] ? 0u : 1u; }
  __device__ void emit(uint64_t u, uint32_t e, uint32_t v) const {
    uo[u] = v ? R_NONE : R_FOUND;
    if (v) {
      P[e] = U[u];
      pidx[e] = (uint32_t)u;
    }
  }
};

// Chunk list for a persistent launch over `*count` keys of table 0.
__global__ __launch_bounds__(TPB) void make_chunks(const uint64_t* __restrict__ count, ChunkK* __restrict__ chunks,
                                                   uint64_t max_chunks, uint64_t* __restrict__ group) {
  const uint64_t m = *count;
  uint64_t nch = (m + 255) / 256;
  if (nch > max_chunks) nch = max_chunks;  // cannot happen: m <= n
  for (uint64_t c = (uint64_t)blockIdx.x * TPB + threadIdx.x; c < nch; c += (uint64_t)gridDim.x * TPB) {
    ChunkK ch;
    ch.start = c * 256;
    ch.table = 0;
    ch.count = (uint32_t)(m - c * 256 < 256 ? m - c * 256 : 256);
    chunks[c] = ch;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    group[0] = 0;
    group[1] = nch;
  }
}

__global__ void store_desc(TableK T, TableK* dst) {
  if (threadIdx.x == 0) *dst = T;
}

__global__ __launch_bounds__(TPB) void put_answers(const uint32_t* __restrict__ pidx,
                                                   const uint8_t* __restrict__ pout, const uint64_t* __restrict__ p,
                                                   uint8_t* __restrict__ uo) {
  const uint64_t np = *p;
  for (uint64_t j = (uint64_t)blockIdx.x * TPB + threadIdx.x; j < np; j += (uint64_t)gridDim.x * TPB)
    uo[pidx[j]] = pout[j];
}

// out[input position] for every sorted position: the distinct key's answer
// at its first occurrence, FOUND after a PUT at the later ones.
__global__ __launch_bounds__(TPB) void final_answers(const uint32_t* __restrict__ uniq,
                                                     const uint32_t* __restrict__ pos,
                                                     const uint8_t* __restrict__ uo, uint64_t n,
                                                     uint8_t* __restrict__ out) {
  for (uint64_t i = (uint64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (uint64_t)gridDim.x * TPB) {
    const uint32_t u = uniq[i];
    const uint8_t o = uo[u];
    const bool head = i == 0 || uniq[i - 1] != u;
    // one byte to a random place; a plain store, so the cache merges the
    // bytes that land in one line (a streaming store measured 1.8x slower)
    out[pos[i]] = head ? o : (o == R_PUT ? (uint8_t)R_FOUND : o);
  }
}

// The same answers as final_answers, packed with their input position for a
// partition by position: packed[i] = pos[i] << 2 | answer (n <= 2^30).
__global__ __launch_bounds__(TPB) void pack_answers(const uint32_t* __restrict__ uniq,
                                                    const uint32_t* __restrict__ pos,
                                                    const uint8_t* __restrict__ uo, uint64_t n,
                                                    uint32_t* __restrict__ packed) {
  for (uint64_t i = (uint64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (uint64_t)gridDim.x * TPB) {
    const uint32_t u = uniq[i];
    const uint8_t o = uo[u];
    const bool head = i == 0 || uniq[i - 1] != u;
    const uint32_t a = head ? o : (o == R_PUT ? (uint32_t)R_FOUND : o);
    packed[i] = (pos[i] << 2) | a;
  }
}

// Answers partitioned by the high bits of their position: tile t of the
// partition writes bytes that all fall in a few windows of the output, and
// consecutive tiles go to the same XCD, so each window's lines fill up in one
// L2 before they are written back.
__global__ __launch_bounds__(TPB) void write_answers(const uint32_t* __restrict__ parts, uint64_t n,
                                                     uint32_t ntiles, uint8_t* __restrict__ out) {
  const uint64_t tile = tile_of_block(ntiles);
  if (tile >= ntiles) return;
  const uint64_t base = tile * TILE + threadIdx.x;
#pragma unroll 4
  for (int r = 0; r < IPT; ++r) {
    const uint64_t j = base + (uint64_t)r * TPB;
    if (j < n) {
      const uint32_t w = parts[j];
      out[w >> 2] = (uint8_t)(w & 3u);
    }
  }
}

// ---------------------------------------------------------------------------
// Workspace layout
// ---------------------------------------------------------------------------

struct Layout {
  uint64_t kA, kB, iA, iB, counts, psum, found, uo, pout, P, pidx, chunks, misc, desc, total;
};

inline uint64_t up256(uint64_t x) { return (x + 255) & ~255ull; }

Layout layout(uint64_t n, int kb) {
  const uint64_t ntiles = (n + TILE - 1) / TILE;
  const uint64_t ncounts = (uint64_t)RADIX * ntiles;
  const uint64_t npsum = (std::max<uint64_t>(ncounts, n) + TILE - 1) / TILE;
  const uint64_t nchunks = (n + 255) / 256;
  Layout L;
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t at = o;
    o += up256(bytes);
    return at;
  };
  L.kA = take(n * kb);
  L.kB = take(n * kb);
  L.iA = take(n * 4);
  L.iB = take(n * 4);
  L.counts = take(ncounts * 4);
  L.psum = take(npsum * 4);
  L.found = take(n);
  L.uo = take(n);
  L.pout = take(n);
  L.P = take(n * kb);
  L.pidx = take(n * 4);
  L.chunks = take(nchunks * sizeof(ChunkK));
  L.misc = take(8 * sizeof(uint64_t));  // [0] distinct, [1] missing, [2..3] group, [4..5] group
  L.desc = take(sizeof(TableK));
  L.total = o;
  return L;
}

template <class P>
void run_scan(const P& p, uint64_t n_upper, uint32_t* psum, uint64_t* grand, hipStream_t s) {
  const uint64_t nt = (n_upper + TILE - 1) / TILE;
  if (nt == 0) return;
  hipLaunchKernelGGL(tile_reduce<P>, dim3((uint32_t)nt), dim3(TPB), 0, s, p, psum);
  hipLaunchKernelGGL(scan_top, dim3(1), dim3(TPB), 0, s, psum, nt, grand);
  hipLaunchKernelGGL(tile_apply<P>, dim3((uint32_t)nt), dim3(TPB), 0, s, p, (const uint32_t*)psum);
}

template <class K>
hipError_t run(const TableK& T, const CkVariant* v, int key_bits, const K* keys, uint64_t n, uint8_t* out,
               uint8_t* ws, uint32_t blocks, hipStream_t s) {
  const Layout L = layout(n, (int)sizeof(K));
  const uint64_t ntiles = (n + TILE - 1) / TILE;
  const uint64_t nchunks = (n + 255) / 256;
  K* ka = reinterpret_cast<K*>(ws + L.kA);
  K* kb = reinterpret_cast<K*>(ws + L.kB);
  uint32_t* ia = reinterpret_cast<uint32_t*>(ws + L.iA);
  uint32_t* ib = reinterpret_cast<uint32_t*>(ws + L.iB);
  uint32_t* counts = reinterpret_cast<uint32_t*>(ws + L.counts);
  uint32_t* psum = reinterpret_cast<uint32_t*>(ws + L.psum);
  uint8_t* found = ws + L.found;
  uint8_t* uo = ws + L.uo;
  uint8_t* pout = ws + L.pout;
  K* P = reinterpret_cast<K*>(ws + L.P);
  uint32_t* pidx = reinterpret_cast<uint32_t*>(ws + L.pidx);
  ChunkK* chunks = reinterpret_cast<ChunkK*>(ws + L.chunks);
  uint64_t* misc = reinterpret_cast<uint64_t*>(ws + L.misc);
  TableK* desc = reinterpret_cast<TableK*>(ws + L.desc);

  // 1. sort (key, position) by the key's w bits
  const int passes = (key_bits + 7) / 8;
  const K* kin = keys;
  const uint32_t* iin = nullptr;
  K* kout = ka;
  uint32_t* iout = ia;
  for (int pass = 0; pass < passes; ++pass) {
    const uint32_t shift = 8u * (uint32_t)pass;
    hipLaunchKernelGGL(sort_hist<K>, dim3(tile_grid(ntiles)), dim3(TPB), 0, s, kin, n, shift, counts,
                       (uint32_t)ntiles);
    run_scan(CountsScan{counts, (uint64_t)RADIX * ntiles}, (uint64_t)RADIX * ntiles, psum, nullptr, s);
    hipLaunchKernelGGL(sort_scatter<K>, dim3(tile_grid(ntiles)), dim3(TPB), 0, s, kin, iin, kout, iout, n, shift,
                       (const uint32_t*)counts, (uint32_t)ntiles);
    kin = kout;
    iin = iout;
    kout = kout == ka ? kb : ka;
    iout = iout == ia ? ib : ia;
  }
  const K* sorted = kin;        // the last pass's output
  const uint32_t* pos = iin;
  K* U = kout;                  // the other buffers are free again
  uint32_t* uniq = iout;

  // 2. distinct keys
  run_scan(Heads<K>{sorted, U, uniq, n}, n, psum, misc + 0, s);

  // 3. one lookup per distinct key
  const uint32_t cgrid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((nchunks + TPB - 1) / TPB, 4096));
  hipLaunchKernelGGL(store_desc, dim3(1), dim3(64), 0, s, T, desc);
  hipLaunchKernelGGL(make_chunks, dim3(cgrid), dim3(TPB), 0, s, (const uint64_t*)(misc + 0), chunks, nchunks,
                     misc + 2);
  MultiK M;
  M.descs = desc;
  M.chunks = chunks;
  M.group = misc + 2;
  M.keys = U;
  M.out = found;
  v->multi_find(M, blocks, s);

  // 4. put the distinct keys that were missing
  run_scan(Missing<K>{U, found, misc + 0, P, pidx, uo}, n, psum, misc + 1, s);
  hipLaunchKernelGGL(make_chunks, dim3(cgrid), dim3(TPB), 0, s, (const uint64_t*)(misc + 1), chunks, nchunks,
                     misc + 4);
  M.group = misc + 4;
  M.keys = P;
  M.out = pout;
  v->multi_put(M, blocks, s);

  // 5. answers
  const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((n + TPB - 1) / TPB, 65536));
  hipLaunchKernelGGL(put_answers, dim3(grid), dim3(TPB), 0, s, (const uint32_t*)pidx, (const uint8_t*)pout,
                     (const uint64_t*)(misc + 1), uo);
  if (n > (1ull << 30)) {  // positions too wide to pack with a 2-bit answer: scatter directly
    hipLaunchKernelGGL(final_answers, dim3(grid), dim3(TPB), 0, s, (const uint32_t*)uniq, pos,
                       (const uint8_t*)uo, n, out);
    return hipGetLastError();
  }
  // pack (position, answer), partition by the top 8 bits of the packed word
  // (one stable radix round), then write each partition's bytes together
  uint32_t* packed = reinterpret_cast<uint32_t*>(const_cast<K*>(sorted));  // free since step 2
  uint32_t* parts = reinterpret_cast<uint32_t*>(U);                        // free since step 4
  hipLaunchKernelGGL(pack_answers, dim3(grid), dim3(TPB), 0, s, (const uint32_t*)uniq, pos, (const uint8_t*)uo, n,
                     packed);
  uint32_t pb = 2;  // bits of the packed word: positions < n, shifted by 2
  while ((1ull << pb) < 4 * n) ++pb;
  const uint32_t pshift = pb > 8 ? pb - 8 : 0;
  hipLaunchKernelGGL(sort_hist<uint32_t>, dim3(tile_grid(ntiles)), dim3(TPB), 0, s, (const uint32_t*)packed, n,
                     pshift, counts, (uint32_t)ntiles);
  run_scan(CountsScan{counts, (uint64_t)RADIX * ntiles}, (uint64_t)RADIX * ntiles, psum, nullptr, s);
  hipLaunchKernelGGL(sort_scatter<uint32_t>, dim3(tile_grid(ntiles)), dim3(TPB), 0, s, (const uint32_t*)packed,
                     (const uint32_t*)nullptr, parts, (uint32_t*)nullptr, n, pshift, (const uint32_t*)counts,
                     (uint32_t)ntiles);
  hipLaunchKernelGGL(write_answers, dim3(tile_grid(ntiles)), dim3(TPB), 0, s, (const uint32_t*)parts, n,
                     (uint32_t)ntiles, out);
  return hipGetLastError();
}

}  // namespace

uint64_t sorted_fop_workspace(uint64_t n, int key_bytes) { return layout(n, key_bytes).total; }

hipError_t sorted_fop_scratch(int device, void** ptr) {
  constexpr int MAX_DEVICES = 64;
  static std::mutex mu;
  static void* addr[MAX_DEVICES] = {};
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[device] = p;
  }
  *ptr = addr[device];
  return hipSuccess;
}

hipError_t launch_sorted_fop(const TableK& T, const CkVariant* v, int key_bits, const void* keys, uint64_t n,
                             uint8_t* out, void* workspace, uint32_t blocks, hipStream_t s) {
  if (n == 0) return hipSuccess;
  uint8_t* ws = static_cast<uint8_t*>(workspace);
  if (key_bits <= 32) return run<uint32_t>(T, v, key_bits, static_cast<const uint32_t*>(keys), n, out, ws, blocks, s);
  return run<uint64_t>(T, v, key_bits, static_cast<const uint64_t*>(keys), n, out, ws, blocks, s);
}

}  // namespace cpht
