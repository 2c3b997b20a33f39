// Measurement kernels for the random-access roofline of the hash tables:
// the rate at which the device serves random 128-byte line reads, random
// 32-bit and 64-bit CAS, and a line read followed by a CAS into that line
// (the access pattern of a put).  They use the same sub-tile shape as the
// table kernels (8 lanes x 16 bytes per line) and keep 8 independent
// accesses in flight per group, like the pipelined batch kernels.  A last
// kernel costs the quotienting split alone: three permutations of every key
// of a buffer, with nothing written but a sink word.
#include "cpht_device.hpp"
#include "cpht_roofline.hpp"

namespace cpht {

namespace {

__device__ __forceinline__ uint64_t line_of(uint64_t group, uint64_t i, uint64_t seed, uint64_t mask) {
  return mix64(seed ^ (group * 0x9E3779B97F4A7C15ull + i)) & mask;
}

constexpr int INFLIGHT = 8;

// Each group of 8 lanes reads `per` random lines of the buffer.
__global__ __launch_bounds__(256) void probe_lines_kernel(const uint4* buf, uint64_t line_mask, uint32_t per,
                                                          uint64_t seed, uint32_t* sink) {
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t group = gid >> 3;
  const uint32_t r = (uint32_t)(gid & 7u);
  uint32_t acc = 0;
#pragma unroll 1
  for (uint32_t i = 0; i < per; i += INFLIGHT) {
    uint4 v[INFLIGHT];
#pragma unroll
    for (int d = 0; d < INFLIGHT; ++d) v[d] = buf[line_of(group, i + d, seed, line_mask) * 8 + r];
#pragma unroll
    for (int d = 0; d < INFLIGHT; ++d) acc ^= v[d].x ^ v[d].y ^ v[d].z ^ v[d].w;
  }
  if (acc == 0x9E3779B9u) sink[0] = acc;  // keeps the loads live; practically never stores
}

// Each group of LANES lanes reads `per` random units of LANES x 16 bytes
// (4 lanes: 64-byte half lines, 8 lanes: whole lines), with plain or with
// non-temporal loads.
template <int LANES, bool NT>
__global__ __launch_bounds__(256) void probe_units_kernel(const uint4* buf, uint64_t unit_mask, uint32_t per,
                                                          uint64_t seed, uint32_t* sink) {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t group = gid / LANES;
  const uint32_t r = (uint32_t)(gid % LANES);
  uint32_t acc = 0;
#pragma unroll 1
  for (uint32_t i = 0; i < per; i += INFLIGHT) {
    u32x4 v[INFLIGHT];
#pragma unroll
    for (int d = 0; d < INFLIGHT; ++d) {
      const u32x4* p = reinterpret_cast<const u32x4*>(buf + line_of(group, i + d, seed, unit_mask) * LANES + r);
      if constexpr (NT) v[d] = __builtin_nontemporal_load(p);
      else v[d] = *p;
    }
#pragma unroll
    for (int d = 0; d < INFLIGHT; ++d) acc ^= v[d].x ^ v[d].y ^ v[d].z ^ v[d].w;
  }
  if (acc == 0x9E3779B9u) sink[0] = acc;
}

// Each lane performs `per` CAS (expected 0) on random 32-bit words.
__global__ __launch_bounds__(256) void probe_cas_kernel(uint32_t* buf, uint64_t word_mask, uint32_t per,
                                                        uint64_t seed, uint32_t* sink) {
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t acc = 0;
#pragma unroll 1
  for (uint32_t i = 0; i < per; i += INFLIGHT) {
    uint32_t got[INFLIGHT];
#pragma unroll
    for (int d = 0; d < INFLIGHT; ++d)
      got[d] = cas32(buf + line_of(gid, i + d, seed, word_mask), 0u, (uint32_t)(gid | 1u));
#pragma unroll
    for (int d = 0; d < INFLIGHT; ++d) acc += got[d];
  }
  if (acc == 0x9E3779B9u) sink[0] = acc;
}

// Each group of 8 lanes reads a random line, then one lane CASes a word of
// that line (the first-empty claim of a put).
__global__ __launch_bounds__(256) void probe_line_cas_kernel(uint4* buf, uint64_t line_mask, uint32_t per,
                                                             uint64_t seed, uint32_t* sink) {
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t group = gid >> 3;
  const uint32_t r = (uint32_t)(gid & 7u);
  uint32_t acc = 0;
#pragma unroll 1
  for (uint32_t i = 0; i < per; i += INFLIGHT) {
    uint4 v[INFLIGHT];
    uint64_t ln[INFLIGHT];
#pragma unroll
    for (int d = 0; d < INFLIGHT; ++d) {
      ln[d] = line_of(group, i + d, seed, line_mask);
      v[d] = buf[ln[d] * 8 + r];
    }
#pragma unroll
    for (int d = 0; d < INFLIGHT; ++d) {
      acc ^= v[d].x;
      if (r == (uint32_t)d) {  // one lane per line claims a word of it
        uint32_t* w = reinterpret_cast<uint32_t*>(buf + ln[d] * 8) + (v[d].y & 31u);
        acc += cas32(w, 0u, (uint32_t)(group | 1u));
      }
    }
  }
  if (acc == 0x9E3779B9u) sink[0] = acc;
}

// Each lane performs `per` 64-bit CAS (expected 0) on random 8-byte words
// (the claim of a plain table's 64-bit slot).
__global__ __launch_bounds__(256) void probe_cas64_kernel(uint64_t* buf, uint64_t word_mask, uint32_t per,
                                                          uint64_t seed, uint32_t* sink) {
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t acc = 0;
#pragma unroll 1
  for (uint32_t i = 0; i < per; i += INFLIGHT) {
    uint64_t got[INFLIGHT];
#pragma unroll
    for (int d = 0; d < INFLIGHT; ++d)
      got[d] = cas64(buf + line_of(gid, i + d, seed, word_mask), 0ull, gid | 1ull);
#pragma unroll
    for (int d = 0; d < INFLIGHT; ++d) acc += got[d];
  }
  if (acc == 0x9E3779B97F4A7C15ull) sink[0] = (uint32_t)acc;
}

// The split of Sec. 2.4 alone: lane g takes keys g, g + T, g + 2T, ... (T
// lanes in the grid, coalesced), `per` of them, wrapping round the buffer;
// every key goes through the three permutations pi_0, pi_1, pi_2 of w-bit
// keys and is cut into a bucket address (high nb bits) and an occupied stored
// form (low w - nb bits), as the table kernels do before every probe.  Only
// a fold of the results is kept.
__global__ __launch_bounds__(256) void probe_split_kernel(const uint64_t* keys, uint64_t key_mask, uint32_t per,
                                                          PermK p0, PermK p1, PermK p2, uint32_t w, uint32_t nb,
                                                          uint32_t* sink) {
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t T = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t M = (w >= 64) ? ~0ull : ((1ull << w) - 1ull);
  const uint32_t h = (w + 1) / 2;
  const uint64_t rmask = (1ull << (w - nb)) - 1ull;
  const uint64_t occ = 1ull << 31;
  uint64_t acc = 0;
#pragma unroll 1
  for (uint32_t i = 0; i < per; ++i) {
    const uint64_t k = keys[(gid + (uint64_t)i * T) & key_mask] & M;
    const uint64_t x0 = perm_fwd<uint64_t>(p0, k, h, M);
    const uint64_t x1 = perm_fwd<uint64_t>(p1, k, h, M);
    const uint64_t x2 = perm_fwd<uint64_t>(p2, k, h, M);
    acc ^= (x0 >> (w - nb)) ^ (occ | (x0 & rmask));
    acc += (x1 >> (w - nb)) ^ (occ | (x1 & rmask));
    acc ^= (x2 >> (w - nb)) + (occ | (x2 & rmask));
  }
  if (acc == 0x9E3779B97F4A7C15ull) sink[0] = (uint32_t)acc;
}

// Constants of a permutation for the split probe: odd multipliers and xor
// constants from splitmix64 of the seed (any such constants cost the same).
uint64_t host_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

PermK probe_perm(uint64_t seed, int i, uint64_t M) {
  PermK P{};
  for (int q = 0; q < 3; ++q) {
    const uint64_t z = seed + (uint64_t)(3 * i + q + 1) * 0x9E3779B97F4A7C15ull;
    P.m[q] = (host_mix(z) | 1ull) & M;
    P.c[q] = host_mix(z ^ 0xD1B54A32D192ED03ull) & M;
    P.minv[q] = 0;
  }
  return P;
}

uint32_t grid_for(uint64_t threads) { return (uint32_t)((threads + 255) / 256); }

}  // namespace

hipError_t launch_probe(int kind, void* buf, uint64_t bytes, uint64_t ops, uint64_t seed, uint32_t* sink,
                        hipStream_t s) {
  // `ops` accesses, 64 per lane (lines: per group of 8 lanes)
  const uint32_t per = 64;
  if (kind == 0) {
    const uint64_t lines = bytes / 128;
    const uint64_t threads = (ops / per) * 8;
    hipLaunchKernelGGL(probe_lines_kernel, dim3(grid_for(threads)), dim3(256), 0, s,
                       static_cast<const uint4*>(buf), lines - 1, per, seed, sink);
  } else if (kind == 1) {
    const uint64_t words = bytes / 4;
    const uint64_t threads = ops / per;
    hipLaunchKernelGGL(probe_cas_kernel, dim3(grid_for(threads)), dim3(256), 0, s, static_cast<uint32_t*>(buf),
                       words - 1, per, seed, sink);
  } else if (kind == 2) {
    const uint64_t lines = bytes / 128;
    const uint64_t threads = (ops / per) * 8;
    hipLaunchKernelGGL(probe_line_cas_kernel, dim3(grid_for(threads)), dim3(256), 0, s, static_cast<uint4*>(buf),
                       lines - 1, per, seed, sink);
  } else if (kind == 3) {
    const uint64_t words = bytes / 8;
    const uint64_t threads = ops / per;
    hipLaunchKernelGGL(probe_cas64_kernel, dim3(grid_for(threads)), dim3(256), 0, s, static_cast<uint64_t*>(buf),
                       words - 1, per, seed, sink);
  } else if (kind == 5 || kind == 6) {
    // kind 5: random 64-byte half-line reads (4 lanes); kind 6: random lines, non-temporal loads
    const uint64_t lanes = kind == 5 ? 4 : 8;
    const uint64_t units = bytes / (16 * lanes);
    const uint64_t threads = (ops / per) * lanes;
    if (kind == 5)
      hipLaunchKernelGGL((probe_units_kernel<4, false>), dim3(grid_for(threads)), dim3(256), 0, s,
                         static_cast<const uint4*>(buf), units - 1, per, seed, sink);
    else
      hipLaunchKernelGGL((probe_units_kernel<8, true>), dim3(grid_for(threads)), dim3(256), 0, s,
                         static_cast<const uint4*>(buf), units - 1, per, seed, sink);
  } else {
    // the headline table's shape: 37-bit keys, 2^22 buckets
    const uint32_t w = 37, nb = 22;
    const uint64_t M = (1ull << w) - 1ull;
    const uint64_t threads = ops / per;
    hipLaunchKernelGGL(probe_split_kernel, dim3(grid_for(threads)), dim3(256), 0, s,
                       static_cast<const uint64_t*>(buf), bytes / 8 - 1, per, probe_perm(seed, 0, M),
                       probe_perm(seed, 1, M), probe_perm(seed, 2, M), w, nb, sink);
  }
  return hipGetLastError();
}

}  // namespace cpht
