// Measurement kernels for the random-access roofline of the hash tables:
// the rate at which the device serves random 128-byte line reads, random
// 32-bit CAS, and a line read followed by a CAS into that line (the access
// pattern of a put).  They use the same sub-tile shape as the table kernels
// (8 lanes x 16 bytes per line) and keep 8 independent accesses in flight
// per group, like the pipelined batch kernels.
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
  } else {
    const uint64_t lines = bytes / 128;
    const uint64_t threads = (ops / per) * 8;
    hipLaunchKernelGGL(probe_line_cas_kernel, dim3(grid_for(threads)), dim3(256), 0, s, static_cast<uint4*>(buf),
                       lines - 1, per, seed, sink);
  }
  return hipGetLastError();
}

}  // namespace cpht
