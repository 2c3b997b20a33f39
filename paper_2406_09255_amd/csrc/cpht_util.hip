// Table-wide kernels: occupancy count (fill factor, Sec. 2.1), clearing a
// level, and the key split a_i(k) / r'_i(k) exposed for direct checking of
// the permutation step (Sec. 2.4).
#include "cpht_device.hpp"
#include "cpht_util.hpp"

namespace cpht {

// Count the slots of S bits that hold a key (occupancy bit, the top bit of
// the slot, set; EMPTY and tombstones have it clear) in a level of `words`
// 32-bit words.  Each thread streams 16-byte pieces (grid-stride), the block
// reduces through LDS and adds its total to *count with one atomic.
template <int S>
__global__ __launch_bounds__(256) void count_kernel(const uint32_t* base, uint64_t words,
                                                    unsigned long long* count) {
  __shared__ unsigned long long part[4];
  const uint64_t nvec = words / 4;
  const uint4* v = reinterpret_cast<const uint4*>(base);
  uint32_t c = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvec;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint4 x = v[i];
    const uint32_t q[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if constexpr (S == 16) c += ((q[j] >> 15) & 1u) + (q[j] >> 31);
      else if constexpr (S == 32) c += q[j] >> 31;
      else if (j % 2 == 1) c += q[j] >> 31;  // high word of a 64-bit slot
    }
  }
  // tail words (levels smaller than 16 bytes or not a multiple of 4 words)
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (uint64_t i = nvec * 4; i < words; ++i) {
      const uint32_t q = base[i];
      if constexpr (S == 16) c += ((q >> 15) & 1u) + (q >> 31);
      else if constexpr (S == 32) c += q >> 31;
      else if ((i & 1) == 1) c += q >> 31;
    }
  }
  unsigned long long s = c;
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(count, part[0] + part[1] + part[2] + part[3]);
}

__global__ __launch_bounds__(256) void zero_kernel(uint32_t* base, uint64_t words) {
  const uint64_t nvec = words / 4;
  uint4* v = reinterpret_cast<uint4*>(base);
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvec;
       i += (uint64_t)gridDim.x * blockDim.x)
    v[i] = make_uint4(0u, 0u, 0u, 0u);
  if (blockIdx.x == 0 && threadIdx.x == 0)
    for (uint64_t i = nvec * 4; i < words; ++i) base[i] = 0u;
}

__global__ __launch_bounds__(256) void zero_u64_kernel(unsigned long long* p) { *p = 0ull; }

__global__ void desc_kernel(TableK T, TableK* dst) {
  if (threadIdx.x == 0) *dst = T;
}

// a_i(k) and the stored form r'_i(k) with tag `tag` at level `level`.
template <class U, int S>
__global__ __launch_bounds__(256) void split_kernel(TableK T, int level, int i, uint32_t tag, const U* keys,
                                                    uint64_t n, uint64_t* addr, uint64_t* stored) {
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const Split<U, S> s = split_key<U, S>(T, T.lv[level], i, keys[idx], tag);
  addr[idx] = s.a;
  stored[idx] = s.e;
}

static uint32_t stream_grid(uint64_t items) {
  uint64_t b = (items + 255) / 256;
  const uint64_t cap = 256ull * 64;  // enough 256-thread blocks to keep every CU busy
  return (uint32_t)(b < 1 ? 1 : (b > cap ? cap : b));
}

hipError_t launch_count(const uint32_t* base, uint64_t words, int slot_bits, unsigned long long* d_count,
                        hipStream_t s) {
  const uint32_t g = stream_grid(words / 4 + 1);
  if (slot_bits == 16) hipLaunchKernelGGL(count_kernel<16>, dim3(g), dim3(256), 0, s, base, words, d_count);
  else if (slot_bits == 32) hipLaunchKernelGGL(count_kernel<32>, dim3(g), dim3(256), 0, s, base, words, d_count);
  else hipLaunchKernelGGL(count_kernel<64>, dim3(g), dim3(256), 0, s, base, words, d_count);
  return hipGetLastError();
}

hipError_t launch_zero(uint32_t* base, uint64_t words, hipStream_t s) {
  hipLaunchKernelGGL(zero_kernel, dim3(stream_grid(words / 4 + 1)), dim3(256), 0, s, base, words);
  return hipGetLastError();
}

hipError_t launch_zero_counter(unsigned long long* p, hipStream_t s) {
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_store_desc(const TableK& T, TableK* dst, hipStream_t s) {
  hipLaunchKernelGGL(desc_kernel, dim3(1), dim3(64), 0, s, T, dst);
  return hipGetLastError();
}

hipError_t launch_split(const TableK& T, int level, int i, uint32_t tag, int key64, int slot_bits,
                        const void* keys, uint64_t n, uint64_t* addr, uint64_t* stored, hipStream_t s) {
  const dim3 g((uint32_t)((n + 255) / 256)), b(256);
#define CPHT_SPLIT(U, S) \
  hipLaunchKernelGGL((split_kernel<U, S>), g, b, 0, s, T, level, i, tag, static_cast<const U*>(keys), n, addr, stored)
  if (key64) {
    if (slot_bits == 16) CPHT_SPLIT(uint64_t, 16);
    else if (slot_bits == 32) CPHT_SPLIT(uint64_t, 32);
    else CPHT_SPLIT(uint64_t, 64);
  } else {
    if (slot_bits == 16) CPHT_SPLIT(uint32_t, 16);
    else if (slot_bits == 32) CPHT_SPLIT(uint32_t, 32);
    else CPHT_SPLIT(uint32_t, 64);
  }
#undef CPHT_SPLIT
  return hipGetLastError();
}

}  // namespace cpht
