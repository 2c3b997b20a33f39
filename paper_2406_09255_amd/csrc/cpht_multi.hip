// Device-side planning of a many-table launch: the concatenated keys of all
// tables (CSR offsets) are cut into chunks of at most 256 keys of one table,
// laid out grouped by kernel variant, so one persistent launch per variant
// group serves every table of that group.  Everything stays on the device,
// which lets a caller capture plan + launches in one graph.
#include "cpht_device.hpp"
#include "cpht_multi.hpp"

namespace cpht {

namespace {

__device__ __forceinline__ void table_range(const uint64_t* off, uint32_t t, uint64_t total, uint64_t& lo,
                                            uint64_t& hi) {
  lo = off[t] < total ? off[t] : total;
  const uint64_t e = off[t + 1] > lo ? off[t + 1] : lo;
  hi = e < total ? e : total;
}

// One block: chunk counts of the tables in group order, their exclusive
// prefix, and each group's (first chunk, chunk count), clamped to the chunk
// capacity (an overflow raises bit 0 of *error and drops the excess chunks).
__global__ __launch_bounds__(1024) void multi_plan_kernel(const uint64_t* off, const uint32_t* order, uint32_t n,
                                                          const uint32_t* group_begin, uint32_t n_groups,
                                                          uint64_t total, uint64_t max_chunks, uint64_t* prefix,
                                                          uint64_t* group_chunk, uint32_t* error) {
  __shared__ uint64_t part[1024];
  const uint32_t tid = threadIdx.x, nt = blockDim.x;
  const uint32_t per = (n + nt - 1) / nt;
  const uint32_t lo = tid * per < n ? tid * per : n;
  const uint32_t hi = lo + per < n ? lo + per : n;
  uint64_t sum = 0;
  for (uint32_t p = lo; p < hi; ++p) {
    uint64_t a, b;
    table_range(off, order[p], total, a, b);
    sum += (b - a + 255) / 256;
  }
  part[tid] = sum;
  __syncthreads();
  for (uint32_t d = 1; d < nt; d <<= 1) {
    const uint64_t v = tid >= d ? part[tid - d] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  uint64_t run = tid ? part[tid - 1] : 0;
  for (uint32_t p = lo; p < hi; ++p) {
    prefix[p] = run;
    uint64_t a, b;
    table_range(off, order[p], total, a, b);
    run += (b - a + 255) / 256;
  }
  if (tid == nt - 1) prefix[n] = part[nt - 1];
  __syncthreads();
  for (uint32_t g = tid; g < n_groups; g += nt) {
    uint64_t s = prefix[group_begin[g]], e = prefix[group_begin[g + 1]];
    s = s < max_chunks ? s : max_chunks;
    e = e < max_chunks ? e : max_chunks;
    group_chunk[2 * g] = s;
    group_chunk[2 * g + 1] = e - s;
  }
  if (tid == 0 && prefix[n] > max_chunks) atomicOr(error, 1u);
}

// One wave per table: its lanes write the table's chunk descriptors.
__global__ __launch_bounds__(256) void multi_fill_kernel(const uint64_t* off, const uint32_t* order, uint32_t n,
                                                         uint64_t total, const uint64_t* prefix, uint64_t max_chunks,
                                                         ChunkK* chunks) {
  const uint64_t gw = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t nw = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  const uint32_t lane = threadIdx.x & 63u;
  for (uint64_t p = gw; p < n; p += nw) {
    const uint32_t t = order[p];
    uint64_t a, b;
    table_range(off, t, total, a, b);
    const uint64_t base = prefix[p];
    const uint64_t cnt = (b - a + 255) / 256;
    for (uint64_t c = lane; c < cnt; c += 64) {
      const uint64_t i = base + c;
      if (i >= max_chunks) break;
      ChunkK ch;
      ch.start = a + 256 * c;
      ch.table = t;
      const uint64_t left = b - ch.start;
      ch.count = (uint32_t)(left < 256 ? left : 256);
      chunks[i] = ch;
    }
  }
}

}  // namespace

hipError_t launch_multi_plan(const MultiPlanK& P, hipStream_t s) {
  hipLaunchKernelGGL(multi_plan_kernel, dim3(1), dim3(1024), 0, s, P.offsets, P.order, P.n_tables, P.group_begin,
                     P.n_groups, P.total_keys, P.max_chunks, P.prefix, P.group_chunk, P.error);
  const uint32_t blocks = (P.n_tables + 3) / 4 < 4096 ? (P.n_tables + 3) / 4 : 4096;
  hipLaunchKernelGGL(multi_fill_kernel, dim3(blocks ? blocks : 1), dim3(256), 0, s, P.offsets, P.order, P.n_tables,
                     P.total_keys, P.prefix, P.max_chunks, P.chunks);
  return hipGetLastError();
}

}  // namespace cpht
