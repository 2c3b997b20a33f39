// Host-callable launchers for the table-wide kernels in cpht_util.hip.
#pragma once
#include "cpht_device.hpp"

namespace cpht {
hipError_t launch_count(const uint32_t* base, uint64_t words, int slot_bits, unsigned long long* d_count,
                        hipStream_t s);
hipError_t launch_zero(uint32_t* base, uint64_t words, hipStream_t s);
hipError_t launch_zero_counter(unsigned long long* p, hipStream_t s);
// Write a kernel view to device memory (a kernel, so it is stream-ordered and
// can be captured in a graph).
hipError_t launch_store_desc(const TableK& T, TableK* dst, hipStream_t s);
hipError_t launch_split(const TableK& T, int level, int i, uint32_t tag, int key64, int slot_bits,
                        const void* keys, uint64_t n, uint64_t* addr, uint64_t* stored, hipStream_t s);
}  // namespace cpht
