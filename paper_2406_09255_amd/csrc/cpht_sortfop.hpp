// Find-or-put on the static cuckoo table by sorting the batch first
// (cpht_sortfop.hip).
#pragma once
#include "cpht_device.hpp"
#include "cpht_registry.hpp"

namespace cpht {

// Bytes of device workspace the pipeline needs for n keys of key_bytes each.
uint64_t sorted_fop_workspace(uint64_t n, int key_bytes);

// The allocation-free variant runs the pipeline in a fixed device array of
// NOALLOC_SCRATCH_BYTES per GPU, enough for NOALLOC_MAX_KEYS keys of either
// key width (64-bit keys need 41,227,520 bytes at 2^20 keys).
constexpr uint64_t NOALLOC_SCRATCH_BYTES = 40ull << 20;
constexpr uint64_t NOALLOC_MAX_KEYS = 1ull << 20;

// Device address of that array on `device`, which must be the current
// device.  The runtime is asked once per device; later calls return the
// stored address.
hipError_t sorted_fop_scratch(int device, void** ptr);

// Runs the whole pipeline on stream s.  `v` is the table's cuckoo variant,
// `blocks` the persistent grid of the lookup and put launches.
hipError_t launch_sorted_fop(const TableK& T, const CkVariant* v, int key_bits, const void* keys, uint64_t n,
                             uint8_t* out, void* workspace, uint32_t blocks, hipStream_t s);

}  // namespace cpht
