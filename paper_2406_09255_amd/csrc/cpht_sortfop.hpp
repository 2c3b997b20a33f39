// Find-or-put on the static cuckoo table by sorting the batch first
// (cpht_sortfop.hip).
#pragma once
#include "cpht_device.hpp"
#include "cpht_registry.hpp"

namespace cpht {

// Bytes of device workspace the pipeline needs for n keys of key_bytes each.
uint64_t sorted_fop_workspace(uint64_t n, int key_bytes);

// Runs the whole pipeline on stream s.  `v` is the table's cuckoo variant,
// `blocks` the persistent grid of the lookup and put launches.
hipError_t launch_sorted_fop(const TableK& T, const CkVariant* v, int key_bits, const void* keys, uint64_t n,
                             uint8_t* out, void* workspace, uint32_t blocks, hipStream_t s);

}  // namespace cpht
