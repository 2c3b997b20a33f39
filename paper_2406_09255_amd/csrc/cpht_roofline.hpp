// Launcher of the random-access roofline probes (cpht_roofline.hip).
#pragma once
#include "cpht_device.hpp"

namespace cpht {
// kind 0: random 128-byte line reads; 1: random 32-bit CAS; 2: line read + CAS;
// 3: random 64-bit CAS; 4: the three-permutation split of every key of a buffer.
hipError_t launch_probe(int kind, void* buf, uint64_t bytes, uint64_t ops, uint64_t seed, uint32_t* sink,
                        hipStream_t s);
}  // namespace cpht
