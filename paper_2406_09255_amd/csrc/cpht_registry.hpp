// Table of compiled kernel variants.  Sizes that shape registers (slot bits,
// bucket slots, sub-tile width) are template parameters; the host library
// picks the variant matching a table's configuration.
#pragma once
#include "cpht_device.hpp"

namespace cpht {

typedef void (*launch_fn)(const TableK&, const BatchK&, hipStream_t);
typedef void (*multi_fn)(const MultiK&, uint32_t blocks, hipStream_t);
struct RingCtl;
struct ResidentState;
// The resident request loop (cpht_resident.hpp): `blocks` = 1 leader + workers.
typedef hipError_t (*resident_fn)(const TableK&, RingCtl* ctl, ResidentState* st, uint32_t epoch,
                                  uint64_t idle_ticks, uint32_t blocks, hipStream_t);

struct IceVariant {
  int key64;           // 1: 64-bit key words
  int S0, S1, B0, B1;  // slot bits and bucket slots per level
  int G;               // sub-tile lanes
  int l3;              // 1: a third level is possible (whole slots per lane on a slab)
  launch_fn find, insert, mixed, erase;
  launch_fn find3, insert3, mixed3, erase3;  // with the third level compiled in (null if l3 = 0)
  launch_fn find_v, insert_v, find_v3, insert_v3;  // map lookup / find-or-put (values), without / with level 3
  multi_fn multi_find, multi_insert;
  resident_fn resident;  // the serving loop's persistent mixed-batch kernel (two levels)
};

struct CkVariant {
  int key64;
  int S, B, G;
  launch_fn put, find, erase;
  multi_fn multi_put, multi_find;
};

// Iceberg variants: (S0, S1, B0, G) with B1 = B0 / 2.  The first entry for a
// given (S0, S1, B0) is the default sub-tile width: two 16-byte loads (32
// bytes) per lane on the primary bucket where the bucket allows it, which
// measured faster than one 16-byte load per lane (fewer ballot rounds per
// wave for the same keys in flight); the second entry is that alternative.
#define CPHT_ICE_LIST(X) \
  X(16, 16, 8, 2)  X(16, 32, 8, 2)  X(32, 32, 8, 2)  X(64, 64, 8, 2)  X(64, 64, 8, 4) \
  X(16, 16, 16, 2) X(16, 32, 16, 2) X(32, 32, 16, 2) X(32, 32, 16, 4) X(64, 64, 16, 4) X(64, 64, 16, 8) \
  X(16, 16, 32, 2) X(16, 16, 32, 4) X(16, 32, 32, 2) X(16, 32, 32, 4) X(32, 32, 32, 4) X(32, 32, 32, 8) \
  X(64, 64, 32, 8) X(64, 64, 32, 16) \
  X(16, 16, 64, 4) X(16, 16, 64, 8) X(16, 32, 64, 4) X(16, 32, 64, 8) X(16, 32, 64, 2) X(32, 32, 64, 8) \
  X(32, 32, 64, 16) \
  X(64, 64, 64, 16) X(64, 64, 64, 32)

// Cuckoo variants: (S, B, G); first entry per (S, B) is the default, then the
// alternatives.  For 128-byte buckets of 32-bit slots 64 bytes per lane
// (G = 2) measured fastest, ahead of 32 (G = 4) and 16 (G = 8) bytes per lane.
#define CPHT_CK_LIST(X) \
  X(32, 8, 2) X(32, 16, 2) X(32, 16, 4) X(32, 32, 2) X(32, 32, 4) X(32, 32, 8) \
  X(64, 8, 2) X(64, 8, 4) X(64, 16, 4) X(64, 16, 8) X(64, 32, 8) X(64, 32, 16)

const IceVariant* ice_variants_u32(int* n);
const IceVariant* ice_variants_u64(int* n);

// Iceberg launchers come from three translation units per key word (compiled
// in parallel), one entry per CPHT_ICE_LIST position; cpht_registry.hip
// assembles them into IceVariant records.
struct IceLaunch4 {
  launch_fn a, b, c, d;
};
struct IceMulti2 {
  multi_fn find, insert;
};
const IceLaunch4* ice_base_u32();   // find, insert, mixed, erase
const IceMulti2* ice_multi_u32();   // table-set find, insert
const IceLaunch4* ice_l3_u32();     // the same four with the third level (null where impossible)
const IceLaunch4* ice_map_u32();    // map find, map insert, and both with the third level
const IceLaunch4* ice_base_u64();
const IceMulti2* ice_multi_u64();
const IceLaunch4* ice_l3_u64();
const IceLaunch4* ice_map_u64();
const resident_fn* ice_resident_u32();  // one per CPHT_ICE_LIST position
const resident_fn* ice_resident_u64();
const CkVariant* ck_variants_u32(int* n);
const CkVariant* ck_variants_u64(int* n);

template <class Kern>
inline void launch_grid(Kern k, const TableK& T, const BatchK& B, hipStream_t s) {
  const uint64_t blocks = (B.n + 255) / 256;
  hipLaunchKernelGGL(k, dim3((uint32_t)blocks), dim3(256), 0, s, T, B);
}

// `blocks` is the fixed (persistent) grid; the blocks walk the group's chunks.
template <class Kern>
inline void launch_chunks(Kern k, const MultiK& M, uint32_t blocks, hipStream_t s) {
  hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, s, M);
}

}  // namespace cpht
