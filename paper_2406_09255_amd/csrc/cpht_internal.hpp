// Host-side internals shared by the C-ABI source files.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cpht.h"
#include "cpht_device.hpp"
#include "cpht_registry.hpp"

// One table: its resolved configuration, kernel view and device memory.
// Images 0 and 1 are the bucket levels; with a third iceberg level, image 2
// is its slab pool and image 3 its list heads (nimages = 4).
struct cpht_table {
  cpht_config_t cfg;
  int device;
  int nlevels;   // bucket levels: 1 (cuckoo) or 2 (iceberg)
  int nimages;   // device arrays exported by cpht_export
  bool owns_memory;
  uint32_t* level[4];
  uint64_t level_words[4];
  uint32_t slot_bits[4];
  uint32_t* l3_used;  // level 3: slabs handed out (device)
  uint8_t* vals[3];   // map values of levels 0, 1 and the slab pool (device)
  uint64_t val_bytes[3];
  unsigned long long* d_counter;
  cpht::TableK tk;
  // Table-set view: the set's device copy of tk, read by its launches (kept
  // equal to tk by every call that changes tk); null for an owning table.
  cpht::TableK* d_desc;
  const cpht::IceVariant* ice;
  const cpht::CkVariant* ck;
};

namespace cpht {

uint64_t splitmix(uint64_t seed, uint64_t i);
uint64_t mask_bits(uint32_t w);
uint64_t inverse_odd(uint64_t m);
void derive_perms(cpht_table* t, uint64_t seed);
uint32_t log2_exact(uint64_t v);
bool pow2(uint64_t v);
cpht_status_t device_status(hipError_t e);

// Validate `c`, resolve the kernel variant and fill t's kernel view (level
// sizes, payload widths, permutation constants).  Allocates nothing.
cpht_status_t configure_table(cpht_table* t, const cpht_config_t& c);

// Makes a device current for the lifetime of the guard.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev);
  ~DeviceGuard();
};

}  // namespace cpht
