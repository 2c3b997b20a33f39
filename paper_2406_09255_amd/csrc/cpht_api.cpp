// C-ABI of the compact hash table library (declared in include/cpht.h):
// table creation and configuration checks, permutation constants, and
// dispatch of batches to the compiled kernel variants.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <new>

#include "cpht.h"
#include "cpht_device.hpp"
#include "cpht_registry.hpp"
#include "cpht_roofline.hpp"
#include "cpht_sortfop.hpp"
#include "cpht_util.hpp"
#include "cpht_internal.hpp"

using namespace cpht;

namespace cpht {

// splitmix64 (Vigna): output number i+1 of the generator started at `seed`.
uint64_t splitmix(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t mask_bits(uint32_t w) { return w >= 64 ? ~0ull : ((1ull << w) - 1ull); }

// Inverse of odd m modulo 2^64 by Newton iteration x <- x(2 - m x); each step
// doubles the number of correct low-order bits (m is its own inverse mod 8).
uint64_t inverse_odd(uint64_t m) {
  uint64_t x = m;
  for (int i = 0; i < 5; ++i) x *= 2 - m * x;
  return x;
}

// Permutation i of the family: rounds q = 0..2 use multiplier
// (splitmix(seed, 3i+q) | 1) and xor constant splitmix(seed, 9+3i+q), both
// reduced mod 2^w.
void derive_perms(cpht_table* t, uint64_t seed) {
  const uint32_t w = t->cfg.key_bits;
  const uint64_t M = mask_bits(w);
  for (int i = 0; i < 3; ++i) {
    for (int q = 0; q < 3; ++q) {
      const uint64_t m = (splitmix(seed, 3 * i + q) | 1ull) & M;
      t->tk.perm[i].m[q] = m;
      t->tk.perm[i].minv[q] = inverse_odd(m) & M;
      t->tk.perm[i].c[q] = splitmix(seed, 9 + 3 * i + q) & M;
    }
  }
  t->cfg.seed = seed;
}

uint32_t log2_exact(uint64_t v) {
  uint32_t r = 0;
  while ((1ull << r) < v) ++r;
  return r;
}
bool pow2(uint64_t v) { return v && !(v & (v - 1)); }

cpht_status_t device_status(hipError_t e) {
  if (e == hipSuccess) return CPHT_OK;
  if (e == hipErrorOutOfMemory) return CPHT_E_NOMEM;
  return CPHT_E_DEVICE;
}

DeviceGuard::DeviceGuard(int dev) {
  if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
  if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
}
DeviceGuard::~DeviceGuard() {
  int cur = -1;
  if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
}

namespace {

// Fill in one level of the kernel view; returns false if the stored form
// (payload + tag + occupancy bit) does not fit the slot.
bool level_view(cpht_table* t, int x, uint32_t log2_slots, uint32_t B, uint32_t S, uint32_t tbits) {
  const uint32_t w = t->cfg.key_bits;
  const uint32_t lb = log2_exact(B);
  if (!pow2(B) || log2_slots < lb || log2_slots > 40) return false;
  const uint32_t nb = log2_slots - lb;
  if (nb > w || nb > 32) return false;
  const uint32_t pbits = t->cfg.compact ? w - nb : w;
  if (pbits + tbits + 1 > S) return false;
  LevelK& L = t->tk.lv[x];
  L.nb = nb;
  L.pbits = pbits;
  L.pmask = mask_bits(pbits);
  L.bucket_words = B * S / 32;
  L.tbits = tbits;
  t->slot_bits[x] = S;
  t->level_words[x] = ((1ull << log2_slots) * S) / 32;
  return true;
}

const IceVariant* find_ice(int key64, const cpht_config_t& c) {
  int n = 0;
  const IceVariant* v = key64 ? ice_variants_u64(&n) : ice_variants_u32(&n);
  for (int i = 0; i < n; ++i) {
    const IceVariant& e = v[i];
    if (e.S0 == (int)c.slot_bits0 && e.S1 == (int)c.slot_bits1 && e.B0 == (int)c.bucket0 &&
        e.B1 == (int)c.bucket1 && (c.subtile == 0 || e.G == (int)c.subtile))
      return &e;
  }
  return nullptr;
}

const CkVariant* find_ck(int key64, const cpht_config_t& c) {
  int n = 0;
  const CkVariant* v = key64 ? ck_variants_u64(&n) : ck_variants_u32(&n);
  for (int i = 0; i < n; ++i) {
    const CkVariant& e = v[i];
    if (e.S == (int)c.slot_bits0 && e.B == (int)c.bucket0 && (c.subtile == 0 || e.G == (int)c.subtile))
      return &e;
  }
  return nullptr;
}

}  // namespace

cpht_status_t configure_table(cpht_table* t, const cpht_config_t& c) {
  if (c.scheme != CPHT_CUCKOO && c.scheme != CPHT_ICEBERG) return CPHT_E_ARG;
  if (c.key_bits < 1 || c.key_bits > 64) return CPHT_E_ARG;
  if (c.compact > 1) return CPHT_E_ARG;
  t->cfg = c;
  const int key64 = c.key_bits > 32;
  TableK& K = t->tk;
  std::memset(&K, 0, sizeof(K));
  K.w = c.key_bits;
  K.h = (c.key_bits + 1) / 2;
  K.kmask = mask_bits(c.key_bits);
  K.compact = c.compact;
  bool ok = true;
  if (c.scheme == CPHT_CUCKOO) {
    if (c.n_hash < 2 || c.n_hash > 3 || c.max_chain < 1) ok = false;
    K.H = c.n_hash;
    K.C = c.max_chain;
    t->nlevels = 1;
    ok = ok && level_view(t, 0, c.log2_slots0, c.bucket0, c.slot_bits0, log2_exact(c.n_hash));
    if (ok) {
      t->ck = find_ck(key64, c);
      ok = t->ck != nullptr;
      if (ok) t->cfg.subtile = (uint32_t)t->ck->G;
    }
    t->cfg.log2_slots1 = 0;
    t->cfg.bucket1 = 0;
  } else {
    t->nlevels = 2;
    ok = c.bucket1 * 2 == c.bucket0;
    ok = ok && level_view(t, 0, c.log2_slots0, c.bucket0, c.slot_bits0, 0);
    ok = ok && level_view(t, 1, c.log2_slots1, c.bucket1, c.slot_bits1, 1);
    if (ok) {
      t->ice = find_ice(key64, c);
      ok = t->ice != nullptr;
      if (ok) t->cfg.subtile = (uint32_t)t->ice->G;
    }
  }
  t->nimages = t->nlevels;
  if (ok && c.pool_slabs > 0) {
    // third iceberg level: lists addressed by the high log2_lists bits of
    // pi_0(k); slots of 32 bits (64 with 64-bit primary slots)
    const uint32_t S3 = c.slot_bits0 == 64 ? 64 : 32;
    const uint32_t nb = c.log2_lists;
    const uint32_t pbits = c.compact ? c.key_bits - (nb <= c.key_bits ? nb : 0) : c.key_bits;
    ok = c.scheme == CPHT_ICEBERG && t->ice->l3 && nb <= c.key_bits && nb <= 30 && pbits + 1 <= S3 &&
         c.pool_slabs < 0x7FFFFFFFu;  // slab ids stay below the busy-link marker
    if (ok) {
      Level3K& L3 = K.l3;
      L3.L.nb = nb;
      L3.L.pbits = pbits;
      L3.L.pmask = mask_bits(pbits);
      L3.L.bucket_words = 32;
      L3.L.tbits = 0;
      L3.nslabs = c.pool_slabs;
      t->nimages = 4;
      t->level_words[2] = (uint64_t)c.pool_slabs * 32;
      t->level_words[3] = 1ull << nb;
      t->slot_bits[2] = S3;
      t->slot_bits[3] = 32;
    }
  } else {
    t->cfg.log2_lists = 0;
  }
  if (ok && c.value_bytes != 0) {  // map values: stable iceberg table only
    ok = c.scheme == CPHT_ICEBERG && (c.value_bytes == 4 || c.value_bytes == 8);
    if (ok) {
      K.vbytes = c.value_bytes;
      t->val_bytes[0] = (1ull << c.log2_slots0) * c.value_bytes;
      t->val_bytes[1] = (1ull << c.log2_slots1) * c.value_bytes;
      if (t->nimages == 4) t->val_bytes[2] = t->level_words[2] * 32 / t->slot_bits[2] * c.value_bytes;
    }
  }
  if (c.pad != 0) ok = false;
  if (!ok) return CPHT_E_UNSUPPORTED;
  derive_perms(t, c.seed);
  return CPHT_OK;
}

}  // namespace cpht

namespace {

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

BatchK batch(const void* keys, const uint8_t* ops, uint8_t* out, uint64_t n) {
  BatchK b;
  b.keys = keys;
  b.ops = ops;
  b.out = out;
  b.n = n;
  b.vin = nullptr;
  b.vout = nullptr;
  return b;
}

cpht_status_t launched() { return device_status(hipGetLastError()); }

}  // namespace

extern "C" {

void cpht_config_default(uint32_t scheme, cpht_config_t* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  c->scheme = scheme;
  c->key_bits = 32;
  c->compact = 1;
  c->seed = 1;
  c->n_hash = 2;
  c->max_chain = 256;
  if (scheme == CPHT_ICEBERG) {
    c->log2_slots0 = 20;
    c->log2_slots1 = 17;
    c->bucket0 = 32;
    c->bucket1 = 16;
    c->slot_bits0 = 16;
    c->slot_bits1 = 32;
  } else {
    c->log2_slots0 = 20;
    c->bucket0 = 32;
    c->slot_bits0 = 32;
  }
}

cpht_status_t cpht_config_check(const cpht_config_t* cfg, cpht_config_t* resolved) {
  if (!cfg) return CPHT_E_ARG;
  cpht_table t{};
  const cpht_status_t st = configure_table(&t, *cfg);
  if (st == CPHT_OK && resolved) *resolved = t.cfg;
  return st;
}

cpht_status_t cpht_create(const cpht_config_t* cfg, cpht_table_t* out) {
  if (!cfg || !out) return CPHT_E_ARG;
  *out = nullptr;
  cpht_table* t = new (std::nothrow) cpht_table();
  if (!t) return CPHT_E_NOMEM;
  const cpht_status_t st = configure_table(t, *cfg);
  if (st != CPHT_OK) {
    delete t;
    return st;
  }
  TableK& K = t->tk;
  t->owns_memory = true;

  if (hipGetDevice(&t->device) != hipSuccess) {
    delete t;
    return CPHT_E_DEVICE;
  }
  hipError_t e = hipSuccess;
  for (int x = 0; x < t->nimages && e == hipSuccess; ++x) {
    e = hipMalloc(reinterpret_cast<void**>(&t->level[x]), t->level_words[x] * 4);
    if (e == hipSuccess) e = hipMemset(t->level[x], 0, t->level_words[x] * 4);
    if (x < t->nlevels) K.lv[x].base = t->level[x];
  }
  if (e == hipSuccess && t->nimages == 4) {
    e = hipMalloc(reinterpret_cast<void**>(&t->l3_used), sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(t->l3_used, 0, sizeof(uint32_t));
    K.l3.L.base = t->level[2];
    K.l3.heads = t->level[3];
    K.l3.used = t->l3_used;
  }
  for (int x = 0; x < 3 && e == hipSuccess; ++x) {
    if (!t->val_bytes[x]) continue;
    e = hipMalloc(reinterpret_cast<void**>(&t->vals[x]), t->val_bytes[x]);
    if (e == hipSuccess) e = hipMemset(t->vals[x], 0, t->val_bytes[x]);
    K.vals[x] = t->vals[x];
  }
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&t->d_counter), sizeof(unsigned long long));
  if (e == hipSuccess && t->ck) {
    // set-up of the allocation-free sorted find-or-put on this device: its
    // scratch array's address is looked up here, once per device, so that
    // the call itself (possibly under graph capture) makes no runtime lookup
    void* scratch_addr = nullptr;
    e = sorted_fop_scratch(t->device, &scratch_addr);
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    for (int x = 0; x < 4; ++x)
      if (t->level[x]) (void)hipFree(t->level[x]);
    for (int x = 0; x < 3; ++x)
      if (t->vals[x]) (void)hipFree(t->vals[x]);
    if (t->l3_used) (void)hipFree(t->l3_used);
    if (t->d_counter) (void)hipFree(t->d_counter);
    delete t;
    return device_status(e);
  }
  *out = t;
  return CPHT_OK;
}

cpht_status_t cpht_destroy(cpht_table_t t) {
  if (!t) return CPHT_E_ARG;
  if (!t->owns_memory) return CPHT_E_STATE;  // a view into a table set
  DeviceGuard g(t->device);
  for (int x = 0; x < 4; ++x)
    if (t->level[x]) (void)hipFree(t->level[x]);
  for (int x = 0; x < 3; ++x)
    if (t->vals[x]) (void)hipFree(t->vals[x]);
  if (t->l3_used) (void)hipFree(t->l3_used);
  if (t->d_counter) (void)hipFree(t->d_counter);
  delete t;
  return CPHT_OK;
}

cpht_status_t cpht_get_config(cpht_table_t t, cpht_config_t* cfg) {
  if (!t || !cfg) return CPHT_E_ARG;
  *cfg = t->cfg;
  return CPHT_OK;
}

cpht_status_t cpht_clear(cpht_table_t t, uint64_t seed, void* stream) {
  if (!t) return CPHT_E_ARG;
  DeviceGuard g(t->device);
  if (!g.ok) return CPHT_E_DEVICE;
  derive_perms(t, seed);
  if (t->d_desc) {  // a table-set view: its set's launches read the device copy
    hipError_t e = launch_store_desc(t->tk, t->d_desc, as_stream(stream));
    if (e != hipSuccess) return device_status(e);
  }
  for (int x = 0; x < t->nimages; ++x) {
    hipError_t e = launch_zero(t->level[x], t->level_words[x], as_stream(stream));
    if (e != hipSuccess) return device_status(e);
  }
  if (t->l3_used) {
    hipError_t e = launch_zero(t->l3_used, 1, as_stream(stream));
    if (e != hipSuccess) return device_status(e);
  }
  for (int x = 0; x < 3; ++x) {
    if (!t->vals[x]) continue;
    hipError_t e = launch_zero(reinterpret_cast<uint32_t*>(t->vals[x]), t->val_bytes[x] / 4, as_stream(stream));
    if (e != hipSuccess) return device_status(e);
  }
  return CPHT_OK;
}

cpht_status_t cpht_insert(cpht_table_t t, const void* d_keys, uint64_t n, uint8_t* d_out, void* stream) {
  if (!t) return CPHT_E_ARG;
  if (n == 0) return CPHT_OK;
  if (!d_keys || !d_out) return CPHT_E_ARG;
  DeviceGuard g(t->device);
  if (!g.ok) return CPHT_E_DEVICE;
  const BatchK b = batch(d_keys, nullptr, d_out, n);
  if (t->ice) (t->nimages == 4 ? t->ice->insert3 : t->ice->insert)(t->tk, b, as_stream(stream));
  else t->ck->put(t->tk, b, as_stream(stream));
  return launched();
}

cpht_status_t cpht_bulk_build(cpht_table_t t, const void* d_keys, uint64_t n, uint8_t* d_out, void* stream) {
  return cpht_insert(t, d_keys, n, d_out, stream);
}

cpht_status_t cpht_find(cpht_table_t t, const void* d_keys, uint64_t n, uint8_t* d_found, void* stream) {
  if (!t) return CPHT_E_ARG;
  if (n == 0) return CPHT_OK;
  if (!d_keys || !d_found) return CPHT_E_ARG;
  DeviceGuard g(t->device);
  if (!g.ok) return CPHT_E_DEVICE;
  const BatchK b = batch(d_keys, nullptr, d_found, n);
  if (t->ice) (t->nimages == 4 ? t->ice->find3 : t->ice->find)(t->tk, b, as_stream(stream));
  else t->ck->find(t->tk, b, as_stream(stream));
  return launched();
}

cpht_status_t cpht_delete(cpht_table_t t, const void* d_keys, uint64_t n, uint8_t* d_out, void* stream) {
  if (!t) return CPHT_E_ARG;
  if (n == 0) return CPHT_OK;
  if (!d_keys || !d_out) return CPHT_E_ARG;
  DeviceGuard g(t->device);
  if (!g.ok) return CPHT_E_DEVICE;
  const BatchK b = batch(d_keys, nullptr, d_out, n);
  if (t->ice) (t->nimages == 4 ? t->ice->erase3 : t->ice->erase)(t->tk, b, as_stream(stream));
  else t->ck->erase(t->tk, b, as_stream(stream));
  return launched();
}

cpht_status_t cpht_mixed(cpht_table_t t, const void* d_keys, const uint8_t* d_ops, uint64_t n, uint8_t* d_out,
                         void* stream) {
  if (!t) return CPHT_E_ARG;
  if (!t->ice) return CPHT_E_STATE;
  if (n == 0) return CPHT_OK;
  if (!d_keys || !d_ops || !d_out) return CPHT_E_ARG;
  DeviceGuard g(t->device);
  if (!g.ok) return CPHT_E_DEVICE;
  (t->nimages == 4 ? t->ice->mixed3 : t->ice->mixed)(t->tk, batch(d_keys, d_ops, d_out, n), as_stream(stream));
  return launched();
}

cpht_status_t cpht_insert_values(cpht_table_t t, const void* d_keys, const void* d_values, uint64_t n,
                                 uint8_t* d_out, void* stream) {
  if (!t) return CPHT_E_ARG;
  if (!t->tk.vbytes) return CPHT_E_STATE;
  if (n == 0) return CPHT_OK;
  if (!d_keys || !d_values || !d_out) return CPHT_E_ARG;
  DeviceGuard g(t->device);
  if (!g.ok) return CPHT_E_DEVICE;
  BatchK b = batch(d_keys, nullptr, d_out, n);
  b.vin = d_values;
  (t->nimages == 4 ? t->ice->insert_v3 : t->ice->insert_v)(t->tk, b, as_stream(stream));
  return launched();
}

cpht_status_t cpht_find_values(cpht_table_t t, const void* d_keys, uint64_t n, uint8_t* d_found,
                               void* d_values_out, void* stream) {
  if (!t) return CPHT_E_ARG;
  if (!t->tk.vbytes) return CPHT_E_STATE;
  if (n == 0) return CPHT_OK;
  if (!d_keys || !d_found || !d_values_out) return CPHT_E_ARG;
  DeviceGuard g(t->device);
  if (!g.ok) return CPHT_E_DEVICE;
  BatchK b = batch(d_keys, nullptr, d_found, n);
  b.vout = d_values_out;
  (t->nimages == 4 ? t->ice->find_v3 : t->ice->find_v)(t->tk, b, as_stream(stream));
  return launched();
}

cpht_status_t cpht_values_bytes(cpht_table_t t, uint32_t level, uint64_t* bytes) {
  if (!t || !bytes || level > 2) return CPHT_E_ARG;
  if (!t->vals[level]) return CPHT_E_STATE;
  *bytes = t->val_bytes[level];
  return CPHT_OK;
}

cpht_status_t cpht_export_values(cpht_table_t t, uint32_t level, void* h_dst, uint64_t bytes) {
  if (!t || !h_dst || level > 2) return CPHT_E_ARG;
  if (!t->vals[level]) return CPHT_E_STATE;
  if (bytes != t->val_bytes[level]) return CPHT_E_ARG;
  DeviceGuard g(t->device);
  if (!g.ok) return CPHT_E_DEVICE;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(h_dst, t->vals[level], bytes, hipMemcpyDeviceToHost);
  return device_status(e);
}

// The sorted find-or-put on t's device (current) with workspace `ws`.
static cpht_status_t run_sorted_fop(cpht_table_t t, const void* d_keys, uint64_t n, uint8_t* d_out, void* ws,
                                    void* stream) {
  int cus = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, t->device);
  if (e != hipSuccess) return device_status(e);
  e = launch_sorted_fop(t->tk, t->ck, (int)t->cfg.key_bits, d_keys, n, d_out, ws,
                        (uint32_t)(cus > 0 ? cus * 8 : 2048), as_stream(stream));
  return device_status(e);
}

cpht_status_t cpht_sorted_fop_workspace(cpht_table_t t, uint64_t n, uint64_t* bytes) {
  if (!t || !bytes) return CPHT_E_ARG;
  if (!t->ck) return CPHT_E_STATE;
  if (n >= (1ull << 32)) return CPHT_E_ARG;
  *bytes = sorted_fop_workspace(n, t->cfg.key_bits > 32 ? 8 : 4);
  return CPHT_OK;
}

cpht_status_t cpht_sorted_fop(cpht_table_t t, const void* d_keys, uint64_t n, uint8_t* d_out, void* d_workspace,
                              uint64_t workspace_bytes, void* stream) {
  if (!t) return CPHT_E_ARG;
  if (!t->ck) return CPHT_E_STATE;
  if (n == 0) return CPHT_OK;
  if (!d_keys || !d_out || !d_workspace || n >= (1ull << 32)) return CPHT_E_ARG;
  if (reinterpret_cast<uintptr_t>(d_workspace) % 256 != 0) return CPHT_E_ARG;
  if (workspace_bytes < sorted_fop_workspace(n, t->cfg.key_bits > 32 ? 8 : 4)) return CPHT_E_ARG;
  DeviceGuard g(t->device);
  if (!g.ok) return CPHT_E_DEVICE;
  return run_sorted_fop(t, d_keys, n, d_out, d_workspace, stream);
}

cpht_status_t cpht_sorted_fop_noalloc(cpht_table_t t, const void* d_keys, uint64_t n, uint8_t* d_out, void* stream) {
  if (!t) return CPHT_E_ARG;
  if (!t->ck) return CPHT_E_STATE;
  if (n == 0) return CPHT_OK;
  if (!d_keys || !d_out || n > NOALLOC_MAX_KEYS) return CPHT_E_ARG;
  if (sorted_fop_workspace(n, t->cfg.key_bits > 32 ? 8 : 4) > NOALLOC_SCRATCH_BYTES) return CPHT_E_ARG;
  DeviceGuard g(t->device);
  if (!g.ok) return CPHT_E_DEVICE;
  void* ws = nullptr;
  const hipError_t e = sorted_fop_scratch(t->device, &ws);
  if (e != hipSuccess) return device_status(e);
  return run_sorted_fop(t, d_keys, n, d_out, ws, stream);
}

cpht_status_t cpht_count(cpht_table_t t, uint64_t* occupied, uint64_t* capacity, void* stream) {
  if (!t) return CPHT_E_ARG;
  DeviceGuard g(t->device);
  if (!g.ok) return CPHT_E_DEVICE;
  const hipStream_t s = as_stream(stream);
  hipError_t e = launch_zero_counter(t->d_counter, s);
  for (int x = 0; x < t->nimages && x < 3 && e == hipSuccess; ++x)  // bucket levels and the slab pool
    e = launch_count(t->level[x], t->level_words[x], (int)t->slot_bits[x], t->d_counter, s);
  unsigned long long h = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&h, t->d_counter, sizeof(h), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return device_status(e);
  if (occupied) *occupied = h;
  if (capacity) {
    uint64_t cap = 0;
    for (int x = 0; x < t->nlevels; ++x) cap += t->level_words[x] * 32 / t->slot_bits[x];
    *capacity = cap;
  }
  return CPHT_OK;
}

cpht_status_t cpht_level_bytes(cpht_table_t t, uint32_t level, uint64_t* bytes) {
  if (!t || !bytes || level >= (uint32_t)t->nimages) return CPHT_E_ARG;
  *bytes = t->level_words[level] * 4;
  return CPHT_OK;
}

cpht_status_t cpht_level_ptr(cpht_table_t t, uint32_t level, void** d_ptr) {
  if (!t || !d_ptr || level >= (uint32_t)t->nimages) return CPHT_E_ARG;
  *d_ptr = t->level[level];
  return CPHT_OK;
}

cpht_status_t cpht_level3_used(cpht_table_t t, uint32_t* slabs) {
  if (!t || !slabs) return CPHT_E_ARG;
  if (t->nimages != 4) return CPHT_E_STATE;
  DeviceGuard g(t->device);
  if (!g.ok) return CPHT_E_DEVICE;
  uint32_t h = 0;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(&h, t->l3_used, sizeof(h), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return device_status(e);
  *slabs = h < t->cfg.pool_slabs ? h : t->cfg.pool_slabs;
  return CPHT_OK;
}

cpht_status_t cpht_export(cpht_table_t t, uint32_t level, void* h_dst, uint64_t bytes) {
  if (!t || !h_dst || level >= (uint32_t)t->nimages || bytes != t->level_words[level] * 4) return CPHT_E_ARG;
  DeviceGuard g(t->device);
  if (!g.ok) return CPHT_E_DEVICE;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(h_dst, t->level[level], bytes, hipMemcpyDeviceToHost);
  return device_status(e);
}

cpht_status_t cpht_import(cpht_table_t t, uint32_t level, const void* h_src, uint64_t bytes) {
  if (!t || !h_src || level >= (uint32_t)t->nimages || bytes != t->level_words[level] * 4) return CPHT_E_ARG;
  DeviceGuard g(t->device);
  if (!g.ok) return CPHT_E_DEVICE;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(t->level[level], h_src, bytes, hipMemcpyHostToDevice);
  if (e == hipSuccess && level == 2) {
    // slabs are taken in id order and each one taken is on a list, so the
    // count taken is the highest slab holding a nonzero word
    const uint32_t* w = static_cast<const uint32_t*>(h_src);
    uint32_t used = 0;
    for (uint64_t i = t->level_words[2]; i-- > 0;)
      if (w[i]) {
        used = (uint32_t)(i / 32 + 1);
        break;
      }
    e = hipMemcpy(t->l3_used, &used, sizeof(used), hipMemcpyHostToDevice);
  }
  return device_status(e);
}

cpht_status_t cpht_import_values(cpht_table_t t, uint32_t level, const void* h_src, uint64_t bytes) {
  if (!t || !h_src || level > 2) return CPHT_E_ARG;
  if (!t->vals[level]) return CPHT_E_STATE;
  if (bytes != t->val_bytes[level]) return CPHT_E_ARG;
  DeviceGuard g(t->device);
  if (!g.ok) return CPHT_E_DEVICE;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(t->vals[level], h_src, bytes, hipMemcpyHostToDevice);
  return device_status(e);
}

cpht_status_t cpht_split(cpht_table_t t, uint32_t perm_index, const void* d_keys, uint64_t n, uint64_t* d_addr,
                         uint64_t* d_stored, void* stream) {
  if (!t) return CPHT_E_ARG;
  const bool ice = t->ice != nullptr;
  if (perm_index >= (ice ? 3u : t->cfg.n_hash)) return CPHT_E_ARG;
  if (n == 0) return CPHT_OK;
  if (!d_keys || !d_addr || !d_stored) return CPHT_E_ARG;
  DeviceGuard g(t->device);
  if (!g.ok) return CPHT_E_DEVICE;
  const int level = ice && perm_index > 0 ? 1 : 0;
  const uint32_t tag = ice ? (perm_index == 2 ? 1u : 0u) : perm_index;
  hipError_t e = launch_split(t->tk, level, (int)perm_index, tag, t->cfg.key_bits > 32, (int)t->slot_bits[level],
                              d_keys, n, d_addr, d_stored, as_stream(stream));
  return device_status(e);
}

int cpht_variant_info(uint32_t scheme, int i, uint32_t* info) {
  int n32 = 0, n64 = 0;
  if (scheme == CPHT_ICEBERG) {
    const IceVariant* a = ice_variants_u32(&n32);
    const IceVariant* b = ice_variants_u64(&n64);
    if (info && i >= 0 && i < n32 + n64) {
      const IceVariant& v = i < n32 ? a[i] : b[i - n32];
      const uint32_t vals[6] = {(uint32_t)v.key64, (uint32_t)v.S0, (uint32_t)v.S1,
                                (uint32_t)v.B0, (uint32_t)v.B1, (uint32_t)v.G};
      std::memcpy(info, vals, sizeof(vals));
    }
  } else if (scheme == CPHT_CUCKOO) {
    const CkVariant* a = ck_variants_u32(&n32);
    const CkVariant* b = ck_variants_u64(&n64);
    if (info && i >= 0 && i < n32 + n64) {
      const CkVariant& v = i < n32 ? a[i] : b[i - n32];
      const uint32_t vals[6] = {(uint32_t)v.key64, (uint32_t)v.S, 0u, (uint32_t)v.B, 0u, (uint32_t)v.G};
      std::memcpy(info, vals, sizeof(vals));
    }
  } else {
    return 0;
  }
  return n32 + n64;
}

cpht_status_t cpht_probe(uint32_t kind, void* d_buf, uint64_t bytes, uint64_t ops, uint64_t seed, uint32_t* d_sink,
                         uint64_t* ops_done, void* stream) {
  if (kind > 6 || !d_buf || !d_sink || bytes < 4096 || !pow2(bytes) || ops == 0) return CPHT_E_ARG;
  // whole 256-thread blocks: 16384 operations per block for every kind
  const uint64_t unit = 16384;
  const uint64_t n = (ops + unit - 1) / unit * unit;
  hipError_t e = launch_probe((int)kind, d_buf, bytes, n, seed, d_sink, as_stream(stream));
  if (e != hipSuccess) return device_status(e);
  if (ops_done) *ops_done = n;
  return CPHT_OK;
}

const char* cpht_status_str(cpht_status_t s) {
  switch (s) {
    case CPHT_OK: return "ok";
    case CPHT_E_ARG: return "invalid argument";
    case CPHT_E_NOMEM: return "out of device memory";
    case CPHT_E_UNSUPPORTED: return "unsupported configuration";
    case CPHT_E_KEYRANGE: return "key out of range";
    case CPHT_E_DEVICE: return "device error";
    case CPHT_E_BUSY: return "busy";
    case CPHT_E_STATE: return "operation not valid for this table";
  }
  return "unknown status";
}

}  // extern "C"
