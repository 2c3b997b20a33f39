// C-ABI of table sets: many independent tables in one device arena, served
// by one persistent launch per kernel variant (include/cpht.h, cpht_multi_*).
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <vector>

#include "cpht.h"
#include "cpht_internal.hpp"
#include "cpht_multi.hpp"
#include "cpht_util.hpp"

using namespace cpht;

struct cpht_multi {
  uint32_t n;
  int device;
  int key64;
  uint32_t scheme;
  uint32_t blocks;                 // persistent grid per launch
  cpht_table* tables;              // n views into the arena
  void* arena;
  uint64_t arena_bytes;
  uint64_t max_chunks;
  uint64_t max_keys;
  TableK* d_descs;                 // n kernel views
  uint32_t* d_order;               // table ids grouped by variant
  uint32_t* d_group_begin;         // n_groups + 1
  uint64_t* d_prefix;              // n + 1
  uint64_t* d_group_chunk;         // 2 * n_groups
  ChunkK* d_chunks;                // max_chunks
  uint32_t* d_error;
  std::vector<const IceVariant*> ice_groups;
  std::vector<const CkVariant*> ck_groups;
};

namespace {

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

void free_multi(cpht_multi* m) {
  if (m->arena) (void)hipFree(m->arena);
  if (m->d_descs) (void)hipFree(m->d_descs);
  if (m->d_order) (void)hipFree(m->d_order);
  if (m->d_group_begin) (void)hipFree(m->d_group_begin);
  if (m->d_prefix) (void)hipFree(m->d_prefix);
  if (m->d_group_chunk) (void)hipFree(m->d_group_chunk);
  if (m->d_chunks) (void)hipFree(m->d_chunks);
  if (m->d_error) (void)hipFree(m->d_error);
  delete[] m->tables;
  delete m;
}

template <class T>
hipError_t dalloc(T** p, uint64_t count) {
  return hipMalloc(reinterpret_cast<void**>(p), (count ? count : 1) * sizeof(T));
}

cpht_status_t run(cpht_multi* m, const void* d_keys, const uint64_t* d_offsets, uint64_t total, uint8_t* d_out,
                  void* stream, bool insert) {
  if (!m) return CPHT_E_ARG;
  if (total == 0) return CPHT_OK;
  if (!d_keys || !d_offsets || !d_out || total > m->max_keys) return CPHT_E_ARG;
  DeviceGuard g(m->device);
  if (!g.ok) return CPHT_E_DEVICE;
  const hipStream_t s = as_stream(stream);
  const uint32_t ng = (uint32_t)(m->ice_groups.size() + m->ck_groups.size());
  MultiPlanK P;
  P.offsets = d_offsets;
  P.order = m->d_order;
  P.group_begin = m->d_group_begin;
  P.n_tables = m->n;
  P.n_groups = ng;
  P.total_keys = total;
  P.max_chunks = m->max_chunks;
  P.prefix = m->d_prefix;
  P.group_chunk = m->d_group_chunk;
  P.chunks = m->d_chunks;
  P.error = m->d_error;
  hipError_t e = launch_multi_plan(P, s);
  if (e != hipSuccess) return device_status(e);
  for (uint32_t gi = 0; gi < ng; ++gi) {
    MultiK M;
    M.descs = m->d_descs;
    M.chunks = m->d_chunks;
    M.group = m->d_group_chunk + 2 * gi;
    M.keys = d_keys;
    M.out = d_out;
    if (m->scheme == CPHT_ICEBERG) {
      const IceVariant* v = m->ice_groups[gi];
      (insert ? v->multi_insert : v->multi_find)(M, m->blocks, s);
    } else {
      const CkVariant* v = m->ck_groups[gi];
      (insert ? v->multi_put : v->multi_find)(M, m->blocks, s);
    }
  }
  return device_status(hipGetLastError());
}

}  // namespace

extern "C" {

cpht_status_t cpht_multi_create(uint32_t n_tables, const cpht_config_t* cfgs, uint64_t max_keys, cpht_multi_t* out) {
  if (!cfgs || !out || n_tables == 0 || n_tables > (1u << 24)) return CPHT_E_ARG;
  *out = nullptr;
  cpht_multi* m = new (std::nothrow) cpht_multi();
  if (!m) return CPHT_E_NOMEM;
  m->n = n_tables;
  m->tables = new (std::nothrow) cpht_table[n_tables]();
  if (!m->tables) {
    delete m;
    return CPHT_E_NOMEM;
  }
  // configure every table; all must share the scheme and the key word size
  for (uint32_t i = 0; i < n_tables; ++i) {
    if (cfgs[i].pool_slabs != 0 || cfgs[i].value_bytes != 0) {  // no third level or map values in a set
      free_multi(m);
      return CPHT_E_UNSUPPORTED;
    }
    const cpht_status_t st = configure_table(&m->tables[i], cfgs[i]);
    if (st != CPHT_OK || cfgs[i].scheme != cfgs[0].scheme ||
        (cfgs[i].key_bits > 32) != (cfgs[0].key_bits > 32)) {
      free_multi(m);
      return st != CPHT_OK ? st : CPHT_E_ARG;
    }
  }
  m->scheme = cfgs[0].scheme;
  m->key64 = cfgs[0].key_bits > 32;
  // group tables by kernel variant (order of first appearance)
  std::vector<uint32_t> order;
  std::vector<uint32_t> begin;
  std::vector<bool> placed(n_tables, false);
  for (uint32_t i = 0; i < n_tables; ++i) {
    if (placed[i]) continue;
    begin.push_back((uint32_t)order.size());
    const void* v = m->scheme == CPHT_ICEBERG ? (const void*)m->tables[i].ice : (const void*)m->tables[i].ck;
    if (m->scheme == CPHT_ICEBERG) m->ice_groups.push_back(m->tables[i].ice);
    else m->ck_groups.push_back(m->tables[i].ck);
    for (uint32_t j = i; j < n_tables; ++j) {
      const void* w = m->scheme == CPHT_ICEBERG ? (const void*)m->tables[j].ice : (const void*)m->tables[j].ck;
      if (!placed[j] && w == v) {
        placed[j] = true;
        order.push_back(j);
      }
    }
  }
  begin.push_back(n_tables);
  const uint32_t ng = (uint32_t)begin.size() - 1;

  if (hipGetDevice(&m->device) != hipSuccess) {
    free_multi(m);
    return CPHT_E_DEVICE;
  }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, m->device) != hipSuccess || cus <= 0)
    cus = 256;
  m->blocks = (uint32_t)cus * 8;  // 2048 threads per CU at 256 threads per block

  // one arena for every level of every table, each level 256-byte aligned
  uint64_t bytes = 0;
  std::vector<uint64_t> offs;
  for (uint32_t i = 0; i < n_tables; ++i)
    for (int x = 0; x < m->tables[i].nlevels; ++x) {
      offs.push_back(bytes);
      bytes += (m->tables[i].level_words[x] * 4 + 255) / 256 * 256;
    }
  m->arena_bytes = bytes;
  m->max_keys = max_keys;
  m->max_chunks = max_keys / 256 + n_tables;
  hipError_t e = hipMalloc(&m->arena, bytes);
  if (e == hipSuccess) e = hipMemset(m->arena, 0, bytes);
  if (e == hipSuccess) e = dalloc(&m->d_descs, n_tables);
  if (e == hipSuccess) e = dalloc(&m->d_order, n_tables);
  if (e == hipSuccess) e = dalloc(&m->d_group_begin, ng + 1);
  if (e == hipSuccess) e = dalloc(&m->d_prefix, n_tables + 1);
  if (e == hipSuccess) e = dalloc(&m->d_group_chunk, 2 * ng);
  if (e == hipSuccess) e = dalloc(&m->d_chunks, m->max_chunks);
  if (e == hipSuccess) e = dalloc(&m->d_error, 1);
  if (e == hipSuccess) e = hipMemset(m->d_error, 0, sizeof(uint32_t));
  if (e != hipSuccess) {
    free_multi(m);
    return device_status(e);
  }
  size_t k = 0;
  std::vector<TableK> descs(n_tables);
  for (uint32_t i = 0; i < n_tables; ++i) {
    cpht_table& t = m->tables[i];
    t.device = m->device;
    t.owns_memory = false;
    for (int x = 0; x < t.nlevels; ++x) {
      t.level[x] = reinterpret_cast<uint32_t*>(static_cast<char*>(m->arena) + offs[k++]);
      t.tk.lv[x].base = t.level[x];
    }
    t.d_desc = m->d_descs + i;
    descs[i] = t.tk;
  }
  e = hipMemcpy(m->d_descs, descs.data(), n_tables * sizeof(TableK), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->d_order, order.data(), n_tables * sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(m->d_group_begin, begin.data(), (ng + 1) * sizeof(uint32_t), hipMemcpyHostToDevice);
  for (uint32_t i = 0; i < n_tables && e == hipSuccess; ++i)
    e = hipMalloc(reinterpret_cast<void**>(&m->tables[i].d_counter), sizeof(unsigned long long));
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    for (uint32_t i = 0; i < n_tables; ++i)
      if (m->tables[i].d_counter) (void)hipFree(m->tables[i].d_counter);
    free_multi(m);
    return device_status(e);
  }
  *out = m;
  return CPHT_OK;
}

cpht_status_t cpht_multi_destroy(cpht_multi_t m) {
  if (!m) return CPHT_E_ARG;
  DeviceGuard g(m->device);
  for (uint32_t i = 0; i < m->n; ++i)
    if (m->tables[i].d_counter) (void)hipFree(m->tables[i].d_counter);
  free_multi(m);
  return CPHT_OK;
}

cpht_status_t cpht_multi_table(cpht_multi_t m, uint32_t i, cpht_table_t* view) {
  if (!m || !view || i >= m->n) return CPHT_E_ARG;
  *view = &m->tables[i];
  return CPHT_OK;
}

cpht_status_t cpht_multi_clear(cpht_multi_t m, void* stream) {
  if (!m) return CPHT_E_ARG;
  DeviceGuard g(m->device);
  if (!g.ok) return CPHT_E_DEVICE;
  return device_status(launch_zero(static_cast<uint32_t*>(m->arena), m->arena_bytes / 4, as_stream(stream)));
}

cpht_status_t cpht_multi_insert(cpht_multi_t m, const void* d_keys, const uint64_t* d_offsets, uint64_t total_keys,
                                uint8_t* d_out, void* stream) {
  return run(m, d_keys, d_offsets, total_keys, d_out, stream, true);
}

cpht_status_t cpht_multi_find(cpht_multi_t m, const void* d_keys, const uint64_t* d_offsets, uint64_t total_keys,
                              uint8_t* d_found, void* stream) {
  return run(m, d_keys, d_offsets, total_keys, d_found, stream, false);
}

cpht_status_t cpht_multi_info(cpht_multi_t m, uint64_t* arena_bytes, uint32_t* n_groups, uint64_t* max_chunks) {
  if (!m) return CPHT_E_ARG;
  if (arena_bytes) *arena_bytes = m->arena_bytes;
  if (n_groups) *n_groups = (uint32_t)(m->ice_groups.size() + m->ck_groups.size());
  if (max_chunks) *max_chunks = m->max_chunks;
  return CPHT_OK;
}

cpht_status_t cpht_multi_error(cpht_multi_t m, uint32_t* flags) {
  if (!m || !flags) return CPHT_E_ARG;
  DeviceGuard g(m->device);
  if (!g.ok) return CPHT_E_DEVICE;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(flags, m->d_error, sizeof(uint32_t), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemset(m->d_error, 0, sizeof(uint32_t));
  return device_status(e);
}

}  // extern "C"
