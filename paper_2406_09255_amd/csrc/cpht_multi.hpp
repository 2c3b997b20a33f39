// Planner of many-table launches (cpht_multi.hip).
#pragma once
#include "cpht_device.hpp"

namespace cpht {

struct MultiPlanK {
  const uint64_t* offsets;     // n_tables + 1 key offsets (device)
  const uint32_t* order;       // table ids grouped by kernel variant (device)
  const uint32_t* group_begin; // n_groups + 1 positions into order (device)
  uint32_t n_tables, n_groups;
  uint64_t total_keys;         // keys past this index are ignored
  uint64_t max_chunks;         // capacity of `chunks`
  uint64_t* prefix;            // n_tables + 1 chunk prefix (device scratch)
  uint64_t* group_chunk;       // 2 * n_groups: first chunk, chunk count (device)
  ChunkK* chunks;              // max_chunks descriptors (device)
  uint32_t* error;             // bit 0: chunk capacity exceeded (device)
};

hipError_t launch_multi_plan(const MultiPlanK& P, hipStream_t s);

}  // namespace cpht
