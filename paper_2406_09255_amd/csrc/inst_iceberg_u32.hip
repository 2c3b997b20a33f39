// Iceberg kernel instantiations for u32 key words: two-level find,
// find-or-put, mixed and delete, and the table-set kernels.
#include "cpht_iceberg.hpp"
#include "cpht_registry.hpp"

namespace cpht {
namespace {
template <int S0, int S1, int B0, int B1, int G, int MODE, bool L3ON>
void launch(const TableK& T, const BatchK& B, hipStream_t s) {
  launch_grid(iceberg_kernel<uint32_t, S0, S1, B0, B1, G, MODE, L3ON>, T, B, s);
}
template <int S0, int S1, int B0, int B1, int G, int MODE>
void launch_multi(const MultiK& M, uint32_t blocks, hipStream_t s) {
  launch_chunks(iceberg_multi_kernel<uint32_t, S0, S1, B0, B1, G, MODE>, M, blocks, s);
}
#define CPHT_ICE_BASE(S0, S1, B0, G) \
  {&launch<S0, S1, B0, B0 / 2, G, MODE_FIND, false>, &launch<S0, S1, B0, B0 / 2, G, MODE_INSERT, false>, \
   &launch<S0, S1, B0, B0 / 2, G, MODE_MIXED, false>, &launch<S0, S1, B0, B0 / 2, G, MODE_ERASE, false>},
#define CPHT_ICE_MULTI(S0, S1, B0, G) \
  {&launch_multi<S0, S1, B0, B0 / 2, G, MODE_FIND>, &launch_multi<S0, S1, B0, B0 / 2, G, MODE_INSERT>},
const IceLaunch4 kBase[] = {CPHT_ICE_LIST(CPHT_ICE_BASE)};
const IceMulti2 kMulti[] = {CPHT_ICE_LIST(CPHT_ICE_MULTI)};
}  // namespace

const IceLaunch4* ice_base_u32() { return kBase; }
const IceMulti2* ice_multi_u32() { return kMulti; }
}  // namespace cpht
