// Iceberg kernel instantiations for u64 key words: map lookup and map
// find-or-put (values beside the keys), without and with the third level.
#include "cpht_iceberg.hpp"
#include "cpht_registry.hpp"

namespace cpht {
namespace {
template <int S0, int S1, int B0, int B1, int G, int MODE, bool L3ON>
void launch(const TableK& T, const BatchK& B, hipStream_t s) {
  launch_grid(iceberg_kernel<uint64_t, S0, S1, B0, B1, G, MODE, L3ON>, T, B, s);
}
template <int S0, int S1, int B0, int B1, int G, int MODE>
constexpr launch_fn launch3() {
  if constexpr (L3Shape<S0, G>::OK) return &launch<S0, S1, B0, B1, G, MODE, true>;
  else return nullptr;
}
#define CPHT_ICE_MAP(S0, S1, B0, G) \
  {&launch<S0, S1, B0, B0 / 2, G, MODE_FIND_V, false>, &launch<S0, S1, B0, B0 / 2, G, MODE_INSERT_V, false>, \
   launch3<S0, S1, B0, B0 / 2, G, MODE_FIND_V>(), launch3<S0, S1, B0, B0 / 2, G, MODE_INSERT_V>()},
const IceLaunch4 kMap[] = {CPHT_ICE_LIST(CPHT_ICE_MAP)};
}  // namespace

const IceLaunch4* ice_map_u64() { return kMap; }
}  // namespace cpht
