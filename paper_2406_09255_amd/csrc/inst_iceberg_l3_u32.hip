// Iceberg kernel instantiations for u32 key words: find, find-or-put,
// mixed and delete with the third level compiled in.
#include "cpht_iceberg.hpp"
#include "cpht_registry.hpp"

namespace cpht {
namespace {
template <int S0, int S1, int B0, int B1, int G, int MODE, bool L3ON>
void launch(const TableK& T, const BatchK& B, hipStream_t s) {
  launch_grid(iceberg_kernel<uint32_t, S0, S1, B0, B1, G, MODE, L3ON>, T, B, s);
}
// The launcher with the third level, or null where the shape has none.
template <int S0, int S1, int B0, int B1, int G, int MODE>
constexpr launch_fn launch3() {
  if constexpr (L3Shape<S0, G>::OK) return &launch<S0, S1, B0, B1, G, MODE, true>;
  else return nullptr;
}
#define CPHT_ICE_L3(S0, S1, B0, G) \
  {launch3<S0, S1, B0, B0 / 2, G, MODE_FIND>(), launch3<S0, S1, B0, B0 / 2, G, MODE_INSERT>(), \
   launch3<S0, S1, B0, B0 / 2, G, MODE_MIXED>(), launch3<S0, S1, B0, B0 / 2, G, MODE_ERASE>()},
const IceLaunch4 kL3[] = {CPHT_ICE_LIST(CPHT_ICE_L3)};
}  // namespace

const IceLaunch4* ice_l3_u32() { return kL3; }
}  // namespace cpht
