// Iceberg kernel instantiations for u32 key words.
#include "cpht_iceberg.hpp"
#include "cpht_registry.hpp"

namespace cpht {
namespace {
template <int S0, int S1, int B0, int B1, int G, int MODE, bool L3ON = false>
void launch(const TableK& T, const BatchK& B, hipStream_t s) {
  launch_grid(iceberg_kernel<uint32_t, S0, S1, B0, B1, G, MODE, L3ON>, T, B, s);
}
// The launcher with the third level compiled in, or null where the shape has none.
template <int S0, int S1, int B0, int B1, int G, int MODE>
constexpr launch_fn launch3() {
  if constexpr (L3Shape<S0, G>::OK) return &launch<S0, S1, B0, B1, G, MODE, true>;
  else return nullptr;
}
template <int S0, int S1, int B0, int B1, int G, int MODE>
void launch_multi(const MultiK& M, uint32_t blocks, hipStream_t s) {
  launch_chunks(iceberg_multi_kernel<uint32_t, S0, S1, B0, B1, G, MODE>, M, blocks, s);
}
#define CPHT_ICE_ENTRY(S0, S1, B0, G) \
  {0, S0, S1, B0, B0 / 2, G, (int)L3Shape<S0, G>::OK, &launch<S0, S1, B0, B0 / 2, G, MODE_FIND>, \
   &launch<S0, S1, B0, B0 / 2, G, MODE_INSERT>, &launch<S0, S1, B0, B0 / 2, G, MODE_MIXED>, \
   &launch<S0, S1, B0, B0 / 2, G, MODE_ERASE>, \
   launch3<S0, S1, B0, B0 / 2, G, MODE_FIND>(), launch3<S0, S1, B0, B0 / 2, G, MODE_INSERT>(), \
   launch3<S0, S1, B0, B0 / 2, G, MODE_MIXED>(), launch3<S0, S1, B0, B0 / 2, G, MODE_ERASE>(), \
   &launch_multi<S0, S1, B0, B0 / 2, G, MODE_FIND>, &launch_multi<S0, S1, B0, B0 / 2, G, MODE_INSERT>},
const IceVariant kList[] = {CPHT_ICE_LIST(CPHT_ICE_ENTRY)};
}  // namespace

const IceVariant* ice_variants_u32(int* n) {
  *n = (int)(sizeof(kList) / sizeof(kList[0]));
  return kList;
}
}  // namespace cpht
