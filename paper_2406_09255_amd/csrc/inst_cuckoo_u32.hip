// Cuckoo kernel instantiations for u32 key words.
#include "cpht_cuckoo.hpp"
#include "cpht_registry.hpp"

namespace cpht {
namespace {
template <int S, int B, int G, int OP>
void launch(const TableK& T, const BatchK& Bt, hipStream_t s) {
  launch_grid(cuckoo_kernel<uint32_t, S, B, G, OP>, T, Bt, s);
}
template <int S, int B, int G, int OP>
void launch_multi(const MultiK& M, uint32_t blocks, hipStream_t s) {
  launch_chunks(cuckoo_multi_kernel<uint32_t, S, B, G, OP>, M, blocks, s);
}
#define CPHT_CK_ENTRY(S, B, G) \
  {0, S, B, G, &launch<S, B, G, CK_PUT>, &launch<S, B, G, CK_FIND>, &launch<S, B, G, CK_ERASE>, \
   &launch_multi<S, B, G, CK_PUT>, &launch_multi<S, B, G, CK_FIND>},
const CkVariant kList[] = {CPHT_CK_LIST(CPHT_CK_ENTRY)};
}  // namespace

const CkVariant* ck_variants_u32(int* n) {
  *n = (int)(sizeof(kList) / sizeof(kList[0]));
  return kList;
}
}  // namespace cpht
