// Instantiations of the serving loop's persistent kernel (cpht_resident.hpp)
// for every iceberg variant and both key word widths.
#include "cpht_registry.hpp"
#include "cpht_resident.hpp"

namespace cpht {
namespace {
template <class KeyT, int S0, int S1, int B0, int G>
hipError_t launch_resident(const TableK& T, RingCtl* ctl, ResidentState* st, uint32_t epoch, uint64_t idle_ticks,
                           uint32_t blocks, hipStream_t s) {
  hipLaunchKernelGGL((iceberg_resident_kernel<KeyT, S0, S1, B0, B0 / 2, G>), dim3(blocks), dim3(256), 0, s, T, ctl,
                     st, epoch, idle_ticks);
  return hipGetLastError();
}
#define CPHT_ICE_RES32(S0, S1, B0, G) &launch_resident<uint32_t, S0, S1, B0, G>,
#define CPHT_ICE_RES64(S0, S1, B0, G) &launch_resident<uint64_t, S0, S1, B0, G>,
const resident_fn kRes32[] = {CPHT_ICE_LIST(CPHT_ICE_RES32)};
const resident_fn kRes64[] = {CPHT_ICE_LIST(CPHT_ICE_RES64)};
}  // namespace

const resident_fn* ice_resident_u32() { return kRes32; }
const resident_fn* ice_resident_u64() { return kRes64; }
}  // namespace cpht
