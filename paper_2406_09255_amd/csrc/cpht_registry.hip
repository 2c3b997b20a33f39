// Assembles the iceberg variant records from the launcher tables of the
// instantiation files (one entry per CPHT_ICE_LIST position in each).
#include "cpht_iceberg.hpp"
#include "cpht_registry.hpp"

namespace cpht {
namespace {

struct Shape {
  int S0, S1, B0, G;
};
#define CPHT_ICE_SHAPE(S0, S1, B0, G) {S0, S1, B0, G},
const Shape kShapes[] = {CPHT_ICE_LIST(CPHT_ICE_SHAPE)};
constexpr int kCount = (int)(sizeof(kShapes) / sizeof(kShapes[0]));

template <int S0, int G>
constexpr int l3_ok() { return L3Shape<S0, G>::OK ? 1 : 0; }
#define CPHT_ICE_L3OK(S0, S1, B0, G) l3_ok<S0, G>(),
const int kL3Ok[] = {CPHT_ICE_LIST(CPHT_ICE_L3OK)};

void assemble(IceVariant* out, int key64, const IceLaunch4* base, const IceMulti2* multi, const IceLaunch4* l3,
              const IceLaunch4* map, const resident_fn* resident) {
  for (int i = 0; i < kCount; ++i) {
    IceVariant& v = out[i];
    v.key64 = key64;
    v.S0 = kShapes[i].S0;
    v.S1 = kShapes[i].S1;
    v.B0 = kShapes[i].B0;
    v.B1 = kShapes[i].B0 / 2;
    v.G = kShapes[i].G;
    v.l3 = kL3Ok[i];
    v.find = base[i].a;
    v.insert = base[i].b;
    v.mixed = base[i].c;
    v.erase = base[i].d;
    v.find3 = l3[i].a;
    v.insert3 = l3[i].b;
    v.mixed3 = l3[i].c;
    v.erase3 = l3[i].d;
    v.find_v = map[i].a;
    v.insert_v = map[i].b;
    v.find_v3 = map[i].c;
    v.insert_v3 = map[i].d;
    v.multi_find = multi[i].find;
    v.multi_insert = multi[i].insert;
    v.resident = resident[i];
  }
}

struct Tables {
  IceVariant u32[kCount];
  IceVariant u64[kCount];
  Tables() {
    assemble(u32, 0, ice_base_u32(), ice_multi_u32(), ice_l3_u32(), ice_map_u32(), ice_resident_u32());
    assemble(u64, 1, ice_base_u64(), ice_multi_u64(), ice_l3_u64(), ice_map_u64(), ice_resident_u64());
  }
};

const Tables& tables() {
  static const Tables t;  // built on first use (after every static table above)
  return t;
}

}  // namespace

const IceVariant* ice_variants_u32(int* n) {
  *n = kCount;
  return tables().u32;
}

const IceVariant* ice_variants_u64(int* n) {
  *n = kCount;
  return tables().u64;
}

}  // namespace cpht
