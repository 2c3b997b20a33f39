// Host-only checks of the serving loop's ticket table (cpht_tickets.hpp):
// records are released once done and collected, or once `keep` later tickets
// exist, so memory stays bounded however many requests are submitted; a
// pending record at the front holds back its successors until it completes.
#include <cstdio>
#include <cstdlib>

#include "cpht_tickets.hpp"

struct Rec {
  uint64_t id;
  bool done;
};

#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::fprintf(stderr, "line %d: check failed: %s\n", __LINE__, #c); \
      return 1;                                                    \
    }                                                              \
  } while (0)

static bool done(const Rec& r) { return r.done; }

int main() {
  const uint64_t keep = 1000;
  // 1. many more requests than `keep`, completed but never collected
  {
    cpht::TicketTable<Rec> t(keep);
    for (uint64_t i = 0; i < 3 * 1000 * 1000; ++i) {
      const uint64_t tk = t.add(Rec{i, true});
      CHECK(tk == i);
      t.trim(done);
      CHECK(t.size() <= keep + 1);
    }
    CHECK(t.next() == 3 * 1000 * 1000);
    CHECK(t.find(0) == nullptr);                    // expired
    CHECK(t.find(t.next()) == nullptr);             // never issued
    CHECK(t.find(t.next() - 1)->id == t.next() - 1);
  }
  // 2. collected records leave at once; records keep their identity
  {
    cpht::TicketTable<Rec> t(keep);
    for (uint64_t i = 0; i < 10; ++i) t.add(Rec{i, false});
    Rec* r5 = t.find(5);
    for (uint64_t i = 0; i < 10; ++i) t.find(i)->done = true;
    t.collect(0);
    t.collect(1);
    t.collect(3);
    t.trim(done);
    CHECK(t.base() == 2);                           // 2 is not collected: 3 stays behind it
    CHECK(t.find(1) == nullptr && t.find(3) != nullptr);
    CHECK(t.find(5) == r5 && r5->id == 5);          // references survive trimming
    t.collect(2);
    t.trim(done);
    CHECK(t.base() == 4);
  }
  // 3. a pending request at the front holds back done, uncollected ones,
  //    which all go once it completes and is collected
  {
    cpht::TicketTable<Rec> t(keep);
    t.add(Rec{0, false});
    for (uint64_t i = 1; i < 5000; ++i) {
      t.add(Rec{i, true});
      t.trim(done);
    }
    CHECK(t.size() == 5000);
    CHECK(t.find(0) != nullptr && t.find(4999) != nullptr);
    t.find(0)->done = true;
    t.trim(done);
    CHECK(t.size() == keep);                        // old enough: only the last `keep` remain
    t.collect(t.base());
    t.trim(done);
    CHECK(t.size() == keep - 1);
  }
  std::printf("ticket table ok\n");
  return 0;
}
