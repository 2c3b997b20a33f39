// Bounded table of request records for the serving loop, indexed by ticket.
//
// Tickets count up from 0.  The table keeps the records of tickets [base,
// next) in order.  A record leaves the table from the front once its
// request has completed and either its ticket has been collected (waited on,
// or polled as done) or at least `keep` later tickets were issued; so memory
// stays bounded by the requests still pending plus `keep`, whatever the
// caller collects.  A ticket below base is expired: lookups return null.
// Host code only (no device types), so it can be compiled and tested alone.
#pragma once
#include <cstdint>
#include <deque>

namespace cpht {

template <class Rec>
class TicketTable {
 public:
  explicit TicketTable(uint64_t keep) : keep_(keep) {}

  uint64_t next() const { return base_ + recs_.size(); }
  uint64_t base() const { return base_; }
  uint64_t size() const { return recs_.size(); }

  // Append a record; returns its ticket.  References to other records stay
  // valid (a deque does not move its elements on push_back / pop_front).
  uint64_t add(const Rec& r) {
    recs_.push_back(Entry{r, false});
    return next() - 1;
  }

  // The record of `ticket`, or nullptr if it expired or was never issued.
  Rec* find(uint64_t ticket) {
    if (ticket < base_ || ticket >= next()) return nullptr;
    return &recs_[ticket - base_].rec;
  }

  // The caller has seen `ticket` complete; its record may be released.
  void collect(uint64_t ticket) {
    if (ticket >= base_ && ticket < next()) recs_[ticket - base_].collected = true;
  }

  // Release records from the front while their request is done (done(rec))
  // and they are collected or old enough.
  template <class Done>
  void trim(Done done) {
    while (!recs_.empty()) {
      const Entry& e = recs_.front();
      if (!done(e.rec) || !(e.collected || next() - base_ > keep_)) break;
      recs_.pop_front();
      ++base_;
    }
  }

 private:
  struct Entry {
    Rec rec;
    bool collected;
  };
  std::deque<Entry> recs_;
  uint64_t base_ = 0;
  uint64_t keep_;
};

}  // namespace cpht
