// Device-resident request loop for the serving mode of the library: one
// persistent launch keeps working through mixed find / find-or-put requests
// that the host publishes into a ring, without a kernel launch per request.
//
// Shared state:
//   RingCtl (pinned host memory, mapped for the device, coherent): the host
//     writes request descriptors and then advances `published`; the device
//     writes done[slot] = seq + 1 when request seq has completed, and the
//     launch's epoch into `ended` when its leader ends it.  `stop` asks the
//     loop to end.
//   ResidentState (device memory): the leader's copy of the published
//     descriptors and of the published chunk count, the chunk claim counter,
//     per-slot completed-chunk counters and the stop epoch.
//
// Work is cut into chunks of 2^chunk_log2 consecutive operations of one
// request (256 to 2048, the host's choice per request: small chunks spread
// a lone request over many blocks, large ones cut the per-chunk costs when
// much work is in flight); chunk ids are global and increase across requests (request seq
// covers [chunk_base, chunk_base + chunks)).  Block 0 is the leader: it
// polls the host ring, copies new descriptors to device memory (up to 256 at
// once, one per thread) and then publishes their chunks to the workers.
// Every other block takes a ticket (the next chunk id, by an atomic add),
// waits until that chunk is published, processes it with the iceberg
// mixed-batch body, and counts it done; the block that completes a request's
// last chunk reports it to the host.
// Completed-chunk counters never reset: the host gives each descriptor the
// running total its slot must reach (slot_target).
//
// Exit: the leader ends the loop (by writing the launch's epoch to
// stop_epoch) when the host asks, or when neither a new request nor a chunk
// claim has happened for idle_ticks of the device's constant-rate clock;
// workers waiting for an unpublished chunk see the epoch and return, workers
// with a published chunk process it first.  So every wave of the launch ends within
// idle_ticks of the last request (and, should the clock not advance, after
// 2^26 polls without progress).  A waiting worker holds a ticket; at the end
// it gives up a ticket whose chunk is not published, and the next launch's
// leader restarts the ticket count at the last published chunk before any
// worker takes one.  The host launches the loop again when it publishes into
// a loop that has ended (the device counters carry over).
#pragma once
#include <cstddef>

#include "cpht_iceberg.hpp"

namespace cpht {

constexpr uint32_t RING_SLOTS = 1024;      // descriptors in flight at most
constexpr uint32_t CHUNK_MIN_LOG2 = 8;     // operations per chunk: 256 ..
constexpr uint32_t CHUNK_MAX_LOG2 = 11;    // .. 2048, chosen per request by the host

struct RingDesc {
  const void* keys;      // device view of the request's pinned key words
  const uint8_t* ops;    // 0 = find, 1 = find-or-put
  uint8_t* out;          // one answer byte per operation
  uint64_t n;            // operations (> 0)
  uint64_t chunk_base;   // first global chunk id of the request
  uint64_t slot_target;  // completed chunks of this slot when the request is done
  uint64_t seq;          // the request's sequence number (its slot is seq % RING_SLOTS)
  uint32_t chunk_log2;   // the request's chunks hold 2^chunk_log2 operations (the last one fewer)
  uint32_t chunks;       // ceil(n / 2^chunk_log2)
};

struct RingCtl {
  uint64_t published;  // descriptors published by the host (descriptor seq sits at slot seq % RING_SLOTS)
  uint32_t stop;       // host: 1 = end the loop
  uint32_t fault;      // device: 1 = a block found no request for its chunk (the ring protocol was broken)
  uint32_t ended;      // device: epoch of the last launch whose leader has ended it
  uint32_t pad;
  uint64_t done[RING_SLOTS];  // device: seq + 1 once request seq has completed
  RingDesc desc[RING_SLOTS];
};

// Words the workers poll share one 128-byte line; the ticket counter, the
// one word every chunk updates, has a line of its own.
struct ResidentState {
  uint64_t pub_chunks;      // chunk ids [0, pub_chunks) are published to the workers
  uint64_t mirrored;        // descriptors the leader has copied (persists across launches)
  uint32_t stop_epoch;      // epoch of the launch that has been told to end
  uint32_t run_epoch;       // epoch of the launch whose leader has set next_chunk up
  uint64_t pad0[13];
  uint64_t next_chunk;      // next chunk ticket
  uint64_t pad1[15];
  uint64_t slot_done[RING_SLOTS];  // completed chunks per slot (running totals)
  RingDesc desc[RING_SLOTS];       // device copies of the descriptors
};
static_assert(offsetof(ResidentState, next_chunk) == 128 && offsetof(ResidentState, slot_done) == 256,
              "hot words on their own lines");

template <class KeyT, int S0, int S1, int B0, int B1, int G>
__global__ __launch_bounds__(256) void iceberg_resident_kernel(TableK T, RingCtl* ctl, ResidentState* st,
                                                               uint32_t epoch, uint64_t idle_ticks) {
  __shared__ uint64_t s_chunk;
  __shared__ RingDesc s_desc;
  __shared__ int s_cmd;  // 1 process s_chunk, 0 leave the loop

  if (blockIdx.x == 0) {
    // Leader: mirror the host ring into device memory.  Thread 0 polls the
    // published count and the stop word (relaxed loads over the host link,
    // then one system-scope acquire), and the whole block copies up to 256
    // new descriptors at once, one per thread, so a burst of publications
    // costs one round trip over the host link rather than one per request.
    __shared__ uint64_t l_pub, l_mirrored, l_end;
    __shared__ int l_exit;
    uint64_t last_claim = 0, quiet = 0;
    long long t_active = 0;
    if (threadIdx.x == 0) {
      // Tickets the previous launch handed out past its last published chunk
      // were given up unused (see the workers' exit), so numbering restarts
      // there; the workers take no ticket before run_epoch says so.
      const uint64_t pc = __hip_atomic_load(&st->pub_chunks, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&st->next_chunk, pc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&st->run_epoch, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      l_mirrored = st->mirrored;
      last_claim = pc;
      t_active = wall_clock64();
    }
#pragma unroll 1
    for (;;) {
      if (threadIdx.x == 0) {
        const uint64_t pub = __hip_atomic_load(&ctl->published, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        const uint32_t stop = __hip_atomic_load(&ctl->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");  // the descriptors the count covers
        l_pub = pub;
        l_exit = stop != 0u ? 1 : 0;
      }
      __syncthreads();
      const uint64_t pub = l_pub, m = l_mirrored;
      const uint64_t n_copy = pub > m ? (pub - m < 256 ? pub - m : 256) : 0;
      if (threadIdx.x < n_copy) {
        const uint64_t q = m + threadIdx.x;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
        const RingDesc d = ctl->desc[q % RING_SLOTS];
        st->desc[q % RING_SLOTS] = d;
        if (threadIdx.x == n_copy - 1) l_end = d.chunk_base + d.chunks;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // this copy is visible device-wide
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        bool progress = false;
        if (n_copy) {
          st->mirrored = m + n_copy;
          l_mirrored = m + n_copy;
          // the descriptors are in device memory before their chunks are published
          __hip_atomic_store(&st->pub_chunks, l_end, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
          progress = true;
        }
        const uint64_t claim = __hip_atomic_load(&st->next_chunk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (claim != last_claim) {
          last_claim = claim;
          progress = true;
        }
        const long long now = wall_clock64();
        if (progress) {
          t_active = now;
          quiet = 0;
        }
        if (l_exit || (uint64_t)(now - t_active) > idle_ticks || ++quiet > (1ull << 26)) {
          __hip_atomic_store(&st->stop_epoch, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
          // tells the host that publications from now on need a new launch
          __hip_atomic_store(&ctl->ended, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          l_exit = 1;
        }
      }
      __syncthreads();
      if (l_exit) return;
      if (!n_copy) __builtin_amdgcn_s_sleep(8);
    }
  }

  uint64_t seq = 0;  // request of this block's last chunk (thread 0)
  if (threadIdx.x == 0) {
#pragma unroll 1
    while (__hip_atomic_load(&st->run_epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch)
      __builtin_amdgcn_s_sleep(2);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
#pragma unroll 1
  for (;;) {
    if (threadIdx.x == 0) {
      int cmd = 0;
      // A ticket is the id of the chunk this block will process: one atomic
      // add that always succeeds (a compare-and-swap on the shared counter
      // lets one block in, per round trip, of all those trying).  The block
      // then waits until its chunk is published, polling with relaxed loads
      // (an acquire on every poll would invalidate this XCD's L2 under the
      // working blocks) and acquiring once it is.  When the launch is told to
      // end, a ticket that is published by then is still processed; one that
      // is not is given up (the next launch restarts numbering at the last
      // published chunk), so every published chunk is processed exactly once.
      const uint64_t ticket = __hip_atomic_fetch_add(&st->next_chunk, 1ull, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll 1
      for (;;) {
        if (ticket < __hip_atomic_load(&st->pub_chunks, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          cmd = 1;
          break;
        }
        if (__hip_atomic_load(&st->stop_epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch) {
          // the leader's last publication was released before its stop
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          if (ticket < __hip_atomic_load(&st->pub_chunks, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) cmd = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(10);
      }
      if (cmd == 1) {
        // pairs with the leader's release of pub_chunks: the descriptors
        // covering the chunk (and the mirrored count) are visible
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_chunk = ticket;
        // The request holding chunk s_chunk.  It was copied before its chunks
        // were published (the acquire above), it has not completed, and at
        // most RING_SLOTS requests are in flight, so it is one of the last
        // RING_SLOTS copied; chunk ids grow with the request number, and so
        // do this block's claims, so the search starts at the later of this
        // block's previous request and that window, and moves forward.
        const uint64_t m = __hip_atomic_load(&st->mirrored, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (m > RING_SLOTS && seq < m - RING_SLOTS) seq = m - RING_SLOTS;
        const RingDesc* dd = st->desc;
#pragma unroll 1
        for (; seq < m; ++seq) {
          const RingDesc& d = dd[seq % RING_SLOTS];
          if (d.seq == seq && s_chunk >= d.chunk_base && s_chunk < d.chunk_base + d.chunks) break;
        }
        if (seq < m) {
          s_desc = dd[seq % RING_SLOTS];
        } else {
          // cannot happen while the host keeps the ring protocol: report it
          // (the host then fails every request instead of waiting) and end this block
          __hip_atomic_store(&ctl->fault, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
          cmd = 0;
        }
      }
      s_cmd = cmd;
    }
    __syncthreads();
    if (s_cmd == 0) return;
    // see the host's writes of this request's keys and opcodes (acquire, system scope)
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
    const RingDesc d = s_desc;
    const uint64_t first = (s_chunk - d.chunk_base) << d.chunk_log2;
    const uint64_t chunk_keys = 1ull << d.chunk_log2;
    const uint64_t count = d.n - first < chunk_keys ? d.n - first : chunk_keys;
#pragma unroll 1
    for (uint64_t o = 0; o < count; o += 256) {
      BatchK Bt;
      Bt.keys = static_cast<const KeyT*>(d.keys) + first + o;
      Bt.ops = d.ops + first + o;
      Bt.out = d.out + first + o;
      Bt.n = count - o < 256 ? count - o : 256;
      Bt.vin = nullptr;
      Bt.vout = nullptr;
      iceberg_body<KeyT, S0, S1, B0, B1, G, MODE_MIXED, false>(T, Bt, threadIdx.x);
    }
    // this block's answers are visible to the host before the chunk counts as done
    // (release, system scope)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    __syncthreads();
    if (threadIdx.x == 0) {
      const uint64_t slot = d.seq % RING_SLOTS;
      const uint64_t before = __hip_atomic_fetch_add(&st->slot_done[slot], 1ull, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_AGENT);
      if (before + 1 == d.slot_target)  // every block's answers were released before its count
        __hip_atomic_store(&ctl->done[slot], d.seq + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    __syncthreads();
  }
}

}  // namespace cpht
