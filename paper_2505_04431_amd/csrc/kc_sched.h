// Admission policy of the request server: which queued job a free worker
// starts, and the account of device bytes against the budget. Pure host
// logic (no HIP), shared by the server and its host-side simulation test.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <deque>

namespace kc {

struct QueuedJob {
  uint64_t id = 0;
  uint64_t n_bytes = 0;     // input bytes
  int k = 0, P = 0;
  uint64_t result_est = 0;  // bytes reserved for its result until the true size is known
  uint32_t bypassed = 0;    // times a later job was started before it
  // the server's memory epoch at which no free range could hold the job's
  // scratch block; it is not tried again before the epoch changes
  uint64_t unplaced_epoch = ~0ull;
};

// Device bytes the server has promised: scratch arenas, results held on the
// device and reservations of running jobs.
struct Ledger {
  uint64_t budget = 0, in_use = 0, peak = 0;
  void add(uint64_t b) {
    in_use += b;
    peak = std::max(peak, in_use);
  }
  void sub(uint64_t b) { in_use -= std::min(b, in_use); }
  uint64_t free_bytes() const { return in_use >= budget ? 0 : budget - in_use; }
};

// The queued job to start next, or -1: the first job in arrival order whose
// need (bytes it would add to the ledger when started now) fits in
// free_bytes. A job passed over max_bypass times blocks all later jobs until
// it fits itself, so a large job waits at most max_bypass starts before memory
// is kept for it. peek_job only looks; pick_job also marks the jobs passed
// over as bypassed.
template <class Need>
long peek_job(const std::deque<QueuedJob>& q, uint64_t free_bytes, uint32_t max_bypass,
              Need&& need) {
  for (size_t i = 0; i < q.size(); ++i) {
    if (need(q[i]) <= free_bytes) return (long)i;
    if (q[i].bypassed >= max_bypass) return -1;
  }
  return -1;
}

template <class Need>
long pick_job(std::deque<QueuedJob>& q, uint64_t free_bytes, uint32_t max_bypass, Need&& need) {
  const long i = peek_job(q, free_bytes, max_bypass, need);
  for (long j = 0; j < i; ++j) ++q[(size_t)j].bypassed;
  return i;
}

// True when no queued job can start until the client releases results it
// holds: nothing is running, every worker has given its scratch back, and
// still no queued job is admitted (what the budget has left after the held
// results is too small). A wait on a queued job then reports KC_E_NOMEM
// instead of blocking for ever.
template <class Need>
bool stalled_on_results(const std::deque<QueuedJob>& q, uint64_t free_bytes, uint32_t max_bypass,
                        uint64_t running, uint64_t arena_total, Need&& need) {
  return !q.empty() && running == 0 && arena_total == 0 &&
         peek_job(q, free_bytes, max_bypass, need) < 0;
}

}  // namespace kc
