// Host-side simulation of the request server's admission policy
// (paper_2505_04431_amd/csrc/kc_sched.h) with a simulated clock and
// simulated memory: no device, no threads. Reads
//   budget workers max_bypass n
//   then n lines: arrival duration scratch result_est result_actual hold
// and prints one line per job: id start end worker, then "peak <bytes>".
// A job holds its scratch only while it runs (the server cuts one block per
// job from its slab and takes it back when the job ends); a result is held
// from the job's end until end + hold. A negative hold models a client that
// waits for the jobs in submission order and releases each result once it
// has waited for it: when the server reports that the queue is stalled on
// held results (kc_server_wait's KC_E_NOMEM), that client releases every
// result it holds. The last line is "stalls <reports>".
#include <cstdio>
#include <deque>
#include <map>
#include <vector>

#include "kc_sched.h"

struct SimJob {
  double arrival, duration, hold;
  uint64_t scratch, est, actual;
  double start = -1, end = -1;
  int worker = -1;
};

int main() {
  uint64_t budget;
  int workers;
  unsigned max_bypass;
  int n;
  if (std::scanf("%llu %d %u %d", (unsigned long long*)&budget, &workers, &max_bypass, &n) != 4)
    return 2;
  std::vector<SimJob> jobs(n);
  for (auto& j : jobs)
    if (std::scanf("%lf %lf %llu %llu %llu %lf", &j.arrival, &j.duration,
                   (unsigned long long*)&j.scratch, (unsigned long long*)&j.est,
                   (unsigned long long*)&j.actual, &j.hold) != 6)
      return 2;
  kc::Ledger L;
  L.budget = budget;
  std::deque<kc::QueuedJob> q;
  std::vector<int> busy(workers, -1);
  std::multimap<double, int> ends, releases;  // time -> job
  size_t next_arrival = 0;
  int done = 0;
  int consumed = 0;  // in-order client: jobs [0, consumed) waited for and released
  int stalls = 0;
  std::vector<int> held;  // finished jobs with negative hold, not yet released
  double now = 0;
  uint64_t reserved_running[64] = {};
  while (done < n) {
    // next event: arrival, end or release
    double t = 1e300;
    if (next_arrival < jobs.size()) t = jobs[next_arrival].arrival;
    if (!ends.empty()) t = std::min(t, ends.begin()->first);
    if (!releases.empty()) t = std::min(t, releases.begin()->first);
    if (t == 1e300) {
      // nothing pending but queued jobs: the server reports the stall to a
      // client waiting on one of them; the client releases what it holds
      const bool stalled = kc::stalled_on_results(
          q, L.free_bytes(), max_bypass, 0, 0,
          [&](const kc::QueuedJob& x) { return jobs[x.id].scratch + x.result_est; });
      if (!stalled || held.empty()) {
        std::printf("stuck %zu\n", q.size());
        return 1;
      }
      ++stalls;
      for (int id : held) L.sub(jobs[id].actual);
      held.clear();
      t = now;
    }
    now = t;
    while (!releases.empty() && releases.begin()->first <= now) {
      L.sub(jobs[releases.begin()->second].actual);
      releases.erase(releases.begin());
    }
    while (!ends.empty() && ends.begin()->first <= now) {
      const int id = ends.begin()->second;
      ends.erase(ends.begin());
      SimJob& j = jobs[id];
      j.end = now;
      const int w = j.worker;
      L.sub(reserved_running[w]);  // its scratch and its reservation
      reserved_running[w] = 0;
      L.add(j.actual);
      if (j.hold >= 0) releases.emplace(now + j.hold, id);
      else held.push_back(id);
      busy[w] = -1;
      ++done;
    }
    // the in-order client releases the held results it has reached
    for (;;) {
      bool moved = false;
      for (size_t i = 0; i < held.size(); ++i)
        if (held[i] == consumed) {
          L.sub(jobs[held[i]].actual);
          held.erase(held.begin() + i);
          ++consumed;
          moved = true;
          break;
        }
      if (!moved) {
        if (consumed < n && jobs[consumed].end >= 0 && jobs[consumed].hold >= 0) {
          ++consumed;  // released by time, not by the client
          continue;
        }
        break;
      }
    }
    while (next_arrival < jobs.size() && jobs[next_arrival].arrival <= now) {
      kc::QueuedJob qj;
      qj.id = next_arrival;
      qj.result_est = jobs[next_arrival].est;
      q.push_back(qj);
      ++next_arrival;
    }
    // every idle worker tries to start a job (lowest index first)
    bool progress = true;
    while (progress) {
      progress = false;
      int running = 0;
      for (int w = 0; w < workers; ++w) running += busy[w] >= 0;
      for (int w = 0; w < workers; ++w) {
        if (busy[w] >= 0) continue;
        const long i = kc::pick_job(q, L.free_bytes(), max_bypass, [&](const kc::QueuedJob& x) {
          return jobs[x.id].scratch + x.result_est;
        });
        if (i >= 0) {
          const int id = (int)q[(size_t)i].id;
          q.erase(q.begin() + i);
          SimJob& j = jobs[id];
          reserved_running[w] = j.scratch + j.est;
          L.add(reserved_running[w]);
          j.start = now;
          j.worker = w;
          busy[w] = id;
          ends.emplace(now + j.duration, id);
          progress = true;
          ++running;
        }
      }
    }
  }
  for (int i = 0; i < n; ++i)
    std::printf("%d %.6f %.6f %d\n", i, jobs[i].start, jobs[i].start + jobs[i].duration,
                jobs[i].worker);
  std::printf("peak %llu\n", (unsigned long long)L.peak);
  std::printf("stalls %d\n", stalls);
  return 0;
}
