// Request server behind the kc_server_* entry points of include/kc.h.
//
// Jobs are plain counts submitted with device-resident inputs. A fixed pool
// of worker threads, each with its own non-blocking HIP stream, takes jobs
// from one queue: a worker starts the first queued job whose device bytes
// (its scratch block plus a reservation for its result) fit under the budget
// (policy in kc_sched.h), so jobs of different sizes run side by side on the
// device and a finished job's slot is refilled at once. Results are allocated
// at their exact size once the number of distinct keys is known and stay on
// the device until released. All of the server's device memory is one slab
// mapped when it is created; each job's scratch block (returned when the job
// ends) and each result are cut from it, so serving maps and unmaps nothing
// (a device free waits for every stream of the device, and mapping fresh
// memory while jobs ran stalled every worker).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <system_error>
#include <thread>
#include <vector>

#include "../../include/kc.h"
#include "kc_host.h"
#include "kc_sched.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Job {
  uint64_t id = 0;
  const uint8_t* reads = nullptr;
  const uint64_t* offsets = nullptr;
  uint64_t n_reads = 0;
  int k = 0, P = 0;
  uint64_t n_bytes = 0;
  uint64_t result_est = 0;
  uint64_t reserved = 0;  // bytes charged to the ledger while running
  int state = KC_JOB_QUEUED;
  int status = KC_OK;
  std::string err;
  int worker = -1;
  uint64_t* keys = nullptr;
  uint32_t* counts = nullptr;
  uint64_t n_out = 0, result_bytes = 0, windows = 0;
  Clock::time_point t_submit, t_start, t_end;
};

// Output allocation of one running job: one block of the server's slab
// (keys, then counts), cut from the slab's high end.
struct JobAlloc {
  Job* job;
  kc::Slab* slab;
};

int alloc_result(void* user, uint64_t distinct, int key_words, uint64_t** keys, uint32_t** counts) {
  JobAlloc* a = (JobAlloc*)user;
  *keys = nullptr;
  *counts = nullptr;
  if (distinct == 0) return KC_OK;
  const uint64_t kbytes = (distinct * 8 * (uint64_t)key_words + 255) & ~255ull;
  char* p = (char*)a->slab->alloc(kbytes + distinct * 4, true);
  if (!p) return KC_E_NOMEM;
  a->job->keys = (uint64_t*)p;
  a->job->counts = (uint32_t*)(p + kbytes);
  a->job->result_bytes = distinct * (8 * (uint64_t)key_words + 4);  // (plus < 256 bytes of alignment)
  *keys = a->job->keys;
  *counts = a->job->counts;
  return KC_OK;
}

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  // nearest rank
  size_t r = (size_t)std::ceil(q * (double)v.size());
  r = std::min(std::max<size_t>(r, 1), v.size());
  return v[r - 1];
}

}  // namespace

struct kc_server {
  int device = 0;
  int n_workers = 0;
  uint32_t max_bypass = 8;
  kc_options opt{};
  Clock::time_point t0;

  std::mutex m;
  std::condition_variable cv_work, cv_done;
  std::deque<kc::QueuedJob> queue;
  std::map<uint64_t, std::unique_ptr<Job>> jobs;
  kc::Ledger ledger;
  std::vector<kc::WorkerArena*> wctx;  // each worker's count context
  kc::Slab* slab = nullptr;     // all device memory of the server
  uint64_t epoch = 0;           // advanced whenever slab memory is given back
  uint64_t next_id = 1;
  bool stop = false;
  uint64_t submitted = 0, completed = 0, failed = 0, running = 0, windows = 0;
  uint64_t est_misses = 0, reserved_total = 0, actual_total = 0, unplaced = 0;
  bool any_start = false;
  Clock::time_point first_start, last_end;
  std::vector<double> lat_ms, wait_ms;

  std::mutex submit_m;  // the control stream and its pinned staging
  hipStream_t ctl = nullptr;
  uint64_t* pinned = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<std::thread> threads;

  void worker_main(int w);
  void finish_locked(Job* j, int w, uint64_t new_arena);
  // Bytes a queued job would add to the ledger if started now: its scratch
  // block and its result reservation; more than any budget while no free
  // range of the slab could hold its block and no memory has come back since.
  uint64_t need_of(const kc::QueuedJob& q) const {
    if (q.unplaced_epoch == epoch) return ~0ull;
    return kc::scratch_bytes(q.n_bytes, q.k, q.P, &opt) + q.result_est;
  }
  bool stalled_locked() const {
    return kc::stalled_on_results(queue, ledger.free_bytes(), max_bypass, running, 0,
                                  [&](const kc::QueuedJob& q) { return need_of(q); });
  }
};

void kc_server::worker_main(int w) {
  if (hipSetDevice(device) != hipSuccess) return;
  const hipStream_t st = streams[w];
  for (;;) {
    Job* job = nullptr;
    void* block = nullptr;
    uint64_t block_bytes = 0;
    {
      std::unique_lock<std::mutex> lk(m);
      for (;;) {
        if (stop) break;
        const long idx = kc::pick_job(queue, ledger.free_bytes(), max_bypass,
                                      [&](const kc::QueuedJob& q) { return need_of(q); });
        if (idx >= 0) {
          kc::QueuedJob& q = queue[(size_t)idx];
          // the job's scratch: one block of the slab, for this job only
          block_bytes = kc::scratch_bytes(q.n_bytes, q.k, q.P, &opt);
          block = block_bytes ? slab->alloc(block_bytes, false) : nullptr;
          if (block_bytes && !block) {
            // the budget has room but no free range is large enough: the job
            // stays queued until memory comes back (a job ends or a result is
            // released)
            q.unplaced_epoch = epoch;
            ++unplaced;
            cv_done.notify_all();  // a waiter may now find the queue stalled
            continue;
          }
          const kc::QueuedJob qj = q;
          queue.erase(queue.begin() + idx);
          job = jobs.at(qj.id).get();
          job->reserved = block_bytes + qj.result_est;
          ledger.add(job->reserved);
          job->state = KC_JOB_RUNNING;
          job->worker = w;
          job->t_start = Clock::now();
          if (!any_start) {
            first_start = job->t_start;
            any_start = true;
          }
          ++running;
          break;
        }
        cv_work.wait(lk);
      }
      if (!job) return;
    }
    JobAlloc a{job, slab};
    kc::OutAlloc oa{alloc_result, &a};
    kc_stats S;
    std::memset(&S, 0, sizeof(S));
    uint64_t n_out = 0;
    std::string err;
    int r = kc::count_in_block(wctx[w], block, block_bytes, slab, job->reads, job->offsets,
                               job->n_reads, job->k, job->P, &opt, st, oa, &n_out, &S, &err);
    if (r != KC_OK && job->keys) {
      slab->free(job->keys, st);
      job->keys = nullptr;
      job->counts = nullptr;
      job->result_bytes = 0;
    }
    if (block) slab->free(block, st);  // the count has synchronized its stream
    std::lock_guard<std::mutex> lk(m);
    job->status = r;
    job->err = err;
    job->n_out = r == KC_OK ? n_out : 0;
    job->windows = r == KC_OK ? S.valid_windows : 0;
    finish_locked(job, w, 0);
  }
}

void kc_server::finish_locked(Job* j, int, uint64_t) {
  ledger.sub(j->reserved);  // its scratch block and reservation
  j->reserved = 0;
  ++epoch;                  // its block is back in the slab
  ledger.add(j->result_bytes);
  reserved_total += j->result_est;
  actual_total += j->result_bytes;
  if (j->result_bytes > j->result_est) ++est_misses;
  j->t_end = Clock::now();
  last_end = j->t_end;
  --running;
  if (j->status == KC_OK) {
    j->state = KC_JOB_DONE;
    ++completed;
    windows += j->windows;
    lat_ms.push_back(ms_between(j->t_submit, j->t_end));
    wait_ms.push_back(ms_between(j->t_submit, j->t_start));
  } else {
    j->state = KC_JOB_FAILED;
    ++failed;
  }
  cv_work.notify_all();
  cv_done.notify_all();
}

namespace {

template <class F>
int server_guard(F f) {
  kc::set_last_error("");
  try {
    return f();
  } catch (const std::bad_alloc&) {
    kc::set_last_error("host allocation failed");
    return KC_E_NOMEM;
  } catch (const std::system_error& e) {
    kc::set_last_error(e.what());
    return KC_E_INTERNAL;
  } catch (...) {
    kc::set_last_error("unexpected C++ exception");
    return KC_E_INTERNAL;
  }
}

int set_err(int code, const std::string& msg) {
  kc::set_last_error(msg);
  return code;
}

void destroy_server(kc_server* s) {
  {
    std::lock_guard<std::mutex> lk(s->m);
    s->stop = true;
    s->cv_work.notify_all();
  }
  for (std::thread& t : s->threads)
    if (t.joinable()) t.join();
  (void)hipSetDevice(s->device);
  for (hipStream_t st : s->streams)
    if (st) (void)hipStreamSynchronize(st);
  for (kc::WorkerArena* wa : s->wctx) kc::worker_arena_destroy(wa);
  for (hipStream_t st : s->streams)
    if (st) (void)hipStreamDestroy(st);
  if (s->ctl) (void)hipStreamDestroy(s->ctl);
  if (s->pinned) (void)hipHostFree(s->pinned);
  // the results and the workers' blocks go with the slab
  delete s->slab;
  delete s;
}

}  // namespace

extern "C" {

int kc_server_create(uint64_t hbm_budget_bytes, int n_workers, const kc_options* opt,
                     kc_server** out) {
  return server_guard([&]() -> int {
    if (!out) return set_err(KC_E_INVAL, "server handle pointer is NULL");
    *out = nullptr;
    if (hbm_budget_bytes == 0) return set_err(KC_E_INVAL, "budget must be > 0");
    if (n_workers < 1 || n_workers > 16) return set_err(KC_E_INVAL, "workers must be in [1, 16]");
    if (opt && opt->mode != 0 && opt->mode != 1) return set_err(KC_E_INVAL, "mode must be 0 or 1");
    std::unique_ptr<kc_server> s(new kc_server());
    if (hipGetDevice(&s->device) != hipSuccess) return set_err(KC_E_DEVICE, "hipGetDevice failed");
    if (opt) s->opt = *opt;
    s->n_workers = n_workers;
    s->t0 = Clock::now();
    // all device memory of the server, mapped now: the budget, or what the
    // device has free less a margin for the rest of the process
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
      (void)hipGetLastError();
      return set_err(KC_E_DEVICE, "hipMemGetInfo failed");
    }
    const uint64_t margin = std::max<uint64_t>(2ull << 30, total_b / 50);
    const uint64_t room = free_b > margin ? free_b - margin : 0;
    const uint64_t slab_bytes = std::min<uint64_t>(hbm_budget_bytes, room);
    std::string err;
    if (slab_bytes < 4096 || !(s->slab = kc::Slab::create(slab_bytes, &err)))
      return set_err(KC_E_NOMEM, err.empty() ? "too little free device memory for a server"
                                             : err);
    s->ledger.budget = s->slab->capacity();
    for (int w = 0; w < n_workers; ++w) {
      s->wctx.push_back(kc::worker_arena_create(s->device));
      if (!s->wctx.back()) {
        kc_server* raw = s.release();
        destroy_server(raw);
        return set_err(KC_E_NOMEM, "worker context creation failed");
      }
    }
    if (hipStreamCreateWithFlags(&s->ctl, hipStreamNonBlocking) != hipSuccess ||
        hipHostMalloc((void**)&s->pinned, 64, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      kc_server* raw = s.release();
      destroy_server(raw);
      return set_err(KC_E_DEVICE, "stream or pinned buffer creation failed");
    }
    s->streams.assign(n_workers, nullptr);
    for (int w = 0; w < n_workers; ++w) {
      if (hipStreamCreateWithFlags(&s->streams[w], hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        kc_server* raw = s.release();
        destroy_server(raw);
        return set_err(KC_E_DEVICE, "worker stream creation failed");
      }
    }
    kc_server* raw = s.release();
    for (int w = 0; w < n_workers; ++w) raw->threads.emplace_back([raw, w] { raw->worker_main(w); });
    *out = raw;
    return KC_OK;
  });
}

int kc_server_submit(kc_server* s, const uint8_t* reads, const uint64_t* offsets,
                     uint64_t n_reads, int k, int P, uint64_t distinct_hint, uint64_t* job_id) {
  return server_guard([&]() -> int {
    if (!s || !job_id) return set_err(KC_E_INVAL, "server or job id pointer is NULL");
    *job_id = 0;
    if (k < 1 || k > 128) return set_err(KC_E_INVAL, "k must be in [1, 128]");
    if (P < 1) return set_err(KC_E_INVAL, "P must be >= 1");
    if (!offsets) return set_err(KC_E_INVAL, "offsets is NULL");
    if (n_reads && !reads) return set_err(KC_E_INVAL, "reads is NULL");
    uint64_t off0 = 0, offn = 0;
    {
      std::lock_guard<std::mutex> lk(s->submit_m);
      if (hipSetDevice(s->device) != hipSuccess ||
          hipMemcpyAsync(s->pinned, offsets, 8, hipMemcpyDeviceToHost, s->ctl) != hipSuccess ||
          hipMemcpyAsync(s->pinned + 1, offsets + n_reads, 8, hipMemcpyDeviceToHost, s->ctl) !=
              hipSuccess ||
          hipStreamSynchronize(s->ctl) != hipSuccess) {
        const hipError_t e = hipGetLastError();
        return set_err(KC_E_DEVICE, std::string("reading the offsets failed: ") +
                                        hipGetErrorString(e));
      }
      off0 = s->pinned[0];
      offn = s->pinned[1];
    }
    if (offn < off0) return set_err(KC_E_INVAL, "offsets must be non-decreasing");
    const uint64_t n_bytes = offn - off0;
    const uint64_t pair = 8 * (uint64_t)(k <= 32 ? 1 : k <= 64 ? 2 : 4) + 4;
    // the number of windows bounds the distinct keys; a hint replaces the bound
    const uint64_t bound = n_bytes * pair;
    const uint64_t est = distinct_hint ? std::min(bound, distinct_hint * pair) : bound;
    const uint64_t need = kc::scratch_bytes(n_bytes, k, P, &s->opt) + est;
    if (need > s->ledger.budget)
      return set_err(KC_E_NOMEM, "job needs about " + std::to_string(need) +
                                     " device bytes, more than the server budget of " +
                                     std::to_string(s->ledger.budget));
    std::unique_ptr<Job> j(new Job());
    j->reads = reads;
    j->offsets = offsets;
    j->n_reads = n_reads;
    j->k = k;
    j->P = P;
    j->n_bytes = n_bytes;
    j->result_est = est;
    std::lock_guard<std::mutex> lk(s->m);
    if (s->stop) return set_err(KC_E_INVAL, "server is shutting down");
    j->id = s->next_id++;
    j->t_submit = Clock::now();
    kc::QueuedJob q;
    q.id = j->id;
    q.n_bytes = n_bytes;
    q.k = k;
    q.P = P;
    q.result_est = est;
    *job_id = j->id;
    s->jobs[j->id] = std::move(j);
    s->queue.push_back(q);
    ++s->submitted;
    s->cv_work.notify_all();
    return KC_OK;
  });
}

int kc_server_poll(kc_server* s, uint64_t job_id, int* state) {
  return server_guard([&]() -> int {
    if (!s || !state) return set_err(KC_E_INVAL, "server or state pointer is NULL");
    std::lock_guard<std::mutex> lk(s->m);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return set_err(KC_E_INVAL, "unknown job id");
    *state = it->second->state;
    return KC_OK;
  });
}

int kc_server_wait(kc_server* s, uint64_t job_id, int* state) {
  return server_guard([&]() -> int {
    if (!s) return set_err(KC_E_INVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(s->m);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return set_err(KC_E_INVAL, "unknown job id");
    Job* j = it->second.get();
    while (j->state != KC_JOB_DONE && j->state != KC_JOB_FAILED) {
      if (j->state == KC_JOB_QUEUED && s->stalled_locked()) {
        if (state) *state = j->state;
        return set_err(KC_E_NOMEM,
                       "job " + std::to_string(job_id) + " cannot start: results held on the "
                       "device (" + std::to_string(s->ledger.in_use) + " of the " +
                       std::to_string(s->ledger.budget) + " budget bytes) leave too little for "
                       "the queued jobs; release results, then wait again");
      }
      s->cv_done.wait(lk);
    }
    if (state) *state = j->state;
    return KC_OK;
  });
}

int kc_server_result(kc_server* s, uint64_t job_id, const uint64_t** keys, const uint32_t** counts,
                     uint64_t* n_out) {
  return server_guard([&]() -> int {
    if (!s || !keys || !counts || !n_out) return set_err(KC_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->m);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return set_err(KC_E_INVAL, "unknown job id");
    Job* j = it->second.get();
    if (j->state == KC_JOB_FAILED) return set_err(j->status, j->err);
    if (j->state != KC_JOB_DONE) return set_err(KC_E_INVAL, "job has not finished");
    *keys = j->keys;
    *counts = j->counts;
    *n_out = j->n_out;
    return KC_OK;
  });
}

int kc_server_result_copy(kc_server* s, uint64_t job_id, uint64_t* out_keys,
                          uint32_t* out_counts, uint64_t out_capacity, uint64_t* n_out,
                          void* stream) {
  return server_guard([&]() -> int {
    if (!s || !n_out) return set_err(KC_E_INVAL, "NULL argument");
    *n_out = 0;
    const uint64_t* keys = nullptr;
    const uint32_t* counts = nullptr;
    uint64_t n = 0;
    int words = 1;
    {
      std::lock_guard<std::mutex> lk(s->m);
      auto it = s->jobs.find(job_id);
      if (it == s->jobs.end()) return set_err(KC_E_INVAL, "unknown job id");
      const Job* j = it->second.get();
      if (j->state == KC_JOB_FAILED) return set_err(j->status, j->err);
      if (j->state != KC_JOB_DONE) return set_err(KC_E_INVAL, "job has not finished");
      keys = j->keys;
      counts = j->counts;
      n = j->n_out;
      words = j->k <= 32 ? 1 : (j->k <= 64 ? 2 : 4);
    }
    *n_out = n;
    if (n > out_capacity) return set_err(KC_E_CAPACITY, "output capacity too small");
    if (n == 0) return KC_OK;
    if (!out_keys || !out_counts) return set_err(KC_E_INVAL, "output pointer is NULL");
    const hipStream_t st = (hipStream_t)stream;
    if (hipMemcpyAsync(out_keys, keys, n * 8 * (uint64_t)words, hipMemcpyDeviceToDevice, st) !=
            hipSuccess ||
        hipMemcpyAsync(out_counts, counts, n * 4, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      const hipError_t e = hipGetLastError();
      return set_err(KC_E_DEVICE, std::string("result copy failed: ") + hipGetErrorString(e));
    }
    return KC_OK;
  });
}

int kc_server_job_info(kc_server* s, uint64_t job_id, kc_job_info* out) {
  return server_guard([&]() -> int {
    if (!s || !out) return set_err(KC_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->m);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return set_err(KC_E_INVAL, "unknown job id");
    const Job* j = it->second.get();
    std::memset(out, 0, sizeof(*out));
    out->state = j->state;
    out->status = j->status;
    out->worker = j->worker;
    out->k = j->k;
    out->n_bytes = j->n_bytes;
    out->valid_windows = j->windows;
    out->distinct = j->n_out;
    out->result_estimate_bytes = j->result_est;
    out->result_bytes = j->result_bytes;
    out->t_submit_ms = ms_between(s->t0, j->t_submit);
    if (j->state != KC_JOB_QUEUED) out->t_start_ms = ms_between(s->t0, j->t_start);
    if (j->state == KC_JOB_DONE || j->state == KC_JOB_FAILED)
      out->t_end_ms = ms_between(s->t0, j->t_end);
    return KC_OK;
  });
}

int kc_server_release(kc_server* s, uint64_t job_id) {
  return server_guard([&]() -> int {
    if (!s) return set_err(KC_E_INVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->m);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return set_err(KC_E_INVAL, "unknown job id");
    Job* j = it->second.get();
    if (j->state != KC_JOB_DONE && j->state != KC_JOB_FAILED)
      return set_err(KC_E_INVAL, "job has not finished");
    if (j->keys) {
      // the job's stream finished before it was marked done: nothing uses it
      std::lock_guard<std::mutex> lk2(s->submit_m);
      (void)hipSetDevice(s->device);
      s->slab->free(j->keys, s->ctl);
    }
    s->ledger.sub(j->result_bytes);
    if (j->result_bytes) ++s->epoch;  // its block is back in the slab
    s->jobs.erase(it);
    s->cv_work.notify_all();
    return KC_OK;
  });
}

int kc_server_stats(kc_server* s, kc_serve_stats* out) {
  return server_guard([&]() -> int {
    if (!s || !out) return set_err(KC_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->m);
    std::memset(out, 0, sizeof(*out));
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->failed = s->failed;
    out->queued = s->queue.size();
    out->running = s->running;
    out->valid_windows = s->windows;
    out->budget = s->ledger.budget;
    out->bytes_in_use = s->ledger.in_use;
    out->bytes_peak = s->ledger.peak;
    out->estimate_misses = s->est_misses;
    out->result_bytes_reserved = s->reserved_total;
    out->result_bytes_actual = s->actual_total;
    out->slab_bytes = s->slab->capacity();
    out->unplaced = s->unplaced;
    out->latency_p50_ms = percentile(s->lat_ms, 0.50);
    out->latency_p99_ms = percentile(s->lat_ms, 0.99);
    out->wait_p50_ms = percentile(s->wait_ms, 0.50);
    out->wait_p99_ms = percentile(s->wait_ms, 0.99);
    out->busy_ms = s->any_start ? ms_between(s->first_start, s->last_end) : 0.0;
    return KC_OK;
  });
}

void kc_server_destroy(kc_server* s) {
  if (!s) return;
  try {
    destroy_server(s);
  } catch (...) {
  }
}

}  // extern "C"
