// Host-side interface between the counting runtime (kc_runtime.cpp) and the
// request server (kc_server.cpp). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/kc.h"

namespace kc {

// Output allocation of a count whose result size is only known on the device:
// fn is called once the number of distinct keys is known (before the pairs are
// written) and must return device memory for `distinct` keys of `key_words`
// uint64 words each and as many uint32 counts, or a KC_E_* status.
struct OutAlloc {
  int (*fn)(void* user, uint64_t distinct, int key_words, uint64_t** keys, uint32_t** counts);
  void* user;
};

// kc_count_ex with the output allocated through `oa` instead of passed in.
// Returns a status; on error *err receives the message. Synchronous on `st`.
int count_with_alloc(const uint8_t* reads, const uint64_t* offsets, uint64_t n_reads, int k,
                     int P, const kc_options* opt, hipStream_t st, const OutAlloc& oa,
                     uint64_t* n_out, kc_stats* stats, std::string* err);

// Device bytes of the arena block a server worker needs for a plain count of
// n_bytes input bytes: every buffer of the device-planned path, plus room for
// the refinement a leaf overflow may need (beyond it, refinement buffers are
// taken from the slab for the job's duration).
uint64_t scratch_bytes(uint64_t n_bytes, int k, int P, const kc_options* opt);

// One device allocation, made when a server is created, from which its
// workers' arena blocks and its results are cut, so that serving maps and
// unmaps no device memory (a device free waits for every stream of the device,
// and mapping fresh memory while other streams run stalls them). A block
// freed on a stream is reused only once that stream's work up to the free has
// completed (an event recorded per freed block). Thread-safe.
class Slab {
 public:
  // Maps `bytes` of device memory on the current device (nullptr on failure,
  // message in *err).
  static Slab* create(uint64_t bytes, std::string* err);
  ~Slab();
  // A block of at least `bytes` bytes (256-byte aligned), or nullptr when no
  // free range is large enough even after waiting for pending frees. Arena
  // blocks are taken from the low end, results (high = true) from the high
  // end, which keeps the few large arena blocks from being cut up.
  void* alloc(uint64_t bytes, bool high);
  // Returns a block; it becomes reusable once the work queued on st so far
  // has finished.
  void free(void* p, hipStream_t st);
  uint64_t capacity() const { return cap_; }

 private:
  Slab() = default;
  struct Pending {
    uint64_t off, size;
    hipEvent_t ev;
  };
  void reclaim(bool wait);  // pending blocks whose work has finished become free
  void insert_free(uint64_t off, uint64_t size);  // with coalescing of neighbours
  char* base_ = nullptr;
  uint64_t cap_ = 0;
  std::mutex m_;
  std::map<uint64_t, uint64_t> free_;  // offset -> size, disjoint, not adjacent
  std::map<uint64_t, uint64_t> live_;  // offset -> size of handed-out blocks
  std::vector<Pending> pending_;       // freed, waiting for their stream
  std::vector<hipEvent_t> events_;     // idle events for later frees
};

// The count context of one server worker: its device buffers are carved,
// job by job, from an arena block the worker holds (cut from the slab); its
// pinned host staging and events are its own.
struct WorkerArena;
WorkerArena* worker_arena_create(int device);
void worker_arena_destroy(WorkerArena* wa);

// count_with_alloc with every device buffer carved from block[0, block_bytes);
// refinement buffers that do not fit are taken from `spill` and returned when
// the count ends. Synchronous on `st`.
int count_in_block(WorkerArena* wa, void* block, uint64_t block_bytes, Slab* spill,
                   const uint8_t* reads, const uint64_t* offsets, uint64_t n_reads, int k, int P,
                   const kc_options* opt, hipStream_t st, const OutAlloc& oa, uint64_t* n_out,
                   kc_stats* stats, std::string* err);

// Device temporaries of the merge and the filter: a buffer of the calling
// thread's context on the current device, grown stream-ordered on st from the
// library pool and kept between calls (the callers are synchronous, so the
// buffer is idle when a call starts). Returns nullptr on failure, with the
// error message in *err and its status in *code.
void* thread_scratch(size_t bytes, hipStream_t st, std::string* err, int* code) noexcept;

// The library's stream-ordered memory pool of a device (created on first
// use): the count arenas of plain calls come from it. It keeps the blocks
// freed into it (no release threshold), so growing an arena while other
// streams run never hands memory back to the driver; trim_device_pool frees
// the arenas of threads that have ended and returns the idle blocks
// (kc_release_scratch calls it).
hipError_t device_pool(int device, hipMemPool_t* pool);
void trim_device_pool(int device);

// Sets the message kc_last_error() returns on the calling thread.
void set_last_error(const std::string& msg);

}  // namespace kc
