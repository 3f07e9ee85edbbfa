// Host-side interface between the counting runtime (kc_runtime.cpp) and the
// request server (kc_server.cpp). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

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

// Device bytes the calling thread's scratch arena (current device) grows by
// for a plain count of n_bytes input bytes. Exact for the device-planned
// path; the recursive fallback taken after a leaf overflow may need more.
uint64_t scratch_growth(uint64_t n_bytes, int k, int P, const kc_options* opt);

// The same for an empty arena.
uint64_t scratch_bytes(uint64_t n_bytes, int k, int P, const kc_options* opt);

// Device bytes held by the calling thread's arena on the current device.
uint64_t arena_bytes();

// Device temporaries of the merge and the filter: a buffer of the calling
// thread's context on the current device, grown stream-ordered on st from the
// library pool and kept between calls (the callers are synchronous, so the
// buffer is idle when a call starts). Returns nullptr on failure, with the
// error message in *err and its status in *code.
void* thread_scratch(size_t bytes, hipStream_t st, std::string* err, int* code) noexcept;

// The library's stream-ordered memory pool of a device (created on first
// use): the count arenas and the server's results come from it. It keeps the
// blocks freed into it (no release threshold), so growing an arena or
// dropping a result while other streams run never hands memory back to the
// driver; trim_device_pool frees the arenas of threads that have ended and
// returns the idle blocks (kc_release_scratch and server teardown call it).
hipError_t device_pool(int device, hipMemPool_t* pool);
void trim_device_pool(int device);

// Returns the calling thread's count arenas to the pool without trimming it
// (a server worker making room under its budget while others run).
void release_thread_arena();

// Sets the message kc_last_error() returns on the calling thread.
void set_last_error(const std::string& msg);

}  // namespace kc
