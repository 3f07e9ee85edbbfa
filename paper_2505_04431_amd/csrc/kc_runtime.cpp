// Host runtime behind the C ABI of include/kc.h: argument checks, a
// per-thread device arena, the partition planner (owner layout, MSD splits,
// leaf list, output offsets) and the launch sequence of the kernels in
// kc_kernels.hip. No exception leaves this file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <optional>
#include <string>
#include <vector>

#include "../../include/kc.h"
#include "kc_host.h"
#include "kc_internal.h"

namespace {

typedef unsigned __int128 u128;

thread_local std::string g_err;
thread_local kc_stats g_stats;

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  bool pooled = false;    // from the library's device pool (freed stream-ordered)
  bool borrowed = false;  // a piece of the allocation-free entry point's scratch (never freed)
};

// Frees an idle buffer.
void drop(DevBuf& b) {
  if (b.p && !b.borrowed) (void)(b.pooled ? hipFreeAsync(b.p, nullptr) : hipFree(b.p));
  b = DevBuf{};
}

// ---- the allocation-free entry point (kc_count_noalloc)
//
// Its device memory is one static array per device, `scratch`; while one of
// its calls runs on a thread, every buffer the call would grow is carved from
// that array instead (a bump pointer reset per call), and small host copies
// go through a static host array instead of pinned memory.
constexpr size_t kNoAllocScratchBytes = (size_t)KC_NOALLOC_SCRATCH_MIB << 20;
constexpr size_t kNoAllocHostBytes = 8u << 20;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

struct Carve {
  char* base;
  size_t cap, used;
  bool static_host;                 // small host copies through the static host array
  kc::Slab* spill;                  // if set: what does not fit is taken from here...
  std::vector<void*>* spilled;      // ...and listed, to be returned when the call ends
};
thread_local Carve* g_carve = nullptr;
alignas(64) char g_noalloc_host[kNoAllocHostBytes];
std::mutex g_noalloc_m;  // one allocation-free call at a time (the host array is shared)

struct Fail;
[[noreturn]] void fail(int code, const std::string& msg);

// Gives b a fresh piece of the scratch array of at least `bytes` bytes (its
// old piece, if any, is abandoned until the call ends).
void carve(DevBuf& b, size_t bytes, const char* name) {
  Carve& cv = *g_carve;
  const size_t want = (std::max<size_t>(bytes, 256) + 255) & ~(size_t)255;
  b.pooled = false;
  b.borrowed = true;
  if (want <= cv.cap - cv.used) {
    b.p = cv.base + cv.used;
    b.cap = want;
    cv.used += want;
    return;
  }
  if (cv.spill) {
    void* p = cv.spill->alloc(want, false);
    if (!p)
      fail(KC_E_NOMEM, std::string("server memory exhausted (") + std::to_string(bytes) +
                           " bytes for " + name + " beyond the worker's arena block)");
    cv.spilled->push_back(p);
    b.p = p;
    b.cap = want;
    return;
  }
  b = DevBuf{};
  fail(KC_E_NOMEM, std::string("kc_count_noalloc: its fixed device scratch of ") +
                       std::to_string(cv.cap >> 20) + " MiB is exhausted (" +
                       std::to_string(bytes) + " more bytes for " + name + ")");
}

struct Ctx {
  int device = -1;
  DevBuf packed, inv, endm, valid, bufA, bufB, tmpcnt;
  DevBuf hist, sbegin, cursor, cursor2, order, items, bins, subhist, leaves, dcnt, outoff, state;
  DevBuf large, ovfl, bsum, itemoff;
  // overflow refinement: overflowed leaves, part attempts, the spliced list
  DevBuf rlist, rleaves, rcount, aleaves, adcnt, alarge, aovfl, rparts, rcnt, leaves2, dcnt2;
  DevBuf post;  // temporaries of kc_merge_counts / kc_filter_min_count
  std::vector<int> order_host;
  int order_P = -1, order_sb = -1;
  void* host = nullptr;  // pinned staging for small device<->host copies
  size_t host_cap = 0;
  hipEvent_t ev[32] = {};
  bool ev_ok = false;
  // The end of the last call's work: a call may return with kernels still
  // reading these buffers (the concat into caller-owned outputs), so the next
  // call, on whatever stream, first waits for it.
  hipEvent_t done = nullptr;
  bool done_set = false;

  ~Ctx() {
    int prev = -1;
    if (hipGetDevice(&prev) == hipSuccess && device >= 0) (void)hipSetDevice(device);
    DevBuf* all[] = {&packed,  &inv,     &endm,   &valid,   &bufA,   &bufB,    &tmpcnt,  &hist,
                     &sbegin,  &cursor,  &cursor2, &order,  &items,  &bins,    &subhist,
                     &leaves,  &dcnt,    &outoff, &state,   &large,  &ovfl,    &bsum,
                     &itemoff, &rlist,   &rleaves, &rcount, &aleaves, &adcnt,  &alarge,
                     &aovfl,   &rparts,  &rcnt,   &leaves2, &dcnt2,  &post};
    // the last call's kernels may still read the buffers
    if (done_set) (void)hipEventSynchronize(done);
    for (DevBuf* b : all) drop(*b);
    if (host) (void)hipHostFree(host);
    if (ev_ok)
      for (hipEvent_t& e : ev) (void)hipEventDestroy(e);
    if (done) (void)hipEventDestroy(done);
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

using CtxMap = std::map<int, std::unique_ptr<Ctx>>;

// Contexts of threads that have ended. A thread-local destructor must not call
// HIP (the runtime's and a profiler's per-thread state may be gone by then),
// so an ending thread only hands its contexts over; they are freed by the next
// count on any thread, kc_release_scratch or a server's teardown. Never
// destroyed: at process exit the device memory goes with the process.
std::mutex g_orphan_m;
std::vector<std::unique_ptr<Ctx>>* const g_orphans = new std::vector<std::unique_ptr<Ctx>>();
std::atomic<bool> g_have_orphans{false};  // a hint read without the lock

struct ThreadCtx {
  CtxMap m;
  ~ThreadCtx() {
    std::lock_guard<std::mutex> lk(g_orphan_m);
    for (auto& kv : m)
      if (kv.second) g_orphans->push_back(std::move(kv.second));
    g_have_orphans.store(!g_orphans->empty(), std::memory_order_relaxed);
  }
};
thread_local ThreadCtx g_ctx;

// Frees the contexts of ended threads (after their last work has finished).
void free_orphans() {
  std::vector<std::unique_ptr<Ctx>> v;
  {
    std::lock_guard<std::mutex> lk(g_orphan_m);
    v.swap(*g_orphans);
    g_have_orphans.store(false, std::memory_order_relaxed);
  }
}

struct Fail {
  int code;
};

[[noreturn]] void fail(int code, const std::string& msg) {
  g_err = msg;
  throw Fail{code};
}

void hipchk(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory) fail(KC_E_NOMEM, std::string(what) + ": " + hipGetErrorString(e));
    fail(KC_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  }
}

// Bytes ensure() allocates for a request (1/8 headroom against regrowth).
size_t alloc_size(size_t bytes) {
  if (bytes == 0) bytes = 256;
  return bytes + bytes / 8;
}

// Synchronous growth (plans, whose buffers are set up before any launch).
void ensure(DevBuf& b, size_t bytes, const char* name) {
  if (bytes == 0) bytes = 256;
  if (b.cap >= bytes) return;
  if (g_carve) return carve(b, bytes, name);
  if (b.p) {
    if (b.pooled) {
      hipchk(hipFreeAsync(b.p, nullptr), "hipFreeAsync");
      hipchk(hipStreamSynchronize(nullptr), "hipStreamSynchronize");
    } else {
      hipchk(hipFree(b.p), "hipFree");
    }
    b = DevBuf{};
  }
  size_t want = alloc_size(bytes);
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    want = bytes;
    e = hipMalloc(&b.p, want);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    fail(KC_E_NOMEM, std::string("device allocation of ") + std::to_string(bytes) + " bytes for " +
                         name + " failed");
  }
  b.cap = want;
}

// Stream-ordered growth of a count buffer: the old block goes back to the
// library pool behind the work queued on st and the new one comes from it, so
// growth neither waits for the device nor frees memory to the driver.
void grow(DevBuf& b, size_t bytes, const char* name, hipStream_t st) {
  if (bytes == 0) bytes = 256;
  if (b.cap >= bytes) return;
  if (g_carve) return carve(b, bytes, name);
  int dev = 0;
  hipchk(hipGetDevice(&dev), "hipGetDevice");
  hipMemPool_t pool = nullptr;
  hipchk(kc::device_pool(dev, &pool), "device memory pool");
  // a buffer that grows again grows by half at least: fewer growths, each of
  // which may map fresh memory, while a server's arenas reach their sizes
  size_t want = std::max(alloc_size(bytes), b.cap + b.cap / 2);
  if (b.p) {
    hipchk(b.pooled ? hipFreeAsync(b.p, st) : hipFree(b.p), "free");
    b = DevBuf{};
  }
  hipError_t e = hipMallocFromPoolAsync(&b.p, want, pool, st);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    want = bytes;
    e = hipMallocFromPoolAsync(&b.p, want, pool, st);
  }
  if (e != hipSuccess) {
    // idle blocks the pool keeps may be what is missing: return them, retry
    (void)hipGetLastError();
    hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
    (void)hipMemPoolTrimTo(pool, 0);
    e = hipMallocFromPoolAsync(&b.p, want, pool, st);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b = DevBuf{};
    fail(KC_E_NOMEM, std::string("device allocation of ") + std::to_string(bytes) + " bytes for " +
                         name + " failed");
  }
  b.cap = want;
  b.pooled = true;
}

void* host_stage(Ctx& c, size_t bytes) {
  if (g_carve && g_carve->static_host) {
    // allocation-free call: the static host array (held under g_noalloc_m)
    if (bytes > kNoAllocHostBytes)
      fail(KC_E_NOMEM, "kc_count_noalloc: " + std::to_string(bytes) +
                           " bytes of host staging exceed its fixed " +
                           std::to_string(kNoAllocHostBytes >> 20) + " MiB");
    return g_noalloc_host;
  }
  // callers only stage device-to-host copies and synchronize before reading,
  // so no copy into this buffer is pending when it is reallocated
  if (c.host_cap < bytes) {
    if (c.host) hipchk(hipHostFree(c.host), "hipHostFree");
    c.host = nullptr;
    size_t want = std::max<size_t>(bytes, 1 << 20);
    hipchk(hipHostMalloc(&c.host, want, hipHostMallocDefault), "hipHostMalloc");
    c.host_cap = want;
  }
  return c.host;
}

Ctx& context() {
  int dev = 0;
  hipchk(hipGetDevice(&dev), "hipGetDevice");
  auto& slot = g_ctx.m[dev];
  if (!slot) {
    slot.reset(new Ctx());
    slot->device = dev;
  }
  return *slot;
}

// Orders a call on `st` after the previous call on this thread's context and,
// on every exit, marks the call's end. The wait is made even when the stream
// handle is the same: a destroyed stream's handle may come back for a new one.
struct CtxUse {
  Ctx& c;
  hipStream_t st;
  CtxUse(Ctx& ctx, hipStream_t s) : c(ctx), st(s) {
    if (!c.done) hipchk(hipEventCreateWithFlags(&c.done, hipEventDisableTiming), "hipEventCreate");
    if (c.done_set) hipchk(hipStreamWaitEvent(st, c.done, 0), "hipStreamWaitEvent");
  }
  ~CtxUse() {
    if (hipEventRecord(c.done, st) == hipSuccess) {
      c.done_set = true;
    } else {
      // without the mark, wait for everything before the context is reused
      (void)hipGetLastError();
      (void)hipStreamSynchronize(st);
      c.done_set = false;
    }
  }
};

uint64_t host_mix(uint64_t h) {  // owner assignment of shards (MurmurHash3 finalizer)
  h ^= h >> 33;
  h *= 0xff51afd7ed558ccdull;
  h ^= h >> 33;
  h *= 0xc4ceb9fe1a85ec53ull;
  h ^= h >> 33;
  return h;
}

int ceil_log2(uint64_t x) {
  int b = 0;
  while (b < 63 && (1ull << b) < x) ++b;
  return b;
}

struct Timer {
  Ctx& c;
  hipStream_t s;
  bool on;
  int n = 0;
  int stage[32];
  Timer(Ctx& c_, hipStream_t s_, bool on_) : c(c_), s(s_), on(on_) {
    if (on && !c.ev_ok) {
      for (hipEvent_t& e : c.ev) hipchk(hipEventCreate(&e), "hipEventCreate");
      c.ev_ok = true;
    }
  }
  void mark(int st) {  // the interval from the previous mark to this one is charged to `st`
    if (!on || n >= 32) return;
    stage[n] = st;
    hipchk(hipEventRecord(c.ev[n], s), "hipEventRecord");
    ++n;
  }
  void collect(kc_stats& out) {
    if (!on) return;
    hipchk(hipEventSynchronize(c.ev[n - 1]), "hipEventSynchronize");
    for (int i = 1; i < n; ++i) {
      float ms = 0;
      hipchk(hipEventElapsedTime(&ms, c.ev[i - 1], c.ev[i]), "hipEventElapsedTime");
      if (stage[i] >= 0 && stage[i] < 12) out.ms_stage[stage[i]] += ms;
    }
  }
};

enum { ST_PACK = 0, ST_HIST = 1, ST_SCATTER = 2, ST_SPLIT_HIST = 3, ST_SPLIT = 4,
       ST_LEAF_SMALL = 5, ST_LEAF = 6, ST_OUT = 7, ST_CONCAT = 8, ST_CHECK = 9, ST_REFINE = 10,
       ST_LEAF_SECOND = 11, ST_NONE = -1 };

// Batch layout check: set s must own the bytes [set_byte_off[s], set_byte_off[s+1])
// of the stream, i.e. offsets[set_first_read[s]] - offsets[0] == set_byte_off[s].
__global__ void k_batch_layout_ok(const uint64_t* off, const unsigned long long* set_first_read,
                                  const unsigned long long* set_byte_off, uint32_t n_sets,
                                  unsigned int* bad) {
  const uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s <= n_sets && off[set_first_read[s]] - off[0] != set_byte_off[s]) atomicOr(bad, 1u);
}

__global__ void k_offsets_ok(const uint64_t* off, uint64_t n, unsigned int* bad) {  // sets *bad if decreasing
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && off[i + 1] < off[i]) atomicOr(bad, 1u);
}


struct Call {
  const uint8_t* reads;
  const uint64_t* offsets;
  uint64_t n_reads;
  int k, P;
  uint64_t* out_keys;
  uint32_t* out_counts;
  uint64_t cap;
  kc_options o;
  hipStream_t st;
  const kc::OutAlloc* oa = nullptr;  // output allocated once D is known (no concat before)
  uint64_t concat_leaves = 0;        // leaf slots the deferred concat covers
  // derived
  uint64_t N = 0, off0 = 0;
  int words = 1;  // 64-bit words per key: 1, 2 or 4
  int keybits = 0, sb = 0, nb = 0, slots_log2 = 0;
  int split_r = 8;
  bool merged = false;  // the split scatter pre-aggregated (leaves may carry counts)
  size_t ksz = 8;
  uint64_t C = 0, T = 0, H = 0;
};

// Owner-major order of the shards: owner(s) = multiply-shift range reduction of
// a 64-bit mix of the shard index onto [0, P). Cached per (P, shard bits).
const std::vector<int>& owner_order(Ctx& c, const Call& q, kc_stats& S,
                                    const std::vector<uint64_t>* hist) {
  static thread_local std::vector<int> order;
  static thread_local std::vector<uint64_t> owner;
  order.resize(q.nb);
  owner.resize(q.nb);
  for (int i = 0; i < q.nb; ++i) {
    order[i] = i;
    owner[i] = (uint64_t)(((u128)host_mix((uint64_t)i * 0x9E3779B97F4A7C15ull + 0x51ED27ull) *
                           (u128)(uint64_t)q.P) >> 64);
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return owner[a] < owner[b]; });
  if (hist) {
    uint64_t cur = ~0ull, w = 0;
    for (int i : order) {
      if (owner[i] != cur) {
        S.max_owner_windows = std::max(S.max_owner_windows, w);
        w = 0;
        cur = owner[i];
      }
      w += (*hist)[i];
    }
    S.max_owner_windows = std::max(S.max_owner_windows, w);
  }
  (void)c;
  return order;
}

void upload_sync(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (!bytes) return;
  hipchk(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
  hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
}

kc::DevState read_state(Ctx& c, hipStream_t st) {
  kc::DevState* h = (kc::DevState*)host_stage(c, sizeof(kc::DevState));
  hipchk(hipMemcpyAsync(h, c.state.p, sizeof(kc::DevState), hipMemcpyDeviceToHost, st),
         "hipMemcpyAsync");
  hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
  return *h;
}

// Recovery after leaves of the device-planned path overflowed their tables:
// only those leaves are partitioned further, level by level under host
// control (split their records on the next key bits into the other buffer,
// count every non-empty part, split again what overflows), and the parts
// replace their parent in the leaf list, which stays in key order. Every part
// is counted as soon as it exists, so a part dominated by one frequent key
// is settled at once however many records it holds. Ends with the output
// offsets (and the concat unless the caller allocates the output first).
// keep_leaves: leaf slots the device-planned path of this call needs (both
// leaf-list buffers keep at least that many).
void refine_overflowed(Ctx& c, Call& q, kc_stats& S, Timer& tm, uint64_t nl0,
                       uint64_t keep_leaves) {
  const hipStream_t st = q.st;
  kc::DevState* dst_state = (kc::DevState*)c.state.p;
  // the overflowed leaves only (the list of all leaves stays on the device)
  grow(c.rlist, nl0 * 4, "overflowed leaf list", st);
  grow(c.rleaves, nl0 * sizeof(kc::Leaf), "overflowed leaves", st);
  grow(c.rcount, 8, "overflow count", st);
  hipchk(kc::launch_list_overflowed((uint32_t*)c.dcnt.p, nl0, (kc::Leaf*)c.leaves.p,
                                    (uint32_t*)c.rlist.p, (kc::Leaf*)c.rleaves.p,
                                    (unsigned long long*)c.rcount.p, st),
         "overflow list launch");
  uint64_t R = 0;
  {
    uint64_t* h = (uint64_t*)host_stage(c, 64);
    hipchk(hipMemcpyAsync(h, c.rcount.p, 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
    R = h[0];
  }
  std::vector<uint32_t> ridx(R);
  std::vector<kc::Leaf> rlv(R);
  if (R) {
    char* h = (char*)host_stage(c, R * (4 + sizeof(kc::Leaf)) + 64);
    hipchk(hipMemcpyAsync(h, c.rlist.p, R * 4, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    hipchk(hipMemcpyAsync(h + R * 4, c.rleaves.p, R * sizeof(kc::Leaf), hipMemcpyDeviceToHost, st),
           "hipMemcpyAsync");
    hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
    std::memcpy(ridx.data(), h, R * 4);
    std::memcpy(rlv.data(), h + R * 4, R * sizeof(kc::Leaf));
  }
  // roots in leaf order (the list came in any order)
  std::vector<uint32_t> ord(R);
  for (uint32_t i = 0; i < R; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](uint32_t a, uint32_t b) { return ridx[a] < ridx[b]; });
  // key bits below a parent leaf's prefix (up to 256 bits for k <= 128)
  struct Rel {
    u128 lo = 0, hi = 0;
    Rel shl(int n) const {  // n < 256
      if (n == 0) return *this;
      if (n >= 128) return Rel{0, lo << (n - 128)};
      return Rel{lo << n, (hi << n) | (lo >> (128 - n))};
    }
    bool operator<(const Rel& o) const { return hi != o.hi ? hi < o.hi : lo < o.lo; }
  };
  struct Part {
    uint64_t begin, end;
    Rel rel;      // key bits below the parent leaf's prefix consumed so far
    int bits;     // key bits consumed in total (from the most significant end)
    int buf;      // buffer holding its records
    uint32_t root;
    uint32_t cshift, shard;  // record format of the root leaf (pre-aggregated or not)
  };
  struct Done {
    uint32_t root;
    Rel start;   // first key of its range, relative to the parent's prefix
    kc::Leaf leaf;
    uint32_t d;
  };
  std::vector<Part> split;
  for (uint32_t r = 0; r < R; ++r) {
    const kc::Leaf& lf = rlv[ord[r]];
    if ((int)lf.bits >= q.keybits) fail(KC_E_INTERNAL, "single-key partition overflowed its table");
    split.push_back(Part{lf.begin, lf.end, Rel{}, (int)lf.bits, (int)lf.buf, r, lf.cshift,
                         lf.shard});  // root = rank r
    ++S.n_overflow;
  }
  std::vector<Done> done;
  void* bufs[2] = {c.bufA.p, c.bufB.p};
  // five bits per level. What reaches this point has overflowed a table of twice
  // the leaf kernel's size as well (one-word keys): a few dense clusters, cut
  // by 5 bits in 5 levels and 120.2 ms against 8 levels and 123.2 ms (3 bits)
  // and 4 levels and 120.2 ms (8 bits) on 40,000,000 reads at k = 31. (Before
  // that second table, 3 bits were best: 4,323 overflowed leaves of 490
  // million records, and 6 bits made 275,703 parts at the first level.)
  const int refine_bits = q.o.refine_bits > 0 ? q.o.refine_bits : 5;
  const uint64_t tile = (uint64_t)kc::split_tile(q.words, q.split_r);
  int level = 0;
  while (!split.empty()) {
    ++level;
    // split every part on its next key bits (at least 2, so each level narrows it)
    const size_t ns = split.size();
    std::vector<kc::SplitBin> sbins(ns);
    std::vector<kc::SplitItem> items;
    uint64_t hoff = 0;
    for (size_t i = 0; i < ns; ++i) {
      const Part& b = split[i];
      const uint64_t n = b.end - b.begin;
      const int remaining = q.keybits - b.bits;
      // A part overflowed because of its distinct keys, not its records (a
      // part of many records and few keys counts fine), so it is cut in a
      // few pieces by key, not by record count; pieces too rich in keys are
      // cut again at the next level. (Cutting into pieces of a leaf target of
      // records each, up to 8 bits a level, took 19.7 against 30.9 ms on a
      // satellite-repeat input but 184 against 136 ms on the 40,000,000-read
      // workload at k = 31: millions of small parts to plan and splice.)
      (void)n;
      const int nbits = std::max(1, std::min(refine_bits, remaining));
      sbins[i] = kc::SplitBin{hoff, (uint32_t)(remaining - nbits), (uint32_t)nbits};
      hoff += 1ull << nbits;
      for (uint64_t a = b.begin; a < b.end; a += tile)
        items.push_back(kc::SplitItem{a, std::min(b.end, a + tile), (uint32_t)i, 0});
    }
    // parts of one level may sit in different buffers: one pass per source buffer
    std::vector<Part> next;
    for (int src = 0; src < 2; ++src) {
      std::vector<kc::SplitItem> it_src;
      for (const kc::SplitItem& it : items)
        if (split[it.bin].buf == src) it_src.push_back(it);
      if (it_src.empty()) continue;
      grow(c.bins, ns * sizeof(kc::SplitBin), "split bins", st);
      grow(c.items, it_src.size() * sizeof(kc::SplitItem), "split items", st);
      grow(c.subhist, hoff * 8, "sub-bin histogram", st);
      grow(c.cursor2, hoff * 8, "sub-bin cursors", st);
      upload_sync(c.items.p, it_src.data(), it_src.size() * sizeof(kc::SplitItem), st);
      upload_sync(c.bins.p, sbins.data(), ns * sizeof(kc::SplitBin), st);
      unsigned long long ni = it_src.size();
      upload_sync(&dst_state->n_items, &ni, 8, st);
      hipchk(kc::launch_fill_u64((unsigned long long*)c.subhist.p, hoff, 0, st), "fill launch");
      hipchk(kc::launch_split_hist(q.words, bufs[src], (kc::SplitItem*)c.items.p, dst_state,
                                   it_src.size(), (kc::SplitBin*)c.bins.p,
                                   (unsigned long long*)c.subhist.p, 1, 0, st),
             "split histogram launch");
      uint64_t* hsub = (uint64_t*)host_stage(c, hoff * 8 + 64);
      hipchk(hipMemcpyAsync(hsub, c.subhist.p, hoff * 8, hipMemcpyDeviceToHost, st),
             "hipMemcpyAsync");
      hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
      std::vector<uint64_t> hcur(hoff, 0);
      for (size_t i = 0; i < ns; ++i) {
        const Part& b = split[i];
        if (b.buf != src) continue;
        const kc::SplitBin& sbn = sbins[i];
        uint64_t r = b.begin;
        for (uint64_t j = 0; j < (1ull << sbn.nbits); ++j) {
          const uint64_t cnt = hsub[sbn.hist_off + j];
          hcur[sbn.hist_off + j] = r;
          if (cnt) {
            Rel nr = b.rel.shl((int)sbn.nbits);
            nr.lo |= (u128)j;
            next.push_back(Part{r, r + cnt, nr, b.bits + (int)sbn.nbits, 1 - b.buf, b.root,
                                b.cshift, b.shard});
          }
          r += cnt;
        }
        if (r != b.end) fail(KC_E_INTERNAL, "split histogram does not match partition size");
      }
      upload_sync(c.cursor2.p, hcur.data(), hoff * 8, st);
      hipchk(kc::launch_split_scatter(q.words, bufs[src], bufs[1 - src],
                                      (kc::SplitItem*)c.items.p, dst_state, it_src.size(),
                                      (kc::SplitBin*)c.bins.p, (unsigned long long*)c.cursor2.p,
                                      q.split_r, 0, 1, 0, st),
             "split scatter launch");
    }
    tm.mark(ST_REFINE);
    // count every part
    const size_t na = next.size();
    std::vector<kc::Leaf> al(na);
    for (size_t i = 0; i < na; ++i)
      al[i] = kc::Leaf{next[i].begin, next[i].end, (uint32_t)next[i].buf, (uint32_t)next[i].bits,
                       next[i].cshift, next[i].shard};
    grow(c.aleaves, na * sizeof(kc::Leaf), "part table", st);
    grow(c.adcnt, na * 4, "part counts", st);
    grow(c.alarge, na * 4, "large-part list", st);
    grow(c.aovfl, na * 4, "overflowed-part list", st);
    upload_sync(c.aleaves.p, al.data(), na * sizeof(kc::Leaf), st);
    unsigned long long nlu = na;
    upload_sync(&dst_state->n_leaves, &nlu, 8, st);
    hipchk(kc::launch_leaf_small(q.words, q.keybits, c.bufA.p, c.bufB.p, (uint32_t*)c.tmpcnt.p,
                                 (kc::Leaf*)c.aleaves.p, dst_state, na, (uint32_t*)c.adcnt.p,
                                 (uint32_t*)c.alarge.p, (uint32_t*)c.aovfl.p, q.slots_log2, st,
                                 q.o.mode, true, q.merged),
           "leaf count launch");
    hipchk(kc::launch_leaf_large(q.words, q.keybits, c.bufA.p, c.bufB.p, (uint32_t*)c.tmpcnt.p,
                                 (kc::Leaf*)c.aleaves.p, dst_state, na, (uint32_t*)c.adcnt.p,
                                 q.slots_log2, (uint32_t*)c.alarge.p, (uint32_t*)c.aovfl.p, st,
                                 q.o.mode, true, q.merged),
           "leaf count launch");
    hipchk(kc::launch_leaf_second(q.words, q.keybits, c.bufA.p, c.bufB.p, (uint32_t*)c.tmpcnt.p,
                                  (kc::Leaf*)c.aleaves.p, dst_state, (uint32_t*)c.adcnt.p,
                                  q.slots_log2, (uint32_t*)c.aovfl.p, st, q.o.mode, q.merged),
           "leaf count launch");
    tm.mark(ST_REFINE);
    uint32_t* hd = (uint32_t*)host_stage(c, na * 4 + 64);
    hipchk(hipMemcpyAsync(hd, c.adcnt.p, na * 4, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
    split.clear();
    for (size_t i = 0; i < na; ++i) {
      const Part& b = next[i];
      if (hd[i] == kc::kLeafOverflow) {
        if (b.bits >= q.keybits) fail(KC_E_INTERNAL, "single-key partition overflowed its table");
        ++S.n_overflow;
        split.push_back(b);
      } else {
        done.push_back(Done{b.root, b.rel.shl(q.keybits - b.bits), al[i], hd[i]});
        S.max_leaf_windows = std::max(S.max_leaf_windows, b.end - b.begin);
      }
    }
  }
  S.n_levels = 1 + level;
  // splice the parts into the leaf list in place of their parents (on the
  // device: only the parts travel)
  std::sort(done.begin(), done.end(), [](const Done& a, const Done& b) {
    return a.root != b.root ? a.root < b.root : a.start < b.start;
  });
  const uint64_t P = done.size();
  // one upload: parts, part counts, then per root its leaf, first part, part count
  const size_t off_d = P * sizeof(kc::Leaf), off_root = off_d + P * 4;
  const size_t bytes = off_root + 3 * R * 4;
  std::vector<char> hb(bytes);
  kc::Leaf* hp = (kc::Leaf*)hb.data();
  uint32_t* hpd = (uint32_t*)(hb.data() + off_d);
  uint32_t* hroot = (uint32_t*)(hb.data() + off_root);
  uint32_t* hbeg = hroot + R;
  uint32_t* hnp = hbeg + R;
  for (uint32_t r = 0; r < R; ++r) {
    hroot[r] = ridx[ord[r]];
    hbeg[r] = 0;
    hnp[r] = 0;
  }
  for (uint64_t i = 0; i < P; ++i) {
    hp[i] = done[i].leaf;
    hpd[i] = done[i].d;
    if (hnp[done[i].root]++ == 0) hbeg[done[i].root] = (uint32_t)i;
  }
  grow(c.rparts, bytes, "refined parts", st);
  upload_sync(c.rparts.p, hb.data(), bytes, st);
  const char* dp = (const char*)c.rparts.p;
  const uint64_t nl = nl0 - R + P;
  grow(c.rcnt, nl0 * 4, "splice counts", st);
  // the spliced list is built beside the old one and the two are swapped;
  // both keep the larger capacity so that the next call does not reallocate
  grow(c.leaves2, std::max(nl, keep_leaves) * sizeof(kc::Leaf), "leaf table", st);
  grow(c.dcnt2, std::max(nl, keep_leaves) * 4, "leaf counts", st);
  grow(c.bsum, kc::scan_blocks(std::max(nl0, nl)) * 8, "scan block sums", st);
  grow(c.outoff, std::max(nl0, nl) * 8, "output offsets", st);
  unsigned long long n0 = nl0;
  upload_sync(&dst_state->n_leaves, &n0, 8, st);
  hipchk(kc::launch_splice((const kc::Leaf*)c.leaves.p, (const uint32_t*)c.dcnt.p, nl0,
                           (const uint32_t*)(dp + off_root), (const uint32_t*)(dp + off_root) + R,
                           (const uint32_t*)(dp + off_root) + 2 * R, (uint32_t)R,
                           (const kc::Leaf*)dp, (const uint32_t*)(dp + off_d),
                           (uint32_t*)c.rcnt.p, dst_state, (unsigned long long*)c.bsum.p,
                           (unsigned long long*)c.outoff.p, (kc::Leaf*)c.leaves2.p,
                           (uint32_t*)c.dcnt2.p, st),
         "splice launch");
  std::swap(c.leaves, c.leaves2);
  std::swap(c.dcnt, c.dcnt2);
  S.n_leaves = nl;
  unsigned long long nlu = nl;
  upload_sync(&dst_state->n_leaves, &nlu, 8, st);
  unsigned int zero = 0;
  upload_sync(&dst_state->overflow, &zero, 4, st);
  hipchk(kc::launch_plan_out((uint32_t*)c.dcnt.p, dst_state, (unsigned long long*)c.bsum.p, nl,
                             (unsigned long long*)c.outoff.p, st),
         "plan_out launch");
  tm.mark(ST_OUT);
  q.concat_leaves = nl;
  if (q.oa) return;  // the caller allocates the output, then runs the concat
  hipchk(kc::launch_concat(q.words, c.bufA.p, c.bufB.p, (uint32_t*)c.tmpcnt.p,
                           (kc::Leaf*)c.leaves.p, (uint32_t*)c.dcnt.p,
                           (unsigned long long*)c.outoff.p, dst_state, nl, q.cap, q.out_keys,
                           q.out_counts, st),
         "concat launch");
  tm.mark(ST_CONCAT);
}

// One run of the device-planned partitioning over bytes [byte_begin,
// byte_end) of the packed stream: shard histogram, shard plan, owner scatter,
// one split level, leaf counts, output offsets and concat. No host
// synchronization and no allocation happens here (buffers are prepared by
// pipeline_prepare), so a run can be captured into a graph.
struct Pipe {
  int words = 1;  // 64-bit words per key: 1, 2 or 4
  int k = 0, keybits = 0, sb = 0, slots_log2 = 0;
  uint64_t byte_begin = 0, byte_end = 0;  // bytes scanned for windows
  uint64_t rec_bound = 0;                 // upper bound of the records (windows)
  uint64_t T = 0, H = 0;
  uint64_t max_items = 0, max_leaves = 0;
  const kc::BatchSets* batch = nullptr;   // batch form (composite keys)
  int mode = 0;                           // leaf count: 0 hash tables, 1 sort
  int scatter_s = 8, split_r = 8;         // LDS tile shape of the two scatters (one-word keys)
  int merge_cshift = 0;                   // != 0: the split scatter pre-aggregates equal keys
  const int* order = nullptr;             // device, owner-major shard order
};

// Tile shapes of the scatters from the options (0 = automatic).
void tile_params(const kc_options& o, Pipe& p) {
  for (int v : {o.scatter_tile, o.split_tile})
    if (v != 0 && v != 8 && v != 16) fail(KC_E_INVAL, "scatter_tile / split_tile must be 0, 8 or 16");
  // measured on 40,000,000 reads (k = 31 / 21): 16-record split tiles 26.3 / 28.6 ms against
  // 29.0 / 31.5 ms; 1,000,000 reads: 0.56 against 0.61 ms. The owner scatter gains
  // nothing from the larger tile (25.6 against 25.4 ms) and keeps two workgroups per CU.
  p.scatter_s = o.scatter_tile ? o.scatter_tile : 8;
  p.split_r = o.split_tile ? o.split_tile : 16;
  if (p.words != 1) p.scatter_s = p.split_r = 8;
}

void pipe_bounds(Pipe& p) {
  const uint64_t tile = (uint64_t)kc::split_tile(p.words, p.split_r);
  const uint64_t nb = 1ull << p.sb;
  p.max_items = p.rec_bound / tile + nb + 1;
  p.max_leaves = std::min<uint64_t>(nb << kc::kSplitMaxBits, 2 * p.rec_bound / p.T + 2 * nb) + 1;
}

// 64-base chunks of the packed stream (five chunks of padding: the window
// kernels of keys over 64 bases read five mask words from a window start).
uint64_t packed_chunks(uint64_t n_bytes) { return (n_bytes + 63) / 64 + 5; }

// The arena buffers a pipeline run needs: f(member, bytes, name) per buffer.
// The one list both allocation (pipeline_prepare) and the memory estimates of
// the server (scratch_bytes) read.
template <class F>
void pipeline_needs(const Pipe& p, F&& f) {
  const size_t ksz = 8 * p.words;
  const uint64_t nb = 1ull << p.sb;
  f(&Ctx::bufA, std::max<uint64_t>(p.rec_bound, 1) * ksz, "record buffer A");
  f(&Ctx::bufB, std::max<uint64_t>(p.rec_bound, 1) * ksz, "record buffer B");
  f(&Ctx::tmpcnt, std::max<uint64_t>(p.rec_bound, 1) * 4, "pair counts");
  f(&Ctx::hist, (1 + kc::kXcds) * nb * 8, "shard histogram");  // totals, then per tile class
  f(&Ctx::sbegin, nb * 8, "shard begins");
  f(&Ctx::cursor, kc::kXcds * nb * 8, "shard cursors");          // per tile class
  f(&Ctx::bins, nb * sizeof(kc::SplitBin), "split bins");
  f(&Ctx::items, p.max_items * sizeof(kc::SplitItem), "split items");
  f(&Ctx::itemoff, (nb + 1) * 8, "split item offsets");
  f(&Ctx::subhist, kc::kXcds * p.max_leaves * 8, "sub-bin histogram");  // per item class
  f(&Ctx::cursor2, kc::kXcds * p.max_leaves * 8, "sub-bin cursors");
  f(&Ctx::leaves, p.max_leaves * sizeof(kc::Leaf), "leaf table");
  f(&Ctx::dcnt, p.max_leaves * 4, "leaf counts");
  f(&Ctx::outoff, p.max_leaves * 8, "output offsets");
  f(&Ctx::large, p.max_leaves * 4, "large-leaf list");
  f(&Ctx::ovfl, p.max_leaves * 4, "overflowed-leaf list");
  f(&Ctx::bsum, kc::scan_blocks(p.max_leaves) * 8, "scan block sums");
}

void pipeline_prepare(Ctx& c, const Pipe& p) {
  pipeline_needs(p, [&](DevBuf Ctx::*m, size_t bytes, const char* name) { ensure(c.*m, bytes, name); });
}

// Plain calls add the packed input, the device state and the owner order.
template <class F>
void plain_needs(const Pipe& p, F&& f) {
  const uint64_t nchunks = packed_chunks(p.byte_end);
  f(&Ctx::packed, nchunks * 16, "packed bases");
  f(&Ctx::inv, nchunks * 8, "invalid mask");
  f(&Ctx::endm, nchunks * 8, "end mask");
  f(&Ctx::valid, nchunks * 8, "valid-start mask");
  f(&Ctx::state, sizeof(kc::DevState), "device state");
  f(&Ctx::order, (size_t)(1ull << p.sb) * 4, "owner order");
  pipeline_needs(p, f);
}

// Output of a pipeline run: plain (keys of 1 or 2 words, counts) or batch
// class output (k-mer word, count, set id within the class).
struct PipeOut {
  uint64_t* keys;
  uint32_t* counts;
  uint32_t* set;  // batch form only
  uint64_t cap;
  bool concat = true;  // false: stop after the output offsets
};

void enqueue_pipeline(Ctx& c, const Pipe& p, kc::DevState* dstate, Timer& tm, const PipeOut& out,
                      hipStream_t st) {
  // item classes of the split scatter (one when a leaf's end is its cursor's last value)
  const int ncls = p.merge_cshift ? 1 : kc::kXcds;
  hipchk(kc::launch_fill_u64((unsigned long long*)c.hist.p, (1ull + kc::kXcds) << p.sb, 0, st),
         "fill launch");
  hipchk(kc::launch_valid_mask(p.words, (uint64_t*)c.inv.p, (uint64_t*)c.endm.p, p.byte_begin,
                               p.byte_end, p.k, (uint64_t*)c.valid.p, st),
         "valid mask launch");
  hipchk(kc::launch_window_hist(p.words, (uint64_t*)c.packed.p, (uint64_t*)c.valid.p,
                                p.byte_begin, p.byte_end, p.k, p.keybits,
                                p.sb, p.batch, (unsigned long long*)c.hist.p, &dstate->W,
                                p.scatter_s, st),
         "window histogram launch");
  tm.mark(ST_HIST);
  hipchk(kc::launch_plan_shards((unsigned long long*)c.hist.p, p.order, p.sb, p.keybits, p.T, p.H,
                                kc::split_tile(p.words, p.split_r), (unsigned long long*)c.sbegin.p,
                                (unsigned long long*)c.cursor.p, (kc::SplitBin*)c.bins.p,
                                (kc::SplitItem*)c.items.p, (unsigned long long*)c.itemoff.p,
                                (unsigned long long*)c.subhist.p, p.max_leaves, p.max_items,
                                ncls, dstate, st),
         "plan_shards launch");
  hipchk(kc::launch_window_scatter(p.words, (uint64_t*)c.packed.p, (uint64_t*)c.valid.p,
                                   p.byte_begin, p.byte_end, p.k, p.keybits,
                                   p.sb, p.batch, (unsigned long long*)c.cursor.p, c.bufA.p,
                                   p.scatter_s, st),
         "owner scatter launch");
  tm.mark(ST_SCATTER);
  hipchk(kc::launch_split_hist(p.words, c.bufA.p, (kc::SplitItem*)c.items.p, dstate, p.max_items,
                               (kc::SplitBin*)c.bins.p, (unsigned long long*)c.subhist.p, ncls,
                               p.max_leaves, st),
         "split histogram launch");
  tm.mark(ST_SPLIT_HIST);
  hipchk(kc::launch_plan_leaves((unsigned long long*)c.hist.p, (unsigned long long*)c.sbegin.p,
                                (kc::SplitBin*)c.bins.p, p.sb, (unsigned long long*)c.subhist.p,
                                (kc::Leaf*)c.leaves.p, (unsigned long long*)c.cursor2.p,
                                p.merge_cshift, ncls, p.max_leaves, st),
         "plan_leaves launch");
  hipchk(kc::launch_split_scatter(p.words, c.bufA.p, c.bufB.p, (kc::SplitItem*)c.items.p, dstate,
                                  p.max_items, (kc::SplitBin*)c.bins.p,
                                  (unsigned long long*)c.cursor2.p, p.split_r, p.merge_cshift,
                                  ncls, p.max_leaves, st),
         "split scatter launch");
  if (p.merge_cshift)
    hipchk(kc::launch_leaf_ends((kc::Leaf*)c.leaves.p, (unsigned long long*)c.cursor2.p, dstate,
                                p.max_leaves, st),
           "leaf ends launch");
  tm.mark(ST_SPLIT);
  hipchk(kc::launch_leaf_small(p.words, p.keybits, c.bufA.p, c.bufB.p, (uint32_t*)c.tmpcnt.p,
                               (kc::Leaf*)c.leaves.p, dstate, p.max_leaves, (uint32_t*)c.dcnt.p,
                               (uint32_t*)c.large.p, (uint32_t*)c.ovfl.p, p.slots_log2, st,
                               p.mode, false, p.merge_cshift != 0),
         "leaf count launch");
  tm.mark(ST_LEAF_SMALL);
  hipchk(kc::launch_leaf_large(p.words, p.keybits, c.bufA.p, c.bufB.p, (uint32_t*)c.tmpcnt.p,
                               (kc::Leaf*)c.leaves.p, dstate, p.max_leaves, (uint32_t*)c.dcnt.p,
                               p.slots_log2, (uint32_t*)c.large.p, (uint32_t*)c.ovfl.p, st,
                               p.mode, false, p.merge_cshift != 0),
         "leaf count launch");
  tm.mark(ST_LEAF);
  hipchk(kc::launch_leaf_second(p.words, p.keybits, c.bufA.p, c.bufB.p, (uint32_t*)c.tmpcnt.p,
                                (kc::Leaf*)c.leaves.p, dstate, (uint32_t*)c.dcnt.p, p.slots_log2,
                                (uint32_t*)c.ovfl.p, st, p.mode, p.merge_cshift != 0),
         "leaf count launch");
  tm.mark(ST_LEAF_SECOND);
  hipchk(kc::launch_plan_out((uint32_t*)c.dcnt.p, dstate, (unsigned long long*)c.bsum.p,
                             p.max_leaves, (unsigned long long*)c.outoff.p, st),
         "plan_out launch");
  tm.mark(ST_OUT);
  if (!out.concat) return;
  if (out.set)
    hipchk(kc::launch_concat_batch(p.words, c.bufA.p, c.bufB.p, (uint32_t*)c.tmpcnt.p,
                                   (kc::Leaf*)c.leaves.p, (uint32_t*)c.dcnt.p,
                                   (unsigned long long*)c.outoff.p, dstate, p.max_leaves, out.cap,
                                   p.k, out.keys, out.counts, out.set, st),
           "concat launch");
  else
    hipchk(kc::launch_concat(p.words, c.bufA.p, c.bufB.p, (uint32_t*)c.tmpcnt.p,
                             (kc::Leaf*)c.leaves.p, (uint32_t*)c.dcnt.p,
                             (unsigned long long*)c.outoff.p, dstate, p.max_leaves, out.cap,
                             out.keys, out.counts, st),
           "concat launch");
  tm.mark(ST_CONCAT);
}

// Leaf table size and leaf size targets from the options.
void table_params(const kc_options& o, int words, int& slots_log2, uint64_t& C, uint64_t& T,
                  uint64_t& H) {
  const int max_slots = kc::max_leaf_slots_log2(words);
  slots_log2 = o.table_slots_log2 > 0 ? std::min(std::max(o.table_slots_log2, 10), max_slots)
                                      : max_slots;
  C = 1ull << slots_log2;
  // default leaf size in records. One-word keys: 1.5 tables, so that a leaf
  // fits its table while at most 58% of its records are distinct (on
  // 1,000,000 reads at k = 31 / 21: 2.76 / 2.71 ms per call against 3.05 /
  // 3.00 ms at three quarters of a table, no overflow; the per-leaf work of
  // clearing, compacting and sorting the table is spread over more records).
  // Wider keys, mostly distinct: three quarters of the largest table (1.5
  // tables overflowed 122 leaves at k = 55 and 8,896 at k = 100: 5.35 and
  // 59.1 ms against 4.68 and 8.4 ms). The sort-based leaves (mode 1) sort
  // all their records in LDS, so they keep three quarters of a table too
  // (1.5 tables: 39 ms against 12 ms on the 1,000,000 reads).
  const bool big = words == 1 && o.mode != 1;
  T = o.leaf_target > 0 ? (uint64_t)o.leaf_target : (big ? (C * 3) / 2 : (C * 3) / 4);
  H = o.leaf_attempt > 0 ? (uint64_t)o.leaf_attempt : (C * 7) / 8;
}

int shard_bits_for(const kc_options& o, int P, uint64_t rec_bound, uint64_t T, int keybits) {
  int sb = o.shard_bits;
  if (sb <= 0) {
    sb = std::max(8, ceil_log2((uint64_t)P));
    sb = std::max(sb, ceil_log2(rec_bound / (T << kc::kSplitMaxBits) + 1));
  }
  sb = std::min(sb, kc::max_shard_bits());
  return std::max(1, std::min(sb, keybits));
}

// The pipeline of a plain call over n_bytes bytes.
Pipe plain_pipe(uint64_t n_bytes, int k, int P, const kc_options& o) {
  Pipe p;
  p.words = k <= 32 ? 1 : (k <= 64 ? 2 : 4);
  p.k = k;
  p.keybits = 2 * k;
  uint64_t C = 0;
  table_params(o, p.words, p.slots_log2, C, p.T, p.H);
  p.sb = shard_bits_for(o, P, n_bytes, p.T, p.keybits);
  // two-word keys: one more shard bit shortens the split's runs more than it
  // lengthens the owner scatter's (measured: 4.67 against 4.77 ms at k = 55,
  // 1,000,000 reads of 150 bp)
  if (p.words == 2 && o.shard_bits <= 0) p.sb = std::min(std::max(p.sb, 9), kc::max_shard_bits());
  p.byte_begin = 0;
  p.byte_end = n_bytes;
  p.rec_bound = n_bytes;  // byte count: an upper bound of the window count
  p.mode = o.mode;
  tile_params(o, p);
  if (o.preagg < 0 || o.preagg > 2) fail(KC_E_INVAL, "preagg must be 0, 1 or 2");
  // a record's count (up to 16) takes the bits from 2k - shard bits up, which
  // the shard makes redundant: 4 of them at least
  const int cshift = p.keybits - p.sb;
  if (p.words == 1 && p.split_r == 16 && o.preagg == 1 && cshift <= 60) p.merge_cshift = cshift;
  pipe_bounds(p);
  return p;
}

// Owner-major shard order on the device, cached in the context per (P, sb).
const int* device_order(Ctx& c, const Call& q, kc_stats& S, hipStream_t st) {
  if (c.order_P != q.P || c.order_sb != q.sb) {
    grow(c.order, (size_t)q.nb * 4, "owner order", st);
    const std::vector<int>& order = owner_order(c, q, S, nullptr);
    c.order_host.assign(order.begin(), order.end());
    upload_sync(c.order.p, c.order_host.data(), (size_t)q.nb * 4, st);
    c.order_P = q.P;
    c.order_sb = q.sb;
  }
  return (const int*)c.order.p;
}

// fixed: the context of an allocation-free call (buffers carved from the
// static scratch), instead of the calling thread's arena.
int count_impl(const uint8_t* reads, const uint64_t* offsets, uint64_t n_reads, int k, int P,
               uint64_t* out_keys, uint32_t* out_counts, uint64_t cap, uint64_t* n_out,
               const kc_options* opt, hipStream_t st, const kc::OutAlloc* oa = nullptr,
               Ctx* fixed = nullptr) {
  auto t_host0 = std::chrono::steady_clock::now();
  if (!n_out) fail(KC_E_INVAL, "n_out is NULL");
  *n_out = 0;
  if (k < 1 || k > 128) fail(KC_E_INVAL, "k must be in [1, 128]");
  if (P < 1) fail(KC_E_INVAL, "P must be >= 1");
  if (!offsets) fail(KC_E_INVAL, "offsets is NULL");
  if (n_reads && !reads) fail(KC_E_INVAL, "reads is NULL");
  if (cap && (!out_keys || !out_counts)) fail(KC_E_INVAL, "output pointer is NULL");
  Call q{reads, offsets, n_reads, k, P, out_keys, out_counts, cap, {}, st, oa};
  std::memset(&q.o, 0, sizeof(q.o));
  if (opt) q.o = *opt;
  if (q.o.mode != 0 && q.o.mode != 1) fail(KC_E_INVAL, "mode must be 0 or 1");

  if (!fixed && g_have_orphans.load(std::memory_order_relaxed)) free_orphans();
  Ctx& c = fixed ? *fixed : context();
  // an allocation-free call is synchronous and records no event or timing
  std::optional<CtxUse> use;
  if (!fixed) use.emplace(c, st);
  std::memset(&g_stats, 0, sizeof(g_stats));
  kc_stats S;
  std::memset(&S, 0, sizeof(S));
  Timer tm(c, st, q.o.timing != 0 && !fixed);

  // ---- offsets: first/last, monotonicity (host sync 1 of 2)
  grow(c.state, sizeof(kc::DevState), "device state", st);
  hipchk(kc::launch_fill_u64((unsigned long long*)c.state.p, sizeof(kc::DevState) / 8, 0, st),
         "fill launch");
  if (n_reads) {
    const unsigned g = (unsigned)((n_reads + 255) / 256);
    hipLaunchKernelGGL(k_offsets_ok, dim3(g), dim3(256), 0, st, offsets, n_reads,
                       &((kc::DevState*)c.state.p)->overflow);
    hipchk(hipGetLastError(), "offsets check launch");
  }
  uint64_t* h = (uint64_t*)host_stage(c, 64);
  hipchk(hipMemcpyAsync(h, offsets, 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
  hipchk(hipMemcpyAsync(h + 1, offsets + n_reads, 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
  hipchk(hipMemcpyAsync(h + 2, &((kc::DevState*)c.state.p)->overflow, 4, hipMemcpyDeviceToHost,
                        st),
         "hipMemcpyAsync");
  hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
  const uint64_t off0 = h[0], offn = h[1];
  if ((uint32_t)h[2] != 0 || offn < off0) fail(KC_E_INVAL, "offsets must be non-decreasing");
  q.off0 = off0;
  q.N = offn - off0;
  S.n_bases = q.N;
  if (q.N == 0) {
    g_stats = S;
    return KC_OK;
  }
  const Pipe p0 = plain_pipe(q.N, k, P, q.o);
  q.words = p0.words;
  q.keybits = p0.keybits;
  q.ksz = 8 * q.words;
  table_params(q.o, q.words, q.slots_log2, q.C, q.T, q.H);
  q.sb = p0.sb;
  q.nb = 1 << q.sb;
  q.split_r = p0.split_r;
  q.merged = p0.merge_cshift != 0;
  if (q.o.refine_bits < 0 || q.o.refine_bits > 8) fail(KC_E_INVAL, "refine_bits must be in [0, 8]");
  Pipe p = p0;
  const uint64_t nchunks = packed_chunks(q.N);
  if (fixed) {
    // the input must fit the fixed scratch before anything is carved from it
    size_t need = 0;
    plain_needs(p, [&](DevBuf Ctx::*, size_t bytes, const char*) {
      need += (std::max<size_t>(bytes, 256) + 255) & ~(size_t)255;
    });
    if (need > g_carve->cap - g_carve->used)
      fail(KC_E_NOMEM, "kc_count_noalloc: an input of " + std::to_string(q.N) + " bytes at k = " +
                           std::to_string(k) + " needs " + std::to_string(need) +
                           " bytes of device scratch; its fixed scratch holds " +
                           std::to_string(kNoAllocScratchBytes) + " bytes");
  }
  plain_needs(p, [&](DevBuf Ctx::*m, size_t bytes, const char* name) { grow(c.*m, bytes, name, st); });
  p.order = device_order(c, q, S, st);
  kc::DevState* dstate = (kc::DevState*)c.state.p;

  tm.mark(ST_NONE);
  hipchk(kc::launch_pack(reads + off0, q.N, offsets, n_reads, off0, (uint64_t*)c.packed.p,
                         (uint64_t*)c.inv.p, (uint64_t*)c.endm.p, nchunks, st),
         "pack launch");
  tm.mark(ST_PACK);
  enqueue_pipeline(c, p, dstate, tm, PipeOut{out_keys, out_counts, nullptr, cap, !oa}, st);
  q.concat_leaves = p.max_leaves;
  kc::DevState ds = read_state(c, st);  // host sync 2 of 2 (3 with an output allocator)
  S.n_levels = 1;
  S.n_leaves = ds.n_leaves;
  // the block-wide leaf kernel's own launch (refinement launches are counted apart)
  S.large_records = ds.large_records;
  S.large_distinct = ds.large_distinct;
  S.second_records = ds.second_records;
  S.second_distinct = ds.second_distinct;
  if (ds.overflow) {
    // some leaves had more distinct keys than their tables hold: partition
    // those further and count their parts
    refine_overflowed(c, q, S, tm, ds.n_leaves, p.max_leaves);
    ds = read_state(c, st);
    if (ds.overflow) fail(KC_E_INTERNAL, "leaf overflow after refinement");
  }
  S.valid_windows = ds.W;
  S.distinct = ds.D;
  S.refined_records =
      ds.large_records + ds.second_records - S.large_records - S.second_records;
  if (ds.count_overflow) fail(KC_E_OVERFLOW, "a k-mer occurs more than 2^32-1 times");
  if (oa) {
    const int r = oa->fn(oa->user, ds.D, q.words, &out_keys, &out_counts);
    if (r != KC_OK) fail(r, "output allocation of " + std::to_string(ds.D) + " pairs failed");
    cap = ds.D;
    tm.mark(ST_NONE);
    hipchk(kc::launch_concat(q.words, c.bufA.p, c.bufB.p, (uint32_t*)c.tmpcnt.p,
                             (kc::Leaf*)c.leaves.p, (uint32_t*)c.dcnt.p,
                             (unsigned long long*)c.outoff.p, dstate, q.concat_leaves, cap,
                             out_keys, out_counts, st),
           "concat launch");
    tm.mark(ST_CONCAT);
  }
  if (ds.D > cap) {
    *n_out = ds.D;
    fail(KC_E_CAPACITY, "output capacity " + std::to_string(cap) + " < " + std::to_string(ds.D) +
                            " distinct k-mers");
  }
  if (q.o.check) {
    hipchk(kc::launch_fill_u64((unsigned long long*)&dstate->check, sizeof(kc::CheckResult) / 8,
                               0, st),
           "fill launch");
    hipchk(kc::launch_check(q.words, out_keys, out_counts, ds.D, k, &dstate->check, st),
           "check launch");
    tm.mark(ST_CHECK);
    const kc::DevState d2 = read_state(c, st);
    const kc::CheckResult& r = d2.check;
    if (r.sum_counts != ds.W || r.not_sorted || r.not_canonical || r.out_of_range ||
        r.zero_count) {
      char msg[256];
      std::snprintf(msg, sizeof msg,
                    "device self-check failed: sum %llu (want %llu), unsorted %u, "
                    "non-canonical %u, out of range %u, zero counts %u",
                    r.sum_counts, (unsigned long long)ds.W, r.not_sorted, r.not_canonical,
                    r.out_of_range, r.zero_count);
      fail(KC_E_INTERNAL, msg);
    }
  }
  if (oa || fixed) hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
  tm.collect(S);
  *n_out = ds.D;
  S.ms_total =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_host0).count();
  g_stats = S;
  return KC_OK;
}

void free_buf(DevBuf& b) { drop(b); }

}  // namespace

// A planned batch of read sets (opaque in the C ABI): the sets are cut into
// memory waves of consecutive sets, each counted by one recorded graph.
struct kc_batch {
  int device = 0;
  uint32_t n_sets = 0;
  int P = 1;
  kc_options o{};
  uint64_t hbm_budget = 0;
  uint64_t n_reads = 0, N = 0;
  std::vector<unsigned long long> set_first_read, set_byte_off;  // whole batch, n_sets + 1 each
  std::vector<int> ks;
  struct Class {
    int k = 0, set_bits = 0;
    std::vector<uint32_t> sets;  // wave-local set indices
    Pipe pipe;
    uint64_t out_base = 0, out_cap = 0, start_base = 0;
    DevBuf order, set_local;
    kc::BatchSets bs{};
  };
  struct Wave {
    uint32_t s0 = 0, ns = 0;      // sets [s0, s0 + ns)
    uint64_t r0 = 0, nr = 0;      // their reads
    uint64_t b0 = 0, nbytes = 0;  // their bytes
    uint64_t need = 0;            // device bytes planned for the wave
    std::vector<unsigned long long> first_read, byte_off;  // wave-relative, ns + 1 each
    std::vector<Class> cls;
    uint64_t out_total = 0, starts_total = 0;
    DevBuf first_read_dev, byte_off_dev, set_class_dev, set_local_dev, starts, start_base_dev,
        class_base_dev, states;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void* key[5] = {};
    uint64_t key_cap = 0, key_off0 = 0;
    kc_stats stats{};
  };
  std::vector<Wave> waves;
  Ctx ctx;  // pipeline buffers, shared by the waves (sized for the largest)
  DevBuf cls_keys, cls_counts, cls_set, set_off, flag;
  hipStream_t cap_stream = nullptr;
  kc_stats stats{};

  ~kc_batch() {
    int prev = -1;
    if (hipGetDevice(&prev) == hipSuccess) (void)hipSetDevice(device);
    for (Wave& w : waves) {
      if (w.exec) (void)hipGraphExecDestroy(w.exec);
      if (w.graph) (void)hipGraphDestroy(w.graph);
      for (Class& c : w.cls) {
        free_buf(c.order);
        free_buf(c.set_local);
      }
      DevBuf* wb[] = {&w.first_read_dev, &w.byte_off_dev, &w.set_class_dev, &w.set_local_dev,
                      &w.starts,        &w.start_base_dev, &w.class_base_dev, &w.states};
      for (DevBuf* b : wb) free_buf(*b);
    }
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    DevBuf* all[] = {&cls_keys, &cls_counts, &cls_set, &set_off, &flag};
    for (DevBuf* b : all) free_buf(*b);
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

namespace {

// Device bytes of one batch pipeline over `bytes` bytes of sets of one k with
// up to `n_sets` sets in a class (keys widen to two words when the set id
// bits and 2k pass 64 bits).
uint64_t class_pipe_bytes(uint64_t bytes, int k, uint64_t n_sets, const kc_options& o) {
  if (bytes == 0) return 0;
  Pipe p;
  p.k = k;
  p.keybits = 2 * k + ceil_log2(std::max<uint64_t>(n_sets, 1));
  p.words = p.keybits > 64 ? 2 : 1;
  uint64_t C;
  table_params(o, p.words, p.slots_log2, C, p.T, p.H);
  p.sb = kc::max_shard_bits();
  p.rec_bound = bytes;
  pipe_bounds(p);
  uint64_t t = 0;
  pipeline_needs(p, [&](DevBuf Ctx::*, size_t b, const char*) { t += alloc_size(b); });
  return t;
}

// Device bytes a wave holds: packed input, class outputs (key, count, set id
// per byte of input at most), the largest class pipeline, per-set tables.
uint64_t wave_bytes(uint64_t bytes, const std::map<int, std::pair<uint64_t, uint64_t>>& by_k,
                    uint64_t n_sets, const kc_options& o) {
  uint64_t pipe = 0;
  for (const auto& kv : by_k)
    pipe = std::max(pipe, class_pipe_bytes(kv.second.first, kv.first, kv.second.second, o));
  return packed_chunks(bytes) * 40 + alloc_size(bytes * 16) + pipe + n_sets * 96 + (1 << 20);
}

// Classes of a wave: sets of one k counted together with keys (set id << 2k)
// | k-mer. Every set of a class gets the same share of the first-level shards,
// so a class holds at most as many sets as its largest set can afford: the
// sets of each k are taken largest first, and a class is closed once
// 2^set_bits sets are in it, set_bits being the most that still leaves the
// largest set enough shards for leaves of the target size (at half of full
// use).
void form_classes(kc_batch* b, kc_batch::Wave& w, const uint64_t* set_bytes) {
  std::vector<int> kv;
  for (uint32_t s = 0; s < w.ns; ++s) kv.push_back(b->ks[w.s0 + s]);
  std::sort(kv.begin(), kv.end());
  kv.erase(std::unique(kv.begin(), kv.end()), kv.end());
  for (int k : kv) {
    std::vector<uint32_t> sk;
    for (uint32_t s = 0; s < w.ns; ++s)
      if (b->ks[w.s0 + s] == k) sk.push_back(s);
    std::stable_sort(sk.begin(), sk.end(), [&](uint32_t x, uint32_t y) {
      return set_bytes[w.s0 + x] > set_bytes[w.s0 + y];
    });
    int slots_log2;
    uint64_t Cs, Tw, Hw;
    table_params(b->o, 2, slots_log2, Cs, Tw, Hw);  // the smaller (two-word) leaf target
    const uint64_t per_shard = (Tw << kc::kSplitMaxBits) / 2;
    size_t i = 0;
    while (i < sk.size()) {
      const uint64_t wb = std::max<uint64_t>(set_bytes[w.s0 + sk[i]], 1);
      int need = 0;  // shard bits the largest set needs
      while (need < kc::kMaxShardBits && ((uint64_t)per_shard << need) < wb) ++need;
      int sbits = std::max(0, kc::kMaxShardBits - need);
      sbits = std::min(sbits, 128 - 2 * k);
      const size_t take = std::min(sk.size() - i, (size_t)1 << sbits);
      kc_batch::Class C;
      C.k = k;
      C.sets.assign(sk.begin() + i, sk.begin() + i + take);
      std::sort(C.sets.begin(), C.sets.end());  // set order inside a class
      w.cls.push_back(std::move(C));
      i += take;
    }
  }
}

int batch_plan_impl(const uint64_t* host_set_reads, const uint64_t* host_set_bytes,
                    const int* host_ks, uint32_t n_sets, int P, uint64_t hbm_budget,
                    const kc_options* opt, kc_batch** out) {
  if (!out) fail(KC_E_INVAL, "plan pointer is NULL");
  *out = nullptr;
  if (!host_set_reads || !host_set_bytes || !host_ks || n_sets == 0)
    fail(KC_E_INVAL, "batch needs at least one set and host arrays");
  if (P < 1) fail(KC_E_INVAL, "P must be >= 1");
  std::unique_ptr<kc_batch> b(new kc_batch());
  hipchk(hipGetDevice(&b->device), "hipGetDevice");
  b->n_sets = n_sets;
  b->P = P;
  b->hbm_budget = hbm_budget;
  std::memset(&b->o, 0, sizeof(b->o));
  if (opt) b->o = *opt;
  if (b->o.mode != 0) fail(KC_E_INVAL, "mode must be 0 for a batch");
  b->ks.assign(host_ks, host_ks + n_sets);
  b->set_first_read.assign(n_sets + 1, 0);
  b->set_byte_off.assign(n_sets + 1, 0);
  for (uint32_t s = 0; s < n_sets; ++s) {
    if (b->ks[s] < 1 || b->ks[s] > 32) fail(KC_E_INVAL, "batched counting takes 1 <= k <= 32");
    b->set_first_read[s + 1] = b->set_first_read[s] + host_set_reads[s];
    b->set_byte_off[s + 1] = b->set_byte_off[s] + host_set_bytes[s];
  }
  b->n_reads = b->set_first_read[n_sets];
  b->N = b->set_byte_off[n_sets];

  // Memory waves: consecutive sets, as many as keep the wave's device bytes
  // within the budget (0 = no budget: one wave).
  {
    uint32_t s0 = 0;
    uint64_t bytes = 0;
    std::map<int, std::pair<uint64_t, uint64_t>> by_k;  // k -> (bytes, sets)
    uint64_t need = 0;
    auto close = [&](uint32_t s1) {
      kc_batch::Wave w;
      w.s0 = s0;
      w.ns = s1 - s0;
      w.need = need;
      b->waves.push_back(std::move(w));
      s0 = s1;
      bytes = 0;
      by_k.clear();
      need = 0;
    };
    for (uint32_t s = 0; s < n_sets; ++s) {
      auto trial = by_k;
      trial[b->ks[s]].first += host_set_bytes[s];
      trial[b->ks[s]].second += 1;
      const uint64_t nt = wave_bytes(bytes + host_set_bytes[s], trial, s - s0 + 1, b->o);
      if (hbm_budget && nt > hbm_budget && s > s0) {
        close(s);
        trial.clear();
        trial[b->ks[s]] = {host_set_bytes[s], 1};
      }
      by_k = std::move(trial);
      bytes += host_set_bytes[s];
      need = wave_bytes(bytes, by_k, s - s0 + 1, b->o);
      if (hbm_budget && need > hbm_budget)
        fail(KC_E_NOMEM, "set " + std::to_string(s) + " alone needs " + std::to_string(need) +
                             " device bytes, more than the batch budget of " +
                             std::to_string(hbm_budget));
    }
    close(n_sets);
  }

  Ctx& c = b->ctx;
  c.device = b->device;
  hipStream_t st = nullptr;
  uint64_t max_bytes = 0, max_out = 0, max_ns = 0;
  for (kc_batch::Wave& w : b->waves) {
    w.r0 = b->set_first_read[w.s0];
    w.nr = b->set_first_read[w.s0 + w.ns] - w.r0;
    w.b0 = b->set_byte_off[w.s0];
    w.nbytes = b->set_byte_off[w.s0 + w.ns] - w.b0;
    w.first_read.assign(w.ns + 1, 0);
    w.byte_off.assign(w.ns + 1, 0);
    for (uint32_t s = 0; s <= w.ns; ++s) {
      w.first_read[s] = b->set_first_read[w.s0 + s] - w.r0;
      w.byte_off[s] = b->set_byte_off[w.s0 + s] - w.b0;
    }
    form_classes(b.get(), w, host_set_bytes);
    std::vector<uint32_t> set_class(w.ns), set_local(w.ns);
    uint64_t out_base = 0, start_base = 0;
    std::vector<unsigned long long> sbase(w.cls.size()), cbase(w.cls.size());
    kc_stats dummy;
    std::memset(&dummy, 0, sizeof(dummy));
    for (size_t ci = 0; ci < w.cls.size(); ++ci) {
      kc_batch::Class& C = w.cls[ci];
      uint64_t bytes = 0, lo = ~0ull, hi = 0;
      for (size_t j = 0; j < C.sets.size(); ++j) {
        const uint32_t s = C.sets[j];
        set_class[s] = (uint32_t)ci;
        set_local[s] = (uint32_t)j;
        bytes += host_set_bytes[w.s0 + s];
        lo = std::min<uint64_t>(lo, w.byte_off[s]);
        hi = std::max<uint64_t>(hi, w.byte_off[s + 1]);
      }
      C.set_bits = ceil_log2(C.sets.size());
      Pipe& p = C.pipe;
      p.k = C.k;
      p.keybits = 2 * C.k + C.set_bits;
      p.words = p.keybits > 64 ? 2 : 1;
      uint64_t Cslots;
      table_params(b->o, p.words, p.slots_log2, Cslots, p.T, p.H);
      p.rec_bound = std::max<uint64_t>(bytes, 1);
      p.sb = b->o.shard_bits > 0 ? std::min(b->o.shard_bits, kc::max_shard_bits())
                                 : std::max(shard_bits_for(b->o, P, p.rec_bound, p.T, p.keybits),
                                            std::min(kc::max_shard_bits(), C.set_bits + 3));
      p.sb = std::max(1, std::min(p.sb, p.keybits));
      p.byte_begin = lo & ~31ull;
      p.byte_end = hi;
      tile_params(b->o, p);
      pipe_bounds(p);
      pipeline_prepare(c, p);
      C.out_base = out_base;
      C.out_cap = p.rec_bound;
      out_base += C.out_cap;
      C.start_base = start_base;
      start_base += C.sets.size() + 1;
      sbase[ci] = C.start_base;
      cbase[ci] = C.out_base;
      // owner order of the class's shards and its set ids
      std::vector<uint32_t> loc(w.ns, kc::kNoSet);
      for (size_t j = 0; j < C.sets.size(); ++j) loc[C.sets[j]] = (uint32_t)j;
      ensure(C.set_local, w.ns * 4, "batch tables");
      upload_sync(C.set_local.p, loc.data(), w.ns * 4, st);
      Call q{};
      q.P = P;
      q.sb = p.sb;
      q.nb = 1 << p.sb;
      const std::vector<int>& order = owner_order(c, q, dummy, nullptr);
      ensure(C.order, (size_t)q.nb * 4, "owner order");
      upload_sync(C.order.p, order.data(), (size_t)q.nb * 4, st);
      p.order = (const int*)C.order.p;
    }
    w.out_total = out_base;
    w.starts_total = start_base;
    ensure(w.first_read_dev, (w.ns + 1) * 8, "batch tables");
    ensure(w.byte_off_dev, (w.ns + 1) * 8, "batch tables");
    ensure(w.set_class_dev, w.ns * 4, "batch tables");
    ensure(w.set_local_dev, w.ns * 4, "batch tables");
    ensure(w.starts, start_base * 8, "set bounds");
    ensure(w.start_base_dev, w.cls.size() * 8, "batch tables");
    ensure(w.class_base_dev, w.cls.size() * 8, "batch tables");
    ensure(w.states, w.cls.size() * sizeof(kc::DevState), "device states");
    upload_sync(w.first_read_dev.p, w.first_read.data(), (w.ns + 1) * 8, st);
    upload_sync(w.byte_off_dev.p, w.byte_off.data(), (w.ns + 1) * 8, st);
    upload_sync(w.set_class_dev.p, set_class.data(), w.ns * 4, st);
    upload_sync(w.set_local_dev.p, set_local.data(), w.ns * 4, st);
    upload_sync(w.start_base_dev.p, sbase.data(), w.cls.size() * 8, st);
    upload_sync(w.class_base_dev.p, cbase.data(), w.cls.size() * 8, st);
    for (kc_batch::Class& C : w.cls) {
      C.bs = kc::BatchSets{(const unsigned long long*)w.byte_off_dev.p,
                           (const uint32_t*)C.set_local.p, w.ns};
      C.pipe.batch = &C.bs;
    }
    max_bytes = std::max(max_bytes, w.nbytes);
    max_out = std::max(max_out, w.out_total);
    max_ns = std::max<uint64_t>(max_ns, w.ns);
  }
  const uint64_t nchunks = packed_chunks(max_bytes);
  ensure(c.packed, nchunks * 16, "packed bases");
  ensure(c.inv, nchunks * 8, "invalid mask");
  ensure(c.endm, nchunks * 8, "end mask");
  ensure(c.valid, nchunks * 8, "valid-start mask");
  ensure(c.state, sizeof(kc::DevState), "device state");
  ensure(b->cls_keys, max_out * 8, "class outputs");
  ensure(b->cls_counts, max_out * 4, "class outputs");
  ensure(b->cls_set, max_out * 4, "class outputs");
  ensure(b->set_off, (max_ns + 1) * 8, "set offsets");
  ensure(b->flag, 64, "flags");
  *out = b.release();
  return KC_OK;
}

// Per-set plain counts of the sets of a wave (used when a class overflowed);
// set_off receives w.ns + 1 wave-relative offsets.
void wave_by_sets(kc_batch* b, const kc_batch::Wave& w, const uint8_t* reads,
                  const uint64_t* offsets, uint64_t* out_keys, uint32_t* out_counts, uint64_t cap,
                  uint64_t* set_off, uint64_t* n_out, hipStream_t st) {
  uint64_t o = 0;
  bool short_cap = false;
  for (uint32_t s = 0; s < w.ns; ++s) {
    set_off[s] = o;
    uint64_t n = 0;
    const uint64_t r0 = w.first_read[s], r1 = w.first_read[s + 1];
    const int rc = count_impl(reads, offsets + r0, r1 - r0, b->ks[w.s0 + s], b->P,
                              short_cap ? nullptr : out_keys + o,
                              short_cap ? nullptr : out_counts + o,
                              short_cap || o > cap ? 0 : cap - o, &n, &b->o, st);
    if (rc == KC_E_CAPACITY) {
      // keep counting the sizes so that the caller learns the total needed
      o += n;
      short_cap = true;
      continue;
    }
    if (rc != KC_OK) throw Fail{rc};
    o += n;
  }
  set_off[w.ns] = o;
  *n_out = o;
}

// Runs wave wi on its own reads (offsets: its w.nr + 1 read offsets), writes
// its pairs to out (cap entries) and w.ns + 1 wave-relative set offsets.
// Returns the number of pairs; pairs past cap are not written.
uint64_t run_wave(kc_batch* b, uint32_t wi, const uint8_t* reads, const uint64_t* offsets,
                  uint64_t* out_keys, uint32_t* out_counts, uint64_t cap, uint64_t* host_set_off,
                  hipStream_t st) {
  auto t0 = std::chrono::steady_clock::now();
  kc_batch::Wave& w = b->waves[wi];
  Ctx& c = b->ctx;
  // inputs must have the layout the plan describes
  hipchk(kc::launch_fill_u64((unsigned long long*)b->flag.p, 8, 0, st), "fill launch");
  if (w.nr) {
    hipLaunchKernelGGL(k_offsets_ok, dim3((unsigned)((w.nr + 255) / 256)), dim3(256), 0, st,
                       offsets, w.nr, (unsigned int*)b->flag.p);
    hipchk(hipGetLastError(), "offsets check launch");
  }
  hipLaunchKernelGGL(k_batch_layout_ok, dim3((w.ns + 256) / 256), dim3(256), 0, st, offsets,
                     (const unsigned long long*)w.first_read_dev.p,
                     (const unsigned long long*)w.byte_off_dev.p, w.ns, (unsigned int*)b->flag.p);
  hipchk(hipGetLastError(), "layout check launch");
  uint64_t* h = (uint64_t*)host_stage(c, 64);
  hipchk(hipMemcpyAsync(h, offsets, 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
  hipchk(hipMemcpyAsync(h + 1, b->flag.p, 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
  hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
  const uint64_t off0 = h[0];
  if (h[1] != 0) fail(KC_E_INVAL, "reads and offsets do not match the batch plan");
  const void* key[5] = {reads, offsets, out_keys, out_counts, nullptr};
  const bool same = std::equal(key, key + 5, w.key) && w.key_cap == cap && w.key_off0 == off0;
  if (!w.exec || !same) {
    if (w.exec) (void)hipGraphExecDestroy(w.exec);
    if (w.graph) (void)hipGraphDestroy(w.graph);
    w.exec = nullptr;
    w.graph = nullptr;
    if (!b->cap_stream)
      hipchk(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
    hipStream_t cs = b->cap_stream;
    hipchk(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    try {
      Timer off(c, cs, false);
      const size_t nst = w.cls.size();
      hipchk(kc::launch_fill_u64((unsigned long long*)w.states.p, nst * sizeof(kc::DevState) / 8,
                                 0, cs),
             "fill launch");
      const uint64_t nchunks = packed_chunks(w.nbytes);
      hipchk(kc::launch_pack(reads + off0, w.nbytes, offsets, w.nr, off0, (uint64_t*)c.packed.p,
                             (uint64_t*)c.inv.p, (uint64_t*)c.endm.p, nchunks, cs),
             "pack launch");
      for (size_t ci = 0; ci < nst; ++ci) {
        kc_batch::Class& C = w.cls[ci];
        kc::DevState* ds = (kc::DevState*)w.states.p + ci;
        PipeOut po{(uint64_t*)b->cls_keys.p + C.out_base, (uint32_t*)b->cls_counts.p + C.out_base,
                   (uint32_t*)b->cls_set.p + C.out_base, C.out_cap};
        enqueue_pipeline(c, C.pipe, ds, off, po, cs);
        hipchk(kc::launch_set_bounds(po.set, ds, C.out_cap, (uint32_t)C.sets.size(),
                                     (unsigned long long*)w.starts.p + C.start_base, cs),
               "set bounds launch");
      }
      hipchk(kc::launch_batch_offsets((const uint32_t*)w.set_class_dev.p,
                                      (const uint32_t*)w.set_local_dev.p,
                                      (const unsigned long long*)w.starts.p,
                                      (const unsigned long long*)w.start_base_dev.p, w.ns,
                                      (unsigned long long*)b->set_off.p, cs),
             "batch offsets launch");
      hipchk(kc::launch_batch_gather(
                 (const uint32_t*)w.set_class_dev.p, (const uint32_t*)w.set_local_dev.p,
                 (const unsigned long long*)w.starts.p,
                 (const unsigned long long*)w.start_base_dev.p,
                 (const unsigned long long*)w.class_base_dev.p, (const uint64_t*)b->cls_keys.p,
                 (const uint32_t*)b->cls_counts.p, (const unsigned long long*)b->set_off.p, w.ns,
                 cap, out_keys, out_counts, cs),
             "batch gather launch");
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(cs, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    hipchk(hipStreamEndCapture(cs, &w.graph), "hipStreamEndCapture");
    hipchk(hipGraphInstantiate(&w.exec, w.graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    std::copy(key, key + 5, w.key);
    w.key_cap = cap;
    w.key_off0 = off0;
  }
  hipchk(hipGraphLaunch(w.exec, st), "hipGraphLaunch");
  const size_t nst = w.cls.size();
  const size_t bytes = nst * sizeof(kc::DevState) + (w.ns + 1) * 8;
  char* hs = (char*)host_stage(c, bytes);
  hipchk(hipMemcpyAsync(hs, w.states.p, nst * sizeof(kc::DevState), hipMemcpyDeviceToHost, st),
         "hipMemcpyAsync");
  hipchk(hipMemcpyAsync(hs + nst * sizeof(kc::DevState), b->set_off.p, (w.ns + 1) * 8,
                        hipMemcpyDeviceToHost, st),
         "hipMemcpyAsync");
  hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
  std::memset(&w.stats, 0, sizeof(w.stats));
  bool overflow = false;
  for (size_t ci = 0; ci < nst; ++ci) {
    kc::DevState ds;
    std::memcpy(&ds, hs + ci * sizeof(kc::DevState), sizeof(ds));
    if (ds.count_overflow) fail(KC_E_OVERFLOW, "a k-mer occurs more than 2^32-1 times");
    overflow |= ds.overflow != 0;
    w.stats.valid_windows += ds.W;
    w.stats.distinct += ds.D;
    w.stats.n_leaves += ds.n_leaves;
    w.stats.large_records += ds.large_records;
    w.stats.large_distinct += ds.large_distinct;
    w.stats.second_records += ds.second_records;
    w.stats.second_distinct += ds.second_distinct;
  }
  w.stats.n_bases = w.nbytes;
  std::memcpy(host_set_off, hs + nst * sizeof(kc::DevState), (w.ns + 1) * 8);
  uint64_t D = host_set_off[w.ns];
  if (overflow) {
    // a class had a leaf too large for the device-planned split: count the
    // wave's sets one by one
    ++w.stats.n_overflow;
    wave_by_sets(b, w, reads, offsets, out_keys, out_counts, cap, host_set_off, &D, st);
    w.stats.distinct = D;
  }
  w.stats.ms_total =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return D;
}

int batch_run_wave_impl(kc_batch* b, uint32_t wi, const uint8_t* reads, const uint64_t* offsets,
                        uint64_t* out_keys, uint32_t* out_counts, uint64_t cap,
                        uint64_t* host_set_off, uint64_t* n_out, hipStream_t st) {
  if (!b || !n_out || !host_set_off) fail(KC_E_INVAL, "NULL argument");
  *n_out = 0;
  if (wi >= b->waves.size()) fail(KC_E_INVAL, "wave index out of range");
  if (!reads || !offsets) fail(KC_E_INVAL, "NULL input pointer");
  if (cap && (!out_keys || !out_counts)) fail(KC_E_INVAL, "output pointer is NULL");
  const uint64_t D = run_wave(b, wi, reads, offsets, out_keys, out_counts, cap, host_set_off, st);
  b->stats = b->waves[wi].stats;
  *n_out = D;
  if (D > cap)
    fail(KC_E_CAPACITY, "output capacity " + std::to_string(cap) + " < " + std::to_string(D) +
                            " pairs in the wave");
  return KC_OK;
}

int batch_run_impl(kc_batch* b, const uint8_t* reads, const uint64_t* offsets, uint64_t* out_keys,
                   uint32_t* out_counts, uint64_t cap, uint64_t* host_set_off, uint64_t* n_out,
                   hipStream_t st) {
  auto t0 = std::chrono::steady_clock::now();
  if (!b || !n_out || !host_set_off) fail(KC_E_INVAL, "NULL argument");
  *n_out = 0;
  if (!reads || !offsets) fail(KC_E_INVAL, "NULL input pointer");
  if (cap && (!out_keys || !out_counts)) fail(KC_E_INVAL, "output pointer is NULL");
  std::memset(&b->stats, 0, sizeof(b->stats));
  uint64_t base = 0;
  bool short_cap = false;
  std::vector<uint64_t> so;
  for (uint32_t wi = 0; wi < b->waves.size(); ++wi) {
    const kc_batch::Wave& w = b->waves[wi];
    so.assign(w.ns + 1, 0);
    // once the output is too small, the remaining waves only count their pairs
    const uint64_t room = short_cap || base > cap ? 0 : cap - base;
    const uint64_t D = run_wave(b, wi, reads, offsets + w.r0, room ? out_keys + base : nullptr,
                                room ? out_counts + base : nullptr, room, so.data(), st);
    if (D > room) short_cap = true;
    for (uint32_t s = 0; s <= w.ns; ++s) host_set_off[w.s0 + s] = base + so[s];
    base += D;
    const kc_stats& ws = w.stats;
    b->stats.n_bases += ws.n_bases;
    b->stats.valid_windows += ws.valid_windows;
    b->stats.distinct += ws.distinct;
    b->stats.n_leaves += ws.n_leaves;
    b->stats.n_overflow += ws.n_overflow;
    b->stats.large_records += ws.large_records;
    b->stats.large_distinct += ws.large_distinct;
    b->stats.second_records += ws.second_records;
    b->stats.second_distinct += ws.second_distinct;
  }
  *n_out = base;
  b->stats.ms_total =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (base > cap)
    fail(KC_E_CAPACITY, "output capacity " + std::to_string(cap) + " < " + std::to_string(base) +
                            " pairs in the batch");
  return KC_OK;
}

template <class F>
int guarded(F f) {
  g_err.clear();
  try {
    return f();
  } catch (const Fail& e) {
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return KC_E_NOMEM;
  } catch (...) {
    g_err = "unexpected C++ exception";
    return KC_E_INTERNAL;
  }
}

}  // namespace

namespace kc {

namespace {
std::mutex g_pool_m;
std::map<int, hipMemPool_t> g_pools;
}  // namespace

hipError_t device_pool(int device, hipMemPool_t* pool) {
  std::lock_guard<std::mutex> lk(g_pool_m);
  auto it = g_pools.find(device);
  if (it != g_pools.end()) {
    *pool = it->second;
    return hipSuccess;
  }
  hipMemPoolProps props;
  std::memset(&props, 0, sizeof(props));
  props.allocType = hipMemAllocationTypePinned;
  props.handleTypes = hipMemHandleTypeNone;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = device;
  hipMemPool_t p = nullptr;
  hipError_t e = hipMemPoolCreate(&p, &props);
  if (e != hipSuccess) return e;
  uint64_t keep = ~0ull;  // never hand idle blocks back on a synchronization
  e = hipMemPoolSetAttribute(p, hipMemPoolAttrReleaseThreshold, &keep);
  // a block freed on one stream is not reused on another before its free has
  // completed (no waits inserted between the server's streams)
  int no = 0;
  if (e == hipSuccess) e = hipMemPoolSetAttribute(p, hipMemPoolReuseAllowInternalDependencies, &no);
  if (e != hipSuccess) {
    (void)hipMemPoolDestroy(p);
    return e;
  }
  g_pools[device] = p;
  *pool = p;
  return hipSuccess;
}

void* thread_scratch(size_t bytes, hipStream_t st, std::string* err, int* code) noexcept {
  try {
    Ctx& c = context();
    grow(c.post, bytes, "merge and filter temporaries", st);
    return c.post.p;
  } catch (const Fail& f) {
    if (err) *err = g_err;
    if (code) *code = f.code;
  } catch (...) {
    if (err) *err = "merge and filter temporaries: allocation failed";
    if (code) *code = KC_E_NOMEM;
  }
  return nullptr;
}

void trim_device_pool(int device) {
  free_orphans();  // arenas of ended threads (a server's workers) first
  hipMemPool_t p = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_pool_m);
    auto it = g_pools.find(device);
    if (it == g_pools.end()) return;
    p = it->second;
  }
  // blocks freed on the null stream (released arenas) become idle first
  (void)hipStreamSynchronize(nullptr);
  (void)hipMemPoolTrimTo(p, 0);
}

int count_with_alloc(const uint8_t* reads, const uint64_t* offsets, uint64_t n_reads, int k,
                     int P, const kc_options* opt, hipStream_t st, const OutAlloc& oa,
                     uint64_t* n_out, kc_stats* stats, std::string* err) {
  const int r = guarded([&] {
    return count_impl(reads, offsets, n_reads, k, P, nullptr, nullptr, 0, n_out, opt, st, &oa);
  });
  if (r == KC_OK && stats) *stats = g_stats;
  if (r != KC_OK && err) *err = g_err;
  return r;
}

uint64_t scratch_bytes(uint64_t n_bytes, int k, int P, const kc_options* opt) {
  if (n_bytes == 0 || k < 1 || k > 128 || P < 1) return 0;
  kc_options o;
  std::memset(&o, 0, sizeof(o));
  if (opt) o = *opt;
  try {
    const Pipe p = plain_pipe(n_bytes, k, P, o);
    uint64_t need = 0;
    plain_needs(p, [&](DevBuf Ctx::*, size_t bytes, const char*) {
      need += (std::max<size_t>(bytes, 256) + 255) & ~(size_t)255;
    });
    // room for the lists and tables of a refinement
    return need + (16ull << 20) + need / 64;
  } catch (...) {
    return 0;
  }
}

void set_last_error(const std::string& msg) { g_err = msg; }

// ---- the server's slab

Slab* Slab::create(uint64_t bytes, std::string* err) {
  std::unique_ptr<Slab> s(new Slab());
  bytes = (bytes + 255) & ~255ull;
  void* p = nullptr;
  const hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    if (err) *err = std::string("device allocation of the server slab (") + std::to_string(bytes) +
                    " bytes) failed: " + hipGetErrorString(e);
    return nullptr;
  }
  s->base_ = (char*)p;
  s->cap_ = bytes;
  s->free_[0] = bytes;
  return s.release();
}

Slab::~Slab() {
  (void)hipDeviceSynchronize();  // nothing may still use the blocks
  for (Pending& q : pending_) (void)hipEventDestroy(q.ev);
  for (hipEvent_t e : events_) (void)hipEventDestroy(e);
  if (base_) (void)hipFree(base_);
}

void Slab::insert_free(uint64_t off, uint64_t size) {
  auto next = free_.lower_bound(off);
  if (next != free_.end() && off + size == next->first) {  // merge with the range after
    size += next->second;
    next = free_.erase(next);
  }
  if (next != free_.begin()) {
    auto prev = std::prev(next);
    if (prev->first + prev->second == off) {  // merge with the range before
      prev->second += size;
      return;
    }
  }
  free_[off] = size;
}

void Slab::reclaim(bool wait) {
  size_t j = 0;
  for (size_t i = 0; i < pending_.size(); ++i) {
    Pending& q = pending_[i];
    const hipError_t r = wait ? hipEventSynchronize(q.ev) : hipEventQuery(q.ev);
    if (r == hipSuccess) {
      insert_free(q.off, q.size);
      events_.push_back(q.ev);
    } else {
      if (r != hipErrorNotReady) (void)hipGetLastError();
      pending_[j++] = q;
    }
  }
  pending_.resize(j);
}

void* Slab::alloc(uint64_t bytes, bool high) {
  const uint64_t want = (std::max<uint64_t>(bytes, 256) + 255) & ~255ull;
  std::lock_guard<std::mutex> lk(m_);
  for (int attempt = 0; attempt < 2; ++attempt) {
    reclaim(attempt == 1);
    // best fit (the smallest free range that holds it; the lowest or highest
    // of equal ones), cut from its low or high end
    auto best = free_.end();
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < want) continue;
      if (best == free_.end() || it->second < best->second ||
          (it->second == best->second && high)) best = it;
    }
    if (best == free_.end()) continue;
    const uint64_t off = high ? best->first + best->second - want : best->first;
    const uint64_t rest = best->second - want;
    const uint64_t at = best->first;
    free_.erase(best);
    if (rest) {
      if (high) free_[at] = rest;
      else free_[off + want] = rest;
    }
    live_[off] = want;
    return base_ + off;
  }
  return nullptr;
}

void Slab::free(void* p, hipStream_t st) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(m_);
  const uint64_t off = (uint64_t)((char*)p - base_);
  auto it = live_.find(off);
  if (it == live_.end()) return;
  const uint64_t size = it->second;
  live_.erase(it);
  hipEvent_t ev = nullptr;
  if (!events_.empty()) {
    ev = events_.back();
    events_.pop_back();
  } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    ev = nullptr;
  }
  if (ev && hipEventRecord(ev, st) == hipSuccess) {
    pending_.push_back(Pending{off, size, ev});
    return;
  }
  // no event: wait for the stream, then the block is free
  (void)hipGetLastError();
  (void)hipStreamSynchronize(st);
  if (ev) events_.push_back(ev);
  insert_free(off, size);
}

// ---- a server worker's count context

}  // namespace kc

struct kc::WorkerArena {
  Ctx ctx;
};

namespace kc {

WorkerArena* worker_arena_create(int device) {
  try {
    WorkerArena* wa = new WorkerArena();
    wa->ctx.device = device;
    return wa;
  } catch (...) {
    return nullptr;
  }
}

void worker_arena_destroy(WorkerArena* wa) {
  try {
    delete wa;
  } catch (...) {
  }
}

int count_in_block(WorkerArena* wa, void* block, uint64_t block_bytes, Slab* spill,
                   const uint8_t* reads, const uint64_t* offsets, uint64_t n_reads, int k, int P,
                   const kc_options* opt, hipStream_t st, const OutAlloc& oa, uint64_t* n_out,
                   kc_stats* stats, std::string* err) {
  std::vector<void*> spilled;
  Carve cv{(char*)block, (size_t)block_bytes, 0, false, spill, &spilled};
  Ctx& c = wa->ctx;
  // every buffer is carved afresh from the block for this job
  DevBuf* all[] = {&c.packed,  &c.inv,     &c.endm,   &c.valid,   &c.bufA,   &c.bufB,   &c.tmpcnt,
                   &c.hist,    &c.sbegin,  &c.cursor, &c.cursor2, &c.order,  &c.items,
                   &c.bins,    &c.subhist, &c.leaves, &c.dcnt,    &c.outoff, &c.state,
                   &c.large,   &c.ovfl,    &c.bsum,   &c.itemoff, &c.rlist, &c.rleaves,
                   &c.rcount,  &c.aleaves, &c.adcnt,  &c.alarge,  &c.aovfl, &c.rparts,
                   &c.rcnt,    &c.leaves2, &c.dcnt2,  &c.post};
  for (DevBuf* b : all) *b = DevBuf{};
  c.order_P = c.order_sb = -1;
  g_carve = &cv;
  const int r = guarded([&] {
    return count_impl(reads, offsets, n_reads, k, P, nullptr, nullptr, 0, n_out, opt, st, &oa,
                      &c);
  });
  g_carve = nullptr;
  for (DevBuf* b : all) *b = DevBuf{};
  for (void* p : spilled) spill->free(p, st);
  if (r == KC_OK && stats) *stats = g_stats;
  if (r != KC_OK && err) *err = g_err;
  return r;
}

}  // namespace kc

namespace {

std::mutex g_scratch_m;
std::map<int, void*> g_scratch_ptr;  // per device: the device address of `scratch`

// The device address of this device's copy of `scratch`, looked up once per
// device (with that device current). In host code the array's own name is a
// host-side stand-in, never a device address, so kernels get this pointer.
char* noalloc_scratch(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_m);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return (char*)it->second;
  void* ptr = nullptr;
  hipchk(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
  if (!ptr) fail(KC_E_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
  g_scratch_ptr[dev] = ptr;
  return (char*)ptr;
}

struct CarveScope {
  explicit CarveScope(Carve* c) { g_carve = c; }
  ~CarveScope() { g_carve = nullptr; }
};

}  // namespace

extern "C" {

int kc_batch_plan(const uint64_t* host_set_reads, const uint64_t* host_set_bytes,
                  const int* host_ks, uint32_t n_sets, int P, uint64_t hbm_budget,
                  const kc_options* opt, kc_batch** plan) {
  return guarded([&] {
    return batch_plan_impl(host_set_reads, host_set_bytes, host_ks, n_sets, P, hbm_budget, opt,
                           plan);
  });
}

uint32_t kc_batch_waves(const kc_batch* plan) { return plan ? (uint32_t)plan->waves.size() : 0; }

int kc_batch_wave_info(const kc_batch* plan, uint32_t wave, kc_batch_wave* out) {
  if (!plan || !out || wave >= plan->waves.size()) return KC_E_INVAL;
  const kc_batch::Wave& w = plan->waves[wave];
  out->first_set = w.s0;
  out->n_sets = w.ns;
  out->first_read = w.r0;
  out->n_reads = w.nr;
  out->first_byte = w.b0;
  out->n_bytes = w.nbytes;
  out->device_bytes = w.need;
  out->n_classes = (uint32_t)w.cls.size();
  return KC_OK;
}

int kc_batch_run_wave(kc_batch* plan, uint32_t wave, const uint8_t* reads,
                      const uint64_t* offsets, uint64_t* out_keys, uint32_t* out_counts,
                      uint64_t out_capacity, uint64_t* host_out_set_offsets, uint64_t* n_out,
                      void* stream) {
  return guarded([&] {
    return batch_run_wave_impl(plan, wave, reads, offsets, out_keys, out_counts, out_capacity,
                               host_out_set_offsets, n_out, (hipStream_t)stream);
  });
}

int kc_batch_run(kc_batch* plan, const uint8_t* reads, const uint64_t* offsets,
                 uint64_t* out_keys, uint32_t* out_counts, uint64_t out_capacity,
                 uint64_t* host_out_set_offsets, uint64_t* n_out, void* stream) {
  return guarded([&] {
    return batch_run_impl(plan, reads, offsets, out_keys, out_counts, out_capacity,
                          host_out_set_offsets, n_out, (hipStream_t)stream);
  });
}

int kc_batch_stats(const kc_batch* plan, kc_stats* out) {
  if (!plan || !out) return KC_E_INVAL;
  *out = plan->stats;
  return KC_OK;
}

uint64_t kc_batch_max_outputs(const kc_batch* plan) { return plan ? plan->N : 0; }

void kc_batch_free(kc_batch* plan) {
  try {
    delete plan;
  } catch (...) {
  }
}


int kc_count_ex(const uint8_t* reads, const uint64_t* offsets, uint64_t n_reads, int k, int P,
                uint64_t* out_keys, uint32_t* out_counts, uint64_t out_capacity, uint64_t* n_out,
                const kc_options* opt, void* stream) {
  g_err.clear();
  try {
    return count_impl(reads, offsets, n_reads, k, P, out_keys, out_counts, out_capacity, n_out,
                      opt, (hipStream_t)stream);
  } catch (const Fail& f) {
    return f.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return KC_E_NOMEM;
  } catch (...) {
    g_err = "unexpected C++ exception";
    return KC_E_INTERNAL;
  }
}

int kc_count(const uint8_t* reads, const uint64_t* offsets, uint64_t n_reads, int k, int P,
             uint64_t* out_keys, uint32_t* out_counts, uint64_t* n_out) {
  return kc_count_ex(reads, offsets, n_reads, k, P, out_keys, out_counts, ~0ull, n_out, nullptr,
                     nullptr);
}

int kc_count_noalloc(const uint8_t* reads, const uint64_t* offsets, uint64_t n_reads, int k,
                     int P, uint64_t* out_keys, uint32_t* out_counts, uint64_t out_capacity,
                     uint64_t* n_out, const kc_options* opt, void* stream) {
  return guarded([&] {
    int dev = 0;
    hipchk(hipGetDevice(&dev), "hipGetDevice");
    char* base = noalloc_scratch(dev);
    std::lock_guard<std::mutex> lk(g_noalloc_m);
    Carve cv{base, kNoAllocScratchBytes, 0, true, nullptr, nullptr};
    const CarveScope scope(&cv);
    Ctx c;
    c.device = dev;
    return count_impl(reads, offsets, n_reads, k, P, out_keys, out_counts, out_capacity, n_out,
                      opt, (hipStream_t)stream, nullptr, &c);
  });
}

uint64_t kc_max_outputs(const uint64_t* host_offsets, uint64_t n_reads, int k) {
  if (!host_offsets || k < 1 || k > 128) return 0;
  uint64_t w = 0;
  for (uint64_t i = 0; i < n_reads; ++i) {
    if (host_offsets[i + 1] < host_offsets[i]) return 0;
    const uint64_t len = host_offsets[i + 1] - host_offsets[i];
    if (len >= (uint64_t)k) w += len - k + 1;
  }
  return w;
}

int kc_last_stats(kc_stats* out) {
  if (!out) return KC_E_INVAL;
  *out = g_stats;
  return KC_OK;
}

void kc_release_scratch(void) {
  try {
    g_ctx.m.clear();
    free_orphans();
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) kc::trim_device_pool(dev);
  } catch (...) {
  }
}

const char* kc_strerror(int status) {
  switch (status) {
    case KC_OK: return "ok";
    case KC_E_INVAL: return "invalid argument";
    case KC_E_NOMEM: return "out of memory";
    case KC_E_CAPACITY: return "output capacity too small";
    case KC_E_OVERFLOW: return "count overflow";
    case KC_E_DEVICE: return "HIP runtime error";
    case KC_E_INTERNAL: return "internal self-check failed";
    default: return "unknown status";
  }
}

const char* kc_last_error(void) { return g_err.c_str(); }

const char* kc_version(void) { return "kc 0.1 gfx950"; }

}  // extern "C"
