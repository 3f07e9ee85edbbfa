// Host runtime behind the C ABI of include/kc.h: argument checks, a
// per-thread device arena, the partition planner (owner layout, MSD splits,
// leaf list, output offsets) and the launch sequence of the kernels in
// kc_kernels.hip. No exception leaves this file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/kc.h"
#include "kc_internal.h"

namespace {

typedef unsigned __int128 u128;

thread_local std::string g_err;
thread_local kc_stats g_stats;

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

struct Ctx {
  int device = -1;
  DevBuf packed, inv, endm, bufA, bufB, tmpcnt;
  DevBuf hist, wcount, cursor, items, bins, subhist, leaves, dcnt, flags, check;
  void* host = nullptr;  // pinned staging for small device<->host copies
  size_t host_cap = 0;
  hipEvent_t ev[16] = {};
  bool ev_ok = false;

  ~Ctx() {
    int prev = -1;
    if (hipGetDevice(&prev) == hipSuccess && device >= 0) (void)hipSetDevice(device);
    DevBuf* all[] = {&packed, &inv, &endm, &bufA, &bufB, &tmpcnt, &hist, &wcount,
                     &cursor, &items, &bins, &subhist, &leaves, &dcnt, &flags, &check};
    for (DevBuf* b : all)
      if (b->p) (void)hipFree(b->p);
    if (host) (void)hipHostFree(host);
    if (ev_ok)
      for (hipEvent_t& e : ev) (void)hipEventDestroy(e);
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

thread_local std::map<int, std::unique_ptr<Ctx>> g_ctx;

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

void ensure(DevBuf& b, size_t bytes, const char* name) {
  if (bytes == 0) bytes = 256;
  if (b.cap >= bytes) return;
  if (b.p) {
    hipchk(hipFree(b.p), "hipFree");
    b.p = nullptr;
    b.cap = 0;
  }
  size_t want = bytes + bytes / 8;
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

void* host_stage(Ctx& c, size_t bytes) {
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
  auto& slot = g_ctx[dev];
  if (!slot) {
    slot.reset(new Ctx());
    slot->device = dev;
  }
  return *slot;
}

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

struct Bin {
  uint64_t begin, end;
  u128 prefix;  // value of the key bits consumed so far
  int bits;     // number of key bits consumed (from the most significant end)
  int buf;      // buffer holding its records
};

struct LeafDone {
  u128 start;  // first key of its range
  uint64_t begin, end;
  uint32_t d;
  int buf;
};

struct Timer {
  Ctx& c;
  hipStream_t s;
  bool on;
  int n = 0;
  int stage[16];
  Timer(Ctx& c_, hipStream_t s_, bool on_) : c(c_), s(s_), on(on_) {
    if (on && !c.ev_ok) {
      for (hipEvent_t& e : c.ev) hipchk(hipEventCreate(&e), "hipEventCreate");
      c.ev_ok = true;
    }
  }
  void mark(int st) {  // the interval from the previous mark to this one is charged to `st`
    if (!on || n >= 16) return;
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
      if (stage[i] >= 0 && stage[i] < 8) out.ms_stage[stage[i]] += ms;
    }
  }
};

enum { ST_PACK = 0, ST_HIST = 1, ST_SCATTER = 2, ST_SPLIT = 3, ST_LEAF = 4, ST_CONCAT = 5,
       ST_CHECK = 6, ST_NONE = -1 };

__global__ void k_offsets_ok(const uint64_t* off, uint64_t n, unsigned int* bad) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && off[i + 1] < off[i]) atomicOr(bad, 1u);
}

int count_impl(const uint8_t* reads, const uint64_t* offsets, uint64_t n_reads, int k, int P,
               uint64_t* out_keys, uint32_t* out_counts, uint64_t cap, uint64_t* n_out,
               const kc_options* opt, hipStream_t st) {
  auto t_host0 = std::chrono::steady_clock::now();
  if (!n_out) fail(KC_E_INVAL, "n_out is NULL");
  *n_out = 0;
  if (k < 1 || k > 64) fail(KC_E_INVAL, "k must be in [1, 64]");
  if (P < 1) fail(KC_E_INVAL, "P must be >= 1");
  if (!offsets) fail(KC_E_INVAL, "offsets is NULL");
  if (n_reads && !reads) fail(KC_E_INVAL, "reads is NULL");
  if (cap && (!out_keys || !out_counts)) fail(KC_E_INVAL, "output pointer is NULL");
  kc_options o;
  std::memset(&o, 0, sizeof(o));
  if (opt) o = *opt;
  if (o.mode != 0) fail(KC_E_INVAL, "mode must be 0");

  Ctx& c = context();
  std::memset(&g_stats, 0, sizeof(g_stats));
  kc_stats S;
  std::memset(&S, 0, sizeof(S));
  Timer tm(c, st, o.timing != 0);

  // ---- offsets: first/last, monotonicity
  ensure(c.flags, 64, "flags");
  uint64_t* h = (uint64_t*)host_stage(c, 64);
  hipchk(hipMemsetAsync(c.flags.p, 0, 16, st), "hipMemsetAsync");
  if (n_reads) {
    const unsigned g = (unsigned)((n_reads + 255) / 256);
    hipLaunchKernelGGL(k_offsets_ok, dim3(g), dim3(256), 0, st, offsets, n_reads,
                       (unsigned int*)c.flags.p);
    hipchk(hipGetLastError(), "offsets check launch");
  }
  hipchk(hipMemcpyAsync(h, offsets, 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
  hipchk(hipMemcpyAsync(h + 1, offsets + n_reads, 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
  hipchk(hipMemcpyAsync(h + 2, c.flags.p, 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
  hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
  const uint64_t off0 = h[0], offn = h[1];
  if ((uint32_t)h[2] != 0 || offn < off0) fail(KC_E_INVAL, "offsets must be non-decreasing");
  const uint64_t N = offn - off0;
  S.n_bases = N;
  if (N == 0) {
    g_stats = S;
    return KC_OK;
  }

  const bool wide = k > 32;
  const int keybits = 2 * k;
  const size_t ksz = wide ? 16 : 8;
  const uint64_t nchunks = (N + 63) / 64 + 2;
  ensure(c.packed, nchunks * 16, "packed bases");
  ensure(c.inv, nchunks * 8, "invalid mask");
  ensure(c.endm, nchunks * 8, "end mask");
  tm.mark(ST_NONE);
  hipchk(kc::launch_pack(reads + off0, N, offsets, n_reads, off0, (uint64_t*)c.packed.p,
                         (uint64_t*)c.inv.p, (uint64_t*)c.endm.p, nchunks, st),
         "pack launch");
  tm.mark(ST_PACK);

  // ---- first level: shard histogram
  int sb = o.shard_bits;
  if (sb <= 0) sb = std::max(8, ceil_log2((uint64_t)P));
  sb = std::min(sb, kc::max_shard_bits());
  sb = std::min(sb, keybits);
  const int nb = 1 << sb;
  ensure(c.hist, (size_t)nb * 8, "shard histogram");
  ensure(c.wcount, 64, "window count");
  hipchk(hipMemsetAsync(c.hist.p, 0, (size_t)nb * 8, st), "hipMemsetAsync");
  hipchk(hipMemsetAsync(c.wcount.p, 0, 8, st), "hipMemsetAsync");
  hipchk(kc::launch_window_hist(wide, (uint64_t*)c.packed.p, (uint64_t*)c.inv.p,
                                (uint64_t*)c.endm.p, N, k, sb, (unsigned long long*)c.hist.p,
                                (unsigned long long*)c.wcount.p, st),
         "window histogram launch");
  tm.mark(ST_HIST);
  uint64_t* hh = (uint64_t*)host_stage(c, (size_t)(nb + 1) * 8);
  hipchk(hipMemcpyAsync(hh, c.hist.p, (size_t)nb * 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
  hipchk(hipMemcpyAsync(hh + nb, c.wcount.p, 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
  hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
  std::vector<uint64_t> hist(hh, hh + nb);
  const uint64_t W = hh[nb];
  S.valid_windows = W;
  uint64_t hsum = 0;
  for (uint64_t x : hist) hsum += x;
  if (hsum != W) fail(KC_E_INTERNAL, "shard histogram does not sum to the valid window count");
  if (W == 0) {
    tm.collect(S);
    g_stats = S;
    return KC_OK;
  }

  // ---- owner-major layout of shards: each owner's shards form one contiguous range
  std::vector<int> order(nb);
  std::vector<uint64_t> owner(nb);
  for (int i = 0; i < nb; ++i) {
    order[i] = i;
    owner[i] = (uint64_t)(((u128)host_mix((uint64_t)i * 0x9E3779B97F4A7C15ull + 0x51ED27ull) *
                           (u128)(uint64_t)P) >> 64);
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return owner[a] < owner[b]; });
  std::vector<uint64_t> sbegin(nb);
  {
    uint64_t run = 0, cur_owner = ~0ull, owner_w = 0;
    for (int i : order) {
      if (owner[i] != cur_owner) {
        S.max_owner_windows = std::max(S.max_owner_windows, owner_w);
        owner_w = 0;
        cur_owner = owner[i];
      }
      sbegin[i] = run;
      run += hist[i];
      owner_w += hist[i];
    }
    S.max_owner_windows = std::max(S.max_owner_windows, owner_w);
  }
  ensure(c.bufA, W * ksz, "record buffer A");
  ensure(c.bufB, W * ksz, "record buffer B");
  ensure(c.tmpcnt, W * 4, "pair counts");
  ensure(c.cursor, (size_t)nb * 8, "cursors");
  // host-to-device copies read pageable vectors that outlive the copy; the
  // pinned staging buffer is used only for device-to-host copies followed by a
  // synchronize, so it is never overwritten while a copy is pending
  hipchk(hipMemcpyAsync(c.cursor.p, sbegin.data(), (size_t)nb * 8, hipMemcpyHostToDevice, st),
         "hipMemcpyAsync");
  hipchk(kc::launch_window_scatter(wide, (uint64_t*)c.packed.p, (uint64_t*)c.inv.p,
                                   (uint64_t*)c.endm.p, N, k, sb, (unsigned long long*)c.cursor.p,
                                   c.bufA.p, st),
         "owner scatter launch");
  tm.mark(ST_SCATTER);

  std::vector<Bin> cur;
  for (int i = 0; i < nb; ++i)
    if (hist[i]) cur.push_back(Bin{sbegin[i], sbegin[i] + hist[i], (u128)i, sb, 0});

  const int max_slots = kc::max_leaf_slots_log2(wide);
  int slots_log2 = o.table_slots_log2 > 0 ? std::min(std::max(o.table_slots_log2, 10), max_slots)
                                          : max_slots;
  const uint64_t C = 1ull << slots_log2;
  const uint64_t T = o.leaf_target > 0 ? (uint64_t)o.leaf_target : C / 2;
  const uint64_t H = o.leaf_attempt > 0 ? (uint64_t)o.leaf_attempt : 2 * C;

  std::vector<LeafDone> done;
  void* bufs[2] = {c.bufA.p, c.bufB.p};
  ensure(c.check, 64, "overflow flag");
  hipchk(hipMemsetAsync(c.check.p, 0, 64, st), "hipMemsetAsync");
  unsigned int* count_ovf = (unsigned int*)c.check.p;

  int level = 0;
  while (!cur.empty()) {
    std::vector<Bin> attempt, split;
    std::vector<bool> ovf_flag;
    for (const Bin& b : cur) {
      const uint64_t n = b.end - b.begin;
      if (b.bits >= keybits || n <= H) {
        if (b.bits >= keybits && n > 0xFFFFFFFFull)
          fail(KC_E_OVERFLOW, "a k-mer occurs more than 2^32-1 times");
        attempt.push_back(b);
      } else {
        split.push_back(b);
      }
    }
    std::vector<bool> was_ovf(split.size(), false);
    if (!attempt.empty()) {
      const size_t na = attempt.size();
      std::vector<kc::Leaf> lv(na);
      for (size_t i = 0; i < na; ++i) lv[i] = kc::Leaf{attempt[i].begin, attempt[i].end, 0,
                                                       (uint32_t)attempt[i].buf, 0};
      ensure(c.leaves, na * sizeof(kc::Leaf), "leaf table");
      ensure(c.dcnt, na * 4, "leaf counts");
      hipchk(hipMemcpyAsync(c.leaves.p, lv.data(), na * sizeof(kc::Leaf), hipMemcpyHostToDevice,
                            st),
             "hipMemcpyAsync");
      hipchk(kc::launch_leaf_count(wide, c.bufA.p, c.bufB.p, (uint32_t*)c.tmpcnt.p,
                                   (kc::Leaf*)c.leaves.p, na, (uint32_t*)c.dcnt.p, slots_log2,
                                   count_ovf, st),
             "leaf count launch");
      tm.mark(ST_LEAF);
      uint32_t* hd = (uint32_t*)host_stage(c, na * 4);
      hipchk(hipMemcpyAsync(hd, c.dcnt.p, na * 4, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
      hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
      for (size_t i = 0; i < na; ++i) {
        const Bin& b = attempt[i];
        if (hd[i] == 0xFFFFFFFFu) {
          if (b.bits >= keybits) fail(KC_E_INTERNAL, "single-key partition overflowed its table");
          ++S.n_overflow;
          split.push_back(b);
          was_ovf.push_back(true);
        } else {
          const u128 start = b.prefix << (keybits - b.bits);
          done.push_back(LeafDone{start, b.begin, b.end, hd[i], b.buf});
          S.max_leaf_windows = std::max(S.max_leaf_windows, b.end - b.begin);
        }
      }
    }
    if (split.empty()) break;
    ++level;
    // ---- split step: histogram of the next key bits, then scatter into sub-bins
    const size_t ns = split.size();
    std::vector<kc::SplitBin> sbins(ns);
    std::vector<kc::SplitItem> items;
    uint64_t hoff = 0;
    const uint64_t tile = (uint64_t)kc::split_tile(wide);
    for (size_t i = 0; i < ns; ++i) {
      const Bin& b = split[i];
      const uint64_t n = b.end - b.begin;
      const int remaining = keybits - b.bits;
      int nbits = ceil_log2((n + T - 1) / T);
      if (was_ovf[i]) nbits = std::max(nbits, 2);
      nbits = std::max(1, std::min(nbits, std::min(kc::kSplitMaxBits, remaining)));
      sbins[i] = kc::SplitBin{hoff, (uint32_t)(keybits - b.bits - nbits), (uint32_t)nbits};
      hoff += 1ull << nbits;
      for (uint64_t a = b.begin; a < b.end; a += tile)
        items.push_back(kc::SplitItem{a, std::min(b.end, a + tile), (uint32_t)i, 0});
    }
    ensure(c.bins, ns * sizeof(kc::SplitBin), "split bins");
    ensure(c.items, items.size() * sizeof(kc::SplitItem), "split items");
    ensure(c.subhist, hoff * 8, "sub-bin histogram");
    hipchk(hipMemcpyAsync(c.items.p, items.data(), items.size() * sizeof(kc::SplitItem),
                          hipMemcpyHostToDevice, st),
           "hipMemcpyAsync");
    hipchk(hipMemcpyAsync(c.bins.p, sbins.data(), ns * sizeof(kc::SplitBin),
                          hipMemcpyHostToDevice, st),
           "hipMemcpyAsync");
    hipchk(hipMemsetAsync(c.subhist.p, 0, hoff * 8, st), "hipMemsetAsync");
    const int src = split[0].buf;
    hipchk(kc::launch_split_hist(wide, bufs[src], (kc::SplitItem*)c.items.p, items.size(),
                                 (kc::SplitBin*)c.bins.p, (unsigned long long*)c.subhist.p, st),
           "split histogram launch");
    uint64_t* hsub = (uint64_t*)host_stage(c, hoff * 8 + 64);
    hipchk(hipMemcpyAsync(hsub, c.subhist.p, hoff * 8, hipMemcpyDeviceToHost, st),
           "hipMemcpyAsync");
    hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
    std::vector<Bin> next;
    std::vector<uint64_t> hcur(hoff);
    for (size_t i = 0; i < ns; ++i) {
      const Bin& b = split[i];
      const kc::SplitBin& sbn = sbins[i];
      uint64_t run = b.begin;
      for (uint64_t j = 0; j < (1ull << sbn.nbits); ++j) {
        const uint64_t cnt = hsub[sbn.hist_off + j];
        hcur[sbn.hist_off + j] = run;
        if (cnt)
          next.push_back(Bin{run, run + cnt, (b.prefix << sbn.nbits) | (u128)j,
                             b.bits + (int)sbn.nbits, 1 - b.buf});
        run += cnt;
      }
      if (run != b.end) fail(KC_E_INTERNAL, "split histogram does not match partition size");
    }
    ensure(c.cursor, hoff * 8, "cursors");
    hipchk(hipMemcpyAsync(c.cursor.p, hcur.data(), hoff * 8, hipMemcpyHostToDevice, st),
           "hipMemcpyAsync");
    hipchk(kc::launch_split_scatter(wide, bufs[src], bufs[1 - src], (kc::SplitItem*)c.items.p,
                                    items.size(), (kc::SplitBin*)c.bins.p,
                                    (unsigned long long*)c.cursor.p, st),
           "split scatter launch");
    tm.mark(ST_SPLIT);
    // the vectors read by the copies above go out of scope at the end of this pass
    hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
    cur.swap(next);
  }
  S.n_levels = level;

  // ---- order leaves by key range, output offsets, concat
  std::sort(done.begin(), done.end(),
            [](const LeafDone& a, const LeafDone& b) { return a.start < b.start; });
  uint64_t D = 0;
  const size_t nl = done.size();
  std::vector<kc::Leaf> lv(nl);
  std::vector<uint32_t> dv(nl);
  for (size_t i = 0; i < nl; ++i) {
    lv[i] = kc::Leaf{done[i].begin, done[i].end, D, (uint32_t)done[i].buf, 0};
    dv[i] = done[i].d;
    D += done[i].d;
  }
  S.distinct = D;
  S.n_leaves = nl;
  if (D > cap) {
    *n_out = D;
    fail(KC_E_CAPACITY, "output capacity " + std::to_string(cap) + " < " + std::to_string(D) +
                            " distinct k-mers");
  }
  ensure(c.leaves, nl * sizeof(kc::Leaf), "leaf table");
  ensure(c.dcnt, nl * 4, "leaf counts");
  hipchk(hipMemcpyAsync(c.leaves.p, lv.data(), nl * sizeof(kc::Leaf), hipMemcpyHostToDevice, st),
         "hipMemcpyAsync");
  hipchk(hipMemcpyAsync(c.dcnt.p, dv.data(), nl * 4, hipMemcpyHostToDevice, st),
         "hipMemcpyAsync");
  hipchk(kc::launch_concat(wide, c.bufA.p, c.bufB.p, (uint32_t*)c.tmpcnt.p,
                           (kc::Leaf*)c.leaves.p, (uint32_t*)c.dcnt.p, nl, out_keys, out_counts,
                           st),
         "concat launch");
  tm.mark(ST_CONCAT);
  if (o.check) {
    hipchk(hipMemsetAsync((char*)c.check.p + 16, 0, sizeof(kc::CheckResult), st),
           "hipMemsetAsync");
    hipchk(kc::launch_check(wide, out_keys, out_counts, D, k,
                            (kc::CheckResult*)((char*)c.check.p + 16), st),
           "check launch");
    tm.mark(ST_CHECK);
  }
  uint32_t* hf = (uint32_t*)host_stage(c, 64);
  hipchk(hipMemcpyAsync(hf, c.check.p, 16 + sizeof(kc::CheckResult), hipMemcpyDeviceToHost, st),
         "hipMemcpyAsync");
  hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
  if (hf[0]) fail(KC_E_OVERFLOW, "a k-mer occurs more than 2^32-1 times");
  if (o.check) {
    kc::CheckResult r;
    std::memcpy(&r, (char*)hf + 16, sizeof(r));
    if (r.sum_counts != W || r.not_sorted || r.not_canonical || r.out_of_range || r.zero_count) {
      char msg[256];
      std::snprintf(msg, sizeof msg,
                    "device self-check failed: sum %llu (want %llu), unsorted %u, "
                    "non-canonical %u, out of range %u, zero counts %u",
                    r.sum_counts, (unsigned long long)W, r.not_sorted, r.not_canonical,
                    r.out_of_range, r.zero_count);
      fail(KC_E_INTERNAL, msg);
    }
  }
  tm.collect(S);
  *n_out = D;
  S.ms_total =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_host0).count();
  g_stats = S;
  return KC_OK;
}

}  // namespace

extern "C" {

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

uint64_t kc_max_outputs(const uint64_t* host_offsets, uint64_t n_reads, int k) {
  if (!host_offsets || k < 1 || k > 64) return 0;
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
    g_ctx.clear();
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
