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
  DevBuf hist, sbegin, cursor, cursor2, order, items, bins, subhist, leaves, dcnt, outoff, state;
  DevBuf large, bsum, itemoff;
  std::vector<int> order_host;
  int order_P = -1, order_sb = -1;
  void* host = nullptr;  // pinned staging for small device<->host copies
  size_t host_cap = 0;
  hipEvent_t ev[16] = {};
  bool ev_ok = false;

  ~Ctx() {
    int prev = -1;
    if (hipGetDevice(&prev) == hipSuccess && device >= 0) (void)hipSetDevice(device);
    DevBuf* all[] = {&packed, &inv, &endm,   &bufA,  &bufB,    &tmpcnt, &hist,   &sbegin, &cursor,
                     &cursor2, &order, &items, &bins, &subhist, &leaves, &dcnt, &outoff, &state,
                     &large,   &bsum,  &itemoff};
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
  int buf, bits;
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
  // derived
  uint64_t N = 0, off0 = 0;
  bool wide = false;
  int keybits = 0, sb = 0, nb = 0, slots_log2 = 0;
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

// Host-driven partitioning with any number of split levels: used when a leaf
// of the device-planned path overflowed its table. Starts from the packed
// input and the shard histogram already on the device.
void general_path(Ctx& c, Call& q, kc_stats& S, Timer& tm) {
  const hipStream_t st = q.st;
  std::vector<uint64_t> hist(q.nb);
  {
    uint64_t* hh = (uint64_t*)host_stage(c, (size_t)q.nb * 8);
    hipchk(hipMemcpyAsync(hh, c.hist.p, (size_t)q.nb * 8, hipMemcpyDeviceToHost, st),
           "hipMemcpyAsync");
    hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
    std::memcpy(hist.data(), hh, (size_t)q.nb * 8);
  }
  const std::vector<int>& order = owner_order(c, q, S, &hist);
  std::vector<uint64_t> sbegin(q.nb);
  uint64_t run = 0;
  for (int i : order) {
    sbegin[i] = run;
    run += hist[i];
  }
  const uint64_t W = run;
  upload_sync(c.cursor.p, sbegin.data(), (size_t)q.nb * 8, st);
  hipchk(kc::launch_window_scatter(q.wide, (uint64_t*)c.packed.p, (uint64_t*)c.inv.p,
                                   (uint64_t*)c.endm.p, q.N, q.k, q.sb,
                                   (unsigned long long*)c.cursor.p, c.bufA.p, st),
         "owner scatter launch");
  tm.mark(ST_SCATTER);

  std::vector<Bin> cur;
  for (int i = 0; i < q.nb; ++i)
    if (hist[i]) cur.push_back(Bin{sbegin[i], sbegin[i] + hist[i], (u128)i, q.sb, 0});
  std::vector<LeafDone> done;
  void* bufs[2] = {c.bufA.p, c.bufB.p};
  kc::DevState* dst_state = (kc::DevState*)c.state.p;
  const uint64_t T = std::min<uint64_t>(q.T, q.C / 4);  // finer leaves than the fast path
  const uint64_t H = q.C / 2;
  int level = 0;
  while (!cur.empty()) {
    std::vector<Bin> attempt, split;
    std::vector<bool> was_ovf;
    for (const Bin& b : cur) {
      const uint64_t n = b.end - b.begin;
      if (b.bits >= q.keybits || n <= H) {
        if (b.bits >= q.keybits && n > 0xFFFFFFFFull)
          fail(KC_E_OVERFLOW, "a k-mer occurs more than 2^32-1 times");
        attempt.push_back(b);
      } else {
        split.push_back(b);
        was_ovf.push_back(false);
      }
    }
    if (!attempt.empty()) {
      const size_t na = attempt.size();
      std::vector<kc::Leaf> lv(na);
      for (size_t i = 0; i < na; ++i)
        lv[i] = kc::Leaf{attempt[i].begin, attempt[i].end, (uint32_t)attempt[i].buf,
                         (uint32_t)attempt[i].bits};
      ensure(c.leaves, na * sizeof(kc::Leaf), "leaf table");
      ensure(c.dcnt, na * 4, "leaf counts");
      ensure(c.large, na * 4, "large-leaf list");
      upload_sync(c.leaves.p, lv.data(), na * sizeof(kc::Leaf), st);
      unsigned long long nl = na;
      upload_sync(&dst_state->n_leaves, &nl, 8, st);
      hipchk(kc::launch_leaf_count(q.wide, q.k, c.bufA.p, c.bufB.p, (uint32_t*)c.tmpcnt.p,
                                   (kc::Leaf*)c.leaves.p, dst_state, na, (uint32_t*)c.dcnt.p,
                                   q.slots_log2, (uint32_t*)c.large.p, st),
             "leaf count launch");
      tm.mark(ST_LEAF);
      uint32_t* hd = (uint32_t*)host_stage(c, na * 4);
      hipchk(hipMemcpyAsync(hd, c.dcnt.p, na * 4, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
      hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
      for (size_t i = 0; i < na; ++i) {
        const Bin& b = attempt[i];
        if (hd[i] == kc::kLeafOverflow) {
          if (b.bits >= q.keybits) fail(KC_E_INTERNAL, "single-key partition overflowed its table");
          ++S.n_overflow;
          split.push_back(b);
          was_ovf.push_back(true);
        } else {
          done.push_back(LeafDone{b.prefix << (q.keybits - b.bits), b.begin, b.end, hd[i], b.buf,
                                  b.bits});
          S.max_leaf_windows = std::max(S.max_leaf_windows, b.end - b.begin);
        }
      }
    }
    if (split.empty()) break;
    ++level;
    const size_t ns = split.size();
    std::vector<kc::SplitBin> sbins(ns);
    std::vector<kc::SplitItem> items;
    uint64_t hoff = 0;
    const uint64_t tile = (uint64_t)kc::split_tile(q.wide);
    for (size_t i = 0; i < ns; ++i) {
      const Bin& b = split[i];
      const uint64_t n = b.end - b.begin;
      const int remaining = q.keybits - b.bits;
      int nbits = ceil_log2((n + T - 1) / T);
      if (was_ovf[i]) nbits = std::max(nbits, 2);
      nbits = std::max(1, std::min(nbits, std::min(kc::kSplitMaxBits, remaining)));
      sbins[i] = kc::SplitBin{hoff, (uint32_t)(q.keybits - b.bits - nbits), (uint32_t)nbits};
      hoff += 1ull << nbits;
      for (uint64_t a = b.begin; a < b.end; a += tile)
        items.push_back(kc::SplitItem{a, std::min(b.end, a + tile), (uint32_t)i, 0});
    }
    ensure(c.bins, ns * sizeof(kc::SplitBin), "split bins");
    ensure(c.items, items.size() * sizeof(kc::SplitItem), "split items");
    ensure(c.subhist, hoff * 8, "sub-bin histogram");
    ensure(c.cursor2, hoff * 8, "sub-bin cursors");
    upload_sync(c.items.p, items.data(), items.size() * sizeof(kc::SplitItem), st);
    upload_sync(c.bins.p, sbins.data(), ns * sizeof(kc::SplitBin), st);
    unsigned long long ni = items.size();
    upload_sync(&dst_state->n_items, &ni, 8, st);
    hipchk(kc::launch_fill_u64((unsigned long long*)c.subhist.p, hoff, 0, st), "fill launch");
    const int src = split[0].buf;
    hipchk(kc::launch_split_hist(q.wide, bufs[src], (kc::SplitItem*)c.items.p, dst_state,
                                 items.size(), (kc::SplitBin*)c.bins.p,
                                 (unsigned long long*)c.subhist.p, st),
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
      uint64_t r = b.begin;
      for (uint64_t j = 0; j < (1ull << sbn.nbits); ++j) {
        const uint64_t cnt = hsub[sbn.hist_off + j];
        hcur[sbn.hist_off + j] = r;
        if (cnt)
          next.push_back(Bin{r, r + cnt, (b.prefix << sbn.nbits) | (u128)j,
                             b.bits + (int)sbn.nbits, 1 - b.buf});
        r += cnt;
      }
      if (r != b.end) fail(KC_E_INTERNAL, "split histogram does not match partition size");
    }
    upload_sync(c.cursor2.p, hcur.data(), hoff * 8, st);
    hipchk(kc::launch_split_scatter(q.wide, bufs[src], bufs[1 - src], (kc::SplitItem*)c.items.p,
                                    dst_state, items.size(), (kc::SplitBin*)c.bins.p,
                                    (unsigned long long*)c.cursor2.p, st),
           "split scatter launch");
    tm.mark(ST_SPLIT);
    hipchk(hipStreamSynchronize(st), "hipStreamSynchronize");
    cur.swap(next);
  }
  S.n_levels = level;
  std::sort(done.begin(), done.end(),
            [](const LeafDone& a, const LeafDone& b) { return a.start < b.start; });
  const size_t nl = done.size();
  std::vector<kc::Leaf> lv(nl);
  std::vector<uint32_t> dv(nl);
  uint64_t D = 0;
  for (size_t i = 0; i < nl; ++i) {
    lv[i] = kc::Leaf{done[i].begin, done[i].end, (uint32_t)done[i].buf, (uint32_t)done[i].bits};
    dv[i] = done[i].d;
    D += done[i].d;
  }
  (void)W;
  S.n_leaves = nl;
  ensure(c.leaves, nl * sizeof(kc::Leaf), "leaf table");
  ensure(c.dcnt, nl * 4, "leaf counts");
  ensure(c.outoff, nl * 8, "output offsets");
  ensure(c.bsum, kc::scan_blocks(nl) * 8, "scan block sums");
  upload_sync(c.leaves.p, lv.data(), nl * sizeof(kc::Leaf), st);
  upload_sync(c.dcnt.p, dv.data(), nl * 4, st);
  unsigned long long nlu = nl;
  upload_sync(&dst_state->n_leaves, &nlu, 8, st);
  unsigned int zero = 0;
  upload_sync(&dst_state->overflow, &zero, 4, st);
  hipchk(kc::launch_plan_out((uint32_t*)c.dcnt.p, dst_state, (unsigned long long*)c.bsum.p, nl,
                             (unsigned long long*)c.outoff.p, st),
         "plan_out launch");
  hipchk(kc::launch_concat(q.wide, c.bufA.p, c.bufB.p, (uint32_t*)c.tmpcnt.p,
                           (kc::Leaf*)c.leaves.p, (uint32_t*)c.dcnt.p,
                           (unsigned long long*)c.outoff.p, dst_state, nl, q.cap, q.out_keys,
                           q.out_counts, st),
         "concat launch");
  tm.mark(ST_CONCAT);
  (void)D;
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
  Call q{reads, offsets, n_reads, k, P, out_keys, out_counts, cap, {}, st};
  std::memset(&q.o, 0, sizeof(q.o));
  if (opt) q.o = *opt;
  if (q.o.mode != 0) fail(KC_E_INVAL, "mode must be 0");

  Ctx& c = context();
  std::memset(&g_stats, 0, sizeof(g_stats));
  kc_stats S;
  std::memset(&S, 0, sizeof(S));
  Timer tm(c, st, q.o.timing != 0);

  // ---- offsets: first/last, monotonicity (host sync 1 of 2)
  ensure(c.state, sizeof(kc::DevState), "device state");
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
  q.wide = k > 32;
  q.keybits = 2 * k;
  q.ksz = q.wide ? 16 : 8;
  const int max_slots = kc::max_leaf_slots_log2(q.wide);
  q.slots_log2 = q.o.table_slots_log2 > 0
                     ? std::min(std::max(q.o.table_slots_log2, 10), max_slots)
                     : max_slots;
  q.C = 1ull << q.slots_log2;
  // default leaf size: about half of what the one-wave leaf kernel takes, so
  // that nearly all leaves (after the split's size spread) stay in that kernel
  // default leaf size: half of the largest table, so that the size spread of
  // the split leaves nearly every leaf within one table
  q.T = q.o.leaf_target > 0 ? (uint64_t)q.o.leaf_target : (q.C * 3) / 4;
  q.H = q.o.leaf_attempt > 0 ? (uint64_t)q.o.leaf_attempt : (q.C * 7) / 8;
  int sb = q.o.shard_bits;
  if (sb <= 0) {
    sb = std::max(8, ceil_log2((uint64_t)P));
    sb = std::max(sb, ceil_log2(q.N / (q.T << kc::kSplitMaxBits) + 1));
  }
  sb = std::min(sb, kc::max_shard_bits());
  sb = std::min(sb, q.keybits);
  q.sb = sb;
  q.nb = 1 << sb;

  const uint64_t nchunks = (q.N + 63) / 64 + 2;
  ensure(c.packed, nchunks * 16, "packed bases");
  ensure(c.inv, nchunks * 8, "invalid mask");
  ensure(c.endm, nchunks * 8, "end mask");
  // record buffers sized by the byte count, an upper bound of the window count
  ensure(c.bufA, q.N * q.ksz, "record buffer A");
  ensure(c.bufB, q.N * q.ksz, "record buffer B");
  ensure(c.tmpcnt, q.N * 4, "pair counts");
  const uint64_t tile = (uint64_t)kc::split_tile(q.wide);
  const uint64_t max_items = q.N / tile + (uint64_t)q.nb + 1;
  const uint64_t max_leaves =
      std::min<uint64_t>((uint64_t)q.nb << kc::kSplitMaxBits, 2 * q.N / q.T + 2 * (uint64_t)q.nb) +
      1;
  ensure(c.hist, (size_t)q.nb * 8, "shard histogram");
  ensure(c.sbegin, (size_t)q.nb * 8, "shard begins");
  ensure(c.cursor, (size_t)q.nb * 8, "shard cursors");
  ensure(c.order, (size_t)q.nb * 4, "owner order");
  ensure(c.bins, (size_t)q.nb * sizeof(kc::SplitBin), "split bins");
  ensure(c.items, max_items * sizeof(kc::SplitItem), "split items");
  ensure(c.itemoff, ((size_t)q.nb + 1) * 8, "split item offsets");
  ensure(c.subhist, max_leaves * 8, "sub-bin histogram");
  ensure(c.cursor2, max_leaves * 8, "sub-bin cursors");
  ensure(c.leaves, max_leaves * sizeof(kc::Leaf), "leaf table");
  ensure(c.dcnt, max_leaves * 4, "leaf counts");
  ensure(c.outoff, max_leaves * 8, "output offsets");
  ensure(c.large, max_leaves * 4, "large-leaf list");
  ensure(c.bsum, kc::scan_blocks(max_leaves) * 8, "scan block sums");
  if (c.order_P != P || c.order_sb != sb) {
    const std::vector<int>& order = owner_order(c, q, S, nullptr);
    c.order_host.assign(order.begin(), order.end());
    upload_sync(c.order.p, c.order_host.data(), (size_t)q.nb * 4, st);
    c.order_P = P;
    c.order_sb = sb;
  }
  kc::DevState* dstate = (kc::DevState*)c.state.p;

  tm.mark(ST_NONE);
  hipchk(kc::launch_pack(reads + off0, q.N, offsets, n_reads, off0, (uint64_t*)c.packed.p,
                         (uint64_t*)c.inv.p, (uint64_t*)c.endm.p, nchunks, st),
         "pack launch");
  tm.mark(ST_PACK);
  hipchk(kc::launch_fill_u64((unsigned long long*)c.hist.p, q.nb, 0, st), "fill launch");
  hipchk(kc::launch_window_hist(q.wide, (uint64_t*)c.packed.p, (uint64_t*)c.inv.p,
                                (uint64_t*)c.endm.p, q.N, k, sb, (unsigned long long*)c.hist.p,
                                &dstate->W, st),
         "window histogram launch");
  tm.mark(ST_HIST);
  // ---- device-planned partitioning: shard plan, scatter, one split level, leaves
  hipchk(kc::launch_plan_shards((unsigned long long*)c.hist.p, (const int*)c.order.p, sb,
                                q.keybits, q.T, q.H, (int)tile, (unsigned long long*)c.sbegin.p,
                                (unsigned long long*)c.cursor.p, (kc::SplitBin*)c.bins.p,
                                (kc::SplitItem*)c.items.p, (unsigned long long*)c.itemoff.p,
                                (unsigned long long*)c.subhist.p, max_leaves, max_items, dstate,
                                st),
         "plan_shards launch");
  hipchk(kc::launch_window_scatter(q.wide, (uint64_t*)c.packed.p, (uint64_t*)c.inv.p,
                                   (uint64_t*)c.endm.p, q.N, k, sb,
                                   (unsigned long long*)c.cursor.p, c.bufA.p, st),
         "owner scatter launch");
  tm.mark(ST_SCATTER);
  hipchk(kc::launch_split_hist(q.wide, c.bufA.p, (kc::SplitItem*)c.items.p, dstate, max_items,
                               (kc::SplitBin*)c.bins.p, (unsigned long long*)c.subhist.p, st),
         "split histogram launch");
  hipchk(kc::launch_plan_leaves((unsigned long long*)c.hist.p, (unsigned long long*)c.sbegin.p,
                                (kc::SplitBin*)c.bins.p, sb, (unsigned long long*)c.subhist.p,
                                (kc::Leaf*)c.leaves.p, (unsigned long long*)c.cursor2.p, st),
         "plan_leaves launch");
  hipchk(kc::launch_split_scatter(q.wide, c.bufA.p, c.bufB.p, (kc::SplitItem*)c.items.p, dstate,
                                  max_items, (kc::SplitBin*)c.bins.p,
                                  (unsigned long long*)c.cursor2.p, st),
         "split scatter launch");
  tm.mark(ST_SPLIT);
  hipchk(kc::launch_leaf_count(q.wide, k, c.bufA.p, c.bufB.p, (uint32_t*)c.tmpcnt.p,
                               (kc::Leaf*)c.leaves.p, dstate, max_leaves, (uint32_t*)c.dcnt.p,
                               q.slots_log2, (uint32_t*)c.large.p, st),
         "leaf count launch");
  tm.mark(ST_LEAF);
  hipchk(kc::launch_plan_out((uint32_t*)c.dcnt.p, dstate, (unsigned long long*)c.bsum.p, max_leaves,
                             (unsigned long long*)c.outoff.p, st),
         "plan_out launch");
  hipchk(kc::launch_concat(q.wide, c.bufA.p, c.bufB.p, (uint32_t*)c.tmpcnt.p,
                           (kc::Leaf*)c.leaves.p, (uint32_t*)c.dcnt.p,
                           (unsigned long long*)c.outoff.p, dstate, max_leaves, cap, out_keys,
                           out_counts, st),
         "concat launch");
  tm.mark(ST_CONCAT);
  kc::DevState ds = read_state(c, st);  // host sync 2 of 2
  S.n_levels = 1;
  S.n_leaves = ds.n_leaves;
  if (ds.overflow) {
    // some leaf had more distinct keys than its table holds: redo the
    // partitioning with host-planned recursive splits
    ++S.n_overflow;
    general_path(c, q, S, tm);
    ds = read_state(c, st);
    if (ds.overflow) fail(KC_E_INTERNAL, "leaf overflow in the recursive path");
  }
  S.valid_windows = ds.W;
  S.distinct = ds.D;
  if (ds.count_overflow) fail(KC_E_OVERFLOW, "a k-mer occurs more than 2^32-1 times");
  if (ds.D > cap) {
    *n_out = ds.D;
    fail(KC_E_CAPACITY, "output capacity " + std::to_string(cap) + " < " + std::to_string(ds.D) +
                            " distinct k-mers");
  }
  if (q.o.check) {
    hipchk(kc::launch_fill_u64((unsigned long long*)&dstate->check, sizeof(kc::CheckResult) / 8,
                               0, st),
           "fill launch");
    hipchk(kc::launch_check(q.wide, out_keys, out_counts, ds.D, k, &dstate->check, st),
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
  tm.collect(S);
  *n_out = ds.D;
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
