// Uses of a count result (entry points kc_spectrum and kc_filter_min_count of
// include/kc.h): the k-mer spectrum (how many distinct keys have each count)
// and the removal of keys below a minimum count, the two most common things
// done with a k-mer histogram (the paper's Section II surveys counters that
// avoid counting singletons for the same reason).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/kc.h"
#include "kc_host.h"

namespace {

constexpr int kTB = 256;
constexpr int kPer = 16;  // items per thread in the compaction
constexpr int kTile = kTB * kPer;
constexpr uint32_t kLdsBins = 4096;

// Spectrum: bins 1..max_count-1 hold exact counts, bin max_count everything
// at or above it. Small bin indices are counted in LDS first.
__global__ void __launch_bounds__(kTB) k_spectrum(const uint32_t* __restrict__ counts, uint64_t n,
                                                  uint32_t max_count,
                                                  unsigned long long* __restrict__ hist) {
  __shared__ uint32_t h[kLdsBins];
  const uint32_t nl = max_count + 1 < kLdsBins ? max_count + 1 : kLdsBins;
  for (uint32_t i = threadIdx.x; i < nl; i += kTB) h[i] = 0;
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * kTB;
  for (uint64_t i = (uint64_t)blockIdx.x * kTB + threadIdx.x; i < n; i += stride) {
    const uint32_t c = counts[i];
    const uint32_t b = c < max_count ? c : max_count;
    if (b < nl) atomicAdd(&h[b], 1u);
    else atomicAdd(&hist[b], 1ull);
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < nl; i += kTB)
    if (h[i]) atomicAdd(&hist[i], (unsigned long long)h[i]);
}

__global__ void k_zero(unsigned long long* p, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Compaction, step 1: kept pairs per tile.
__global__ void __launch_bounds__(kTB) k_keep_count(const uint32_t* __restrict__ counts,
                                                    uint64_t n, uint32_t min_count,
                                                    unsigned long long* __restrict__ tsum) {
  __shared__ uint32_t s;
  if (threadIdx.x == 0) s = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * kTile;
  uint32_t c = 0;
  for (int j = 0; j < kPer; ++j) {
    const uint64_t i = base + (uint64_t)j * kTB + threadIdx.x;
    c += (i < n && counts[i] >= min_count) ? 1u : 0u;
  }
  atomicAdd(&s, c);
  __syncthreads();
  if (threadIdx.x == 0) tsum[blockIdx.x] = s;
}

// Step 2 (one block): exclusive scan of the tile sums; tsum[nt] = total.
__global__ void __launch_bounds__(1024) k_scan_tiles(unsigned long long* __restrict__ tsum,
                                                     uint64_t nt) {
  __shared__ unsigned long long part[1024];
  const uint64_t per = (nt + 1023) / 1024;
  const uint64_t b = threadIdx.x * per, e = b + per < nt ? b + per : nt;
  unsigned long long s = 0;
  for (uint64_t i = b; i < e; ++i) s += tsum[i];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long run = 0;
    for (int t = 0; t < 1024; ++t) {
      const unsigned long long x = part[t];
      part[t] = run;
      run += x;
    }
    tsum[nt] = run;
  }
  __syncthreads();
  unsigned long long run = part[threadIdx.x];
  for (uint64_t i = b; i < e; ++i) {
    const unsigned long long x = tsum[i];
    tsum[i] = run;
    run += x;
  }
}

// Step 3: each tile writes its kept pairs in order from its offset.
__global__ void __launch_bounds__(kTB) k_keep_write(const uint64_t* __restrict__ keys,
                                                    const uint32_t* __restrict__ counts,
                                                    uint64_t n, int words, uint32_t min_count,
                                                    const unsigned long long* __restrict__ tsum,
                                                    uint64_t* __restrict__ out_keys,
                                                    uint32_t* __restrict__ out_counts) {
  __shared__ uint32_t wsum[kTB / 64 + 1];
  const uint64_t base = (uint64_t)blockIdx.x * kTile;
  unsigned long long at = tsum[blockIdx.x];
  for (int j = 0; j < kPer; ++j) {
    const uint64_t i = base + (uint64_t)j * kTB + threadIdx.x;
    const bool keep = i < n && counts[i] >= min_count;
    // rank among the kept items of this row of the tile, in index order
    const unsigned long long m = __ballot(keep);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) wsum[w] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t before = 0, row = 0;
    for (int v = 0; v < kTB / 64; ++v) {
      if (v < w) before += wsum[v];
      row += wsum[v];
    }
    if (keep) {
      const unsigned long long o = at + before + __popcll(m & ((1ull << lane) - 1));
      out_counts[o] = counts[i];
      for (int q = 0; q < words; ++q) out_keys[words * o + q] = keys[words * i + q];
    }
    at += row;
    __syncthreads();
  }
}

struct Fail {
  int code;
};

void chk(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    (void)hipGetLastError();
    kc::set_last_error(std::string(what) + ": " + hipGetErrorString(e));
    throw Fail{e == hipErrorOutOfMemory ? KC_E_NOMEM : KC_E_DEVICE};
  }
}

int bad(const char* msg) {
  kc::set_last_error(msg);
  return KC_E_INVAL;
}

// Temporary device memory of the merge and the filter: the calling thread's
// buffer, kept between calls (kc_release_scratch frees it).
void* post_scratch(size_t bytes, hipStream_t st) {
  std::string err;
  int code = KC_E_NOMEM;
  void* p = kc::thread_scratch(bytes, st, &err, &code);
  if (!p) {
    kc::set_last_error(err);
    throw Fail{code};
  }
  return p;
}

unsigned grid_of(uint64_t n, uint64_t per, unsigned cap) {
  const uint64_t g = (n + per - 1) / per;
  return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace


extern "C" {

int kc_spectrum(const uint32_t* counts, uint64_t n, uint32_t max_count, uint64_t* host_hist,
                void* stream) {
  kc::set_last_error("");
  if (!host_hist) return bad("host_hist is NULL");
  if (n && !counts) return bad("counts is NULL");
  if (max_count < 1 || max_count > (1u << 24)) return bad("max_count must be in [1, 2^24]");
  const hipStream_t st = (hipStream_t)stream;
  void* d = nullptr;
  try {
    chk(hipMallocAsync(&d, (size_t)(max_count + 1) * 8, st), "hipMallocAsync");
    unsigned long long* hist = (unsigned long long*)d;
    hipLaunchKernelGGL(k_zero, dim3(grid_of(max_count + 1, 256, 1u << 20)), dim3(256), 0, st,
                       hist, (uint64_t)max_count + 1);
    if (n)
      hipLaunchKernelGGL(k_spectrum, dim3(grid_of(n, (uint64_t)kTB * 16, 4096)), dim3(kTB), 0, st,
                         counts, n, max_count, hist);
    chk(hipGetLastError(), "spectrum launch");
    chk(hipMemcpyAsync(host_hist, hist, (size_t)(max_count + 1) * 8, hipMemcpyDeviceToHost, st),
        "hipMemcpyAsync");
    chk(hipFreeAsync(d, st), "hipFreeAsync");
    d = nullptr;
    chk(hipStreamSynchronize(st), "hipStreamSynchronize");
  } catch (const Fail& f) {
    if (d) (void)hipFreeAsync(d, st);
    return f.code;
  }
  return KC_OK;
}

int kc_filter_min_count(const uint64_t* keys, const uint32_t* counts, uint64_t n, int k,
                        uint32_t min_count, uint64_t* out_keys, uint32_t* out_counts,
                        uint64_t* n_out, void* stream) {
  kc::set_last_error("");
  if (!n_out) return bad("n_out is NULL");
  *n_out = 0;
  if (k < 1 || k > 128) return bad("k must be in [1, 128]");
  if (n && (!keys || !counts || !out_keys || !out_counts)) return bad("NULL array");
  if (n == 0) return KC_OK;
  const int words = k <= 32 ? 1 : (k <= 64 ? 2 : 4);
  const hipStream_t st = (hipStream_t)stream;
  const uint64_t nt = (n + kTile - 1) / kTile;
  void* d = nullptr;
  try {
    d = post_scratch((size_t)(nt + 1) * 8, st);
    unsigned long long* tsum = (unsigned long long*)d;
    hipLaunchKernelGGL(k_keep_count, dim3((unsigned)nt), dim3(kTB), 0, st, counts, n, min_count,
                       tsum);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, st, tsum, nt);
    hipLaunchKernelGGL(k_keep_write, dim3((unsigned)nt), dim3(kTB), 0, st, keys, counts, n, words,
                       min_count, tsum, out_keys, out_counts);
    chk(hipGetLastError(), "filter launch");
    uint64_t total = 0;
    chk(hipMemcpyAsync(&total, tsum + nt, 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    chk(hipStreamSynchronize(st), "hipStreamSynchronize");
    *n_out = total;
  } catch (const Fail& f) {
    return f.code;
  }
  return KC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- merging two results

namespace {

// Key i of a result (W = 1, 2 or 4 words, least significant first) as one
// comparable value.
struct Key4 {
  unsigned __int128 lo, hi;
};
__device__ __forceinline__ bool operator<(const Key4& a, const Key4& b) {
  return a.hi != b.hi ? a.hi < b.hi : a.lo < b.lo;
}
__device__ __forceinline__ bool operator==(const Key4& a, const Key4& b) {
  return a.hi == b.hi && a.lo == b.lo;
}
__device__ __forceinline__ bool operator!=(const Key4& a, const Key4& b) { return !(a == b); }

template <int W> struct KeyOf { typedef unsigned __int128 type; };
template <> struct KeyOf<4> { typedef Key4 type; };

template <int W>
__device__ __forceinline__ typename KeyOf<W>::type key_at(const uint64_t* keys, uint64_t i) {
  if constexpr (W == 4) {
    const uint64_t* p = keys + 4 * i;
    return Key4{((unsigned __int128)p[1] << 64) | p[0], ((unsigned __int128)p[3] << 64) | p[2]};
  } else if constexpr (W == 2) {
    return ((unsigned __int128)keys[2 * i + 1] << 64) | keys[2 * i];
  } else {
    return keys[i];
  }
}

template <int W>
__device__ __forceinline__ void key_put(uint64_t* keys, uint64_t i,
                                        const typename KeyOf<W>::type& v) {
  if constexpr (W == 4) {
    keys[4 * i] = (uint64_t)v.lo;
    keys[4 * i + 1] = (uint64_t)(v.lo >> 64);
    keys[4 * i + 2] = (uint64_t)v.hi;
    keys[4 * i + 3] = (uint64_t)(v.hi >> 64);
  } else if constexpr (W == 2) {
    keys[2 * i] = (uint64_t)v;
    keys[2 * i + 1] = (uint64_t)(v >> 64);
  } else {
    keys[i] = (uint64_t)v;
  }
}

constexpr int kMergeItems = 8;

constexpr uint64_t kMergeTile = (uint64_t)kTB * kMergeItems;  // merged positions per block

// Number of a's among the first d merged positions (a first on ties), by
// binary search over i in [lo, hi]: the largest i with a[i-1] <= b[d-i].
template <int W>
__device__ __forceinline__ uint64_t merge_split(const uint64_t* __restrict__ ak, uint64_t na,
                                                const uint64_t* __restrict__ bk, uint64_t nb,
                                                uint64_t d, uint64_t lo, uint64_t hi) {
  while (lo < hi) {
    const uint64_t i = (lo + hi + 1) >> 1;  // candidate: take i items of a
    if (d - i >= nb || !(key_at<W>(bk, d - i) < key_at<W>(ak, i - 1))) lo = i;
    else hi = i - 1;
  }
  return lo;
}

// Split of every block boundary (part[q] for diagonal q * kMergeTile, q =
// 0..nblocks), so that each thread of k_merge searches only its block's window.
template <int W>
__global__ void __launch_bounds__(kTB) k_merge_part(const uint64_t* __restrict__ ak, uint64_t na,
                                                    const uint64_t* __restrict__ bk, uint64_t nb,
                                                    uint64_t nblocks,
                                                    unsigned long long* __restrict__ part) {
  const uint64_t q = (uint64_t)blockIdx.x * kTB + threadIdx.x;
  if (q > nblocks) return;
  const uint64_t total = na + nb;
  const uint64_t d = q * kMergeTile < total ? q * kMergeTile : total;
  part[q] = merge_split<W>(ak, na, bk, nb, d, d > nb ? d - nb : 0, d < na ? d : na);
}

// Merge path: thread t writes merged positions [t*items, t*items + items) of
// the ordered union of a and b (ties: a first). Its start in a is the
// largest i with i + j = d and a[i-1] <= b[j] ... found by binary search.
template <int W>
__global__ void __launch_bounds__(kTB) k_merge(const uint64_t* __restrict__ ak,
                                               const uint32_t* __restrict__ ac, uint64_t na,
                                               const uint64_t* __restrict__ bk,
                                               const uint32_t* __restrict__ bc, uint64_t nb,
                                               uint64_t* __restrict__ mk,
                                               uint32_t* __restrict__ mc,
                                               const unsigned long long* __restrict__ part) {
  const uint64_t total = na + nb;
  const uint64_t d = ((uint64_t)blockIdx.x * kTB + threadIdx.x) * kMergeItems;
  if (d >= total) return;
  // i in [max(0, d - nb), min(d, na)] and within this block's split range
  const uint64_t p0 = part[blockIdx.x], p1 = part[blockIdx.x + 1];
  uint64_t lo = d > nb ? d - nb : 0, hi = d < na ? d : na;
  lo = lo > p0 ? lo : p0;
  hi = hi < p1 ? hi : p1;
  const uint64_t i0 = merge_split<W>(ak, na, bk, nb, d, lo, hi);
  uint64_t i = i0, j = d - i0;
  for (int t = 0; t < kMergeItems && d + t < total; ++t) {
    bool take_a;
    if (i >= na) take_a = false;
    else if (j >= nb) take_a = true;
    else take_a = !(key_at<W>(bk, j) < key_at<W>(ak, i));
    if (take_a) {
      key_put<W>(mk, d + t, key_at<W>(ak, i));
      mc[d + t] = ac[i];
      ++i;
    } else {
      key_put<W>(mk, d + t, key_at<W>(bk, j));
      mc[d + t] = bc[j];
      ++j;
    }
  }
}

// Dedup of the merged sequence: a key present in both inputs sits at two
// neighbouring positions (a's first); the first keeps the summed count.
template <int W>
__global__ void __launch_bounds__(kTB) k_dedup_count(const uint64_t* __restrict__ mk, uint64_t n,
                                                     unsigned long long* __restrict__ tsum) {
  __shared__ uint32_t s;
  if (threadIdx.x == 0) s = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * kTile;
  uint32_t c = 0;
  for (int j = 0; j < kPer; ++j) {
    const uint64_t i = base + (uint64_t)j * kTB + threadIdx.x;
    c += (i < n && (i == 0 || key_at<W>(mk, i) != key_at<W>(mk, i - 1))) ? 1u : 0u;
  }
  atomicAdd(&s, c);
  __syncthreads();
  if (threadIdx.x == 0) tsum[blockIdx.x] = s;
}

template <int W>
__global__ void __launch_bounds__(kTB) k_dedup_write(const uint64_t* __restrict__ mk,
                                                     const uint32_t* __restrict__ mc, uint64_t n,
                                                     const unsigned long long* __restrict__ tsum,
                                                     uint64_t* __restrict__ out_keys,
                                                     uint32_t* __restrict__ out_counts,
                                                     unsigned int* __restrict__ overflow) {
  __shared__ uint32_t wsum[kTB / 64 + 1];
  const uint64_t base = (uint64_t)blockIdx.x * kTile;
  unsigned long long at = tsum[blockIdx.x];
  for (int j = 0; j < kPer; ++j) {
    const uint64_t i = base + (uint64_t)j * kTB + threadIdx.x;
    bool keep = false;
    typename KeyOf<W>::type key{};
    if (i < n) {
      key = key_at<W>(mk, i);
      keep = i == 0 || key != key_at<W>(mk, i - 1);
    }
    const unsigned long long m = __ballot(keep);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) wsum[w] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t before = 0, row = 0;
    for (int v = 0; v < kTB / 64; ++v) {
      if (v < w) before += wsum[v];
      row += wsum[v];
    }
    if (keep) {
      unsigned long long c = mc[i];
      if (i + 1 < n && key_at<W>(mk, i + 1) == key) c += mc[i + 1];
      if (c > 0xFFFFFFFFull) atomicOr(overflow, 1u);
      const unsigned long long o = at + before + __popcll(m & ((1ull << lane) - 1));
      key_put<W>(out_keys, o, key);
      out_counts[o] = (uint32_t)c;
    }
    at += row;
    __syncthreads();
  }
}

}  // namespace

extern "C" int kc_merge_counts(const uint64_t* a_keys, const uint32_t* a_counts, uint64_t na,
                               const uint64_t* b_keys, const uint32_t* b_counts, uint64_t nb,
                               int k, uint64_t* out_keys, uint32_t* out_counts, uint64_t* n_out,
                               void* stream) {
  kc::set_last_error("");
  if (!n_out) return bad("n_out is NULL");
  *n_out = 0;
  if (k < 1 || k > 128) return bad("k must be in [1, 128]");
  if ((na && (!a_keys || !a_counts)) || (nb && (!b_keys || !b_counts)))
    return bad("NULL input array");
  const uint64_t n = na + nb;
  if (n && (!out_keys || !out_counts)) return bad("NULL output array");
  if (n == 0) return KC_OK;
  const int words = k <= 32 ? 1 : (k <= 64 ? 2 : 4);
  const hipStream_t st = (hipStream_t)stream;
  const uint64_t nt = (n + kTile - 1) / kTile;
  void* d = nullptr;
  try {
    // merged sequence, tile sums and the overflow flag in one allocation
    const size_t kb = n * 8 * (size_t)words, cb = n * 4, tb = (nt + 1) * 8;
    const uint64_t nblk = (n + kMergeTile - 1) / kMergeTile;
    // layout: merged keys, counts, (pad to 8), tile sums, flag (16 bytes), splits
    d = post_scratch(kb + cb + 8 + tb + 16 + (nblk + 1) * 8, st);
    uint64_t* mk = (uint64_t*)d;
    uint32_t* mc = (uint32_t*)((char*)d + kb);
    unsigned long long* tsum = (unsigned long long*)((char*)d + kb + cb + (8 - (cb & 7)) % 8);
    unsigned int* ovf = (unsigned int*)(tsum + nt + 1);
    unsigned long long* part = (unsigned long long*)(ovf + 4);
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, (unsigned long long*)ovf, (uint64_t)1);
    const dim3 gm((unsigned)nblk), gt((unsigned)nt), gp((unsigned)((nblk + kTB) / kTB));
    if (words == 4) {
      hipLaunchKernelGGL(k_merge_part<4>, gp, dim3(kTB), 0, st, a_keys, na, b_keys, nb, nblk,
                         part);
      hipLaunchKernelGGL(k_merge<4>, gm, dim3(kTB), 0, st, a_keys, a_counts, na, b_keys, b_counts,
                         nb, mk, mc, part);
      hipLaunchKernelGGL(k_dedup_count<4>, gt, dim3(kTB), 0, st, mk, n, tsum);
    } else if (words == 2) {
      hipLaunchKernelGGL(k_merge_part<2>, gp, dim3(kTB), 0, st, a_keys, na, b_keys, nb, nblk,
                         part);
      hipLaunchKernelGGL(k_merge<2>, gm, dim3(kTB), 0, st, a_keys, a_counts, na, b_keys, b_counts,
                         nb, mk, mc, part);
      hipLaunchKernelGGL(k_dedup_count<2>, gt, dim3(kTB), 0, st, mk, n, tsum);
    } else {
      hipLaunchKernelGGL(k_merge_part<1>, gp, dim3(kTB), 0, st, a_keys, na, b_keys, nb, nblk,
                         part);
      hipLaunchKernelGGL(k_merge<1>, gm, dim3(kTB), 0, st, a_keys, a_counts, na, b_keys, b_counts,
                         nb, mk, mc, part);
      hipLaunchKernelGGL(k_dedup_count<1>, gt, dim3(kTB), 0, st, mk, n, tsum);
    }
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, st, tsum, nt);
    if (words == 4)
      hipLaunchKernelGGL(k_dedup_write<4>, gt, dim3(kTB), 0, st, mk, mc, n, tsum, out_keys,
                         out_counts, ovf);
    else if (words == 2)
      hipLaunchKernelGGL(k_dedup_write<2>, gt, dim3(kTB), 0, st, mk, mc, n, tsum, out_keys,
                         out_counts, ovf);
    else
      hipLaunchKernelGGL(k_dedup_write<1>, gt, dim3(kTB), 0, st, mk, mc, n, tsum, out_keys,
                         out_counts, ovf);
    chk(hipGetLastError(), "merge launch");
    uint64_t h[2] = {0, 0};
    chk(hipMemcpyAsync(&h[0], tsum + nt, 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    chk(hipMemcpyAsync(&h[1], ovf, 4, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    chk(hipStreamSynchronize(st), "hipStreamSynchronize");
    if ((uint32_t)h[1]) {
      kc::set_last_error("a merged count exceeds 2^32-1");
      return KC_E_OVERFLOW;
    }
    *n_out = h[0];
  } catch (const Fail& f) {
    return f.code;
  }
  return KC_OK;
}
