// Device kernels of the canonical k-mer counting path for gfx950 (CDNA4).
//
// Path (one call):
//   pack           ASCII -> 2-bit bases (32 per uint64, base i at bits 2i) plus
//                  two bit masks: invalid byte, last byte of a read.
//   window_hist    every valid window -> canonical key -> histogram over the
//                  first-level key-range shards (top bits of the key).
//   window_scatter every valid window -> its shard's slice of the owner-major
//                  record buffer (each owner's shards are contiguous: the
//                  owner's receive buffer), staged in LDS so that each shard
//                  gets one coalesced run per tile.
//   split_hist /   partitions too large for one LDS table are split by the next
//   split_scatter  key bits (MSD radix step) into sub-partitions.
//   leaf_count     one workgroup per leaf partition: open-addressing hash table
//                  in LDS (linear probing, CAS claim of an EMPTY slot, atomic
//                  add of the count), overflow detection, compaction, bitonic
//                  sort of the distinct keys -> sorted (key, count) pairs.
//   concat         leaves are disjoint key ranges, so concatenating their
//                  sorted pairs in key-range order gives the sorted output.
//   check          device self-check of the output.
//
// Nothing here is a dense contraction: the path is bound by HBM traffic and
// LDS atomics, not by MFMA.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kc_internal.h"

namespace kc {
namespace {

typedef unsigned __int128 u128;

// ---------------------------------------------------------------- key helpers

__device__ __forceinline__ uint64_t mask64(int k) { return k >= 32 ? ~0ull : ((1ull << (2 * k)) - 1); }
__device__ __forceinline__ u128 mask128(int k) {
  return k >= 64 ? ~(u128)0 : (((u128)1 << (2 * k)) - 1);
}

// Reverse the order of the 32 two-bit groups of a word.
__device__ __forceinline__ uint64_t rev2(uint64_t x) {
  x = __builtin_bitreverse64(x);
  return ((x >> 1) & 0x5555555555555555ull) | ((x & 0x5555555555555555ull) << 1);
}

// MurmurHash3 64-bit finalizer (Appleby): slot selection inside hash tables.
__device__ __forceinline__ uint64_t fmix64(uint64_t h) {
  h ^= h >> 33;
  h *= 0xff51afd7ed558ccdull;
  h ^= h >> 33;
  h *= 0xc4ceb9fe1a85ec53ull;
  h ^= h >> 33;
  return h;
}

template <typename K> struct Key;

template <> struct Key<uint64_t> {
  static constexpr bool kWide = false;
  __device__ static uint64_t empty() { return ~0ull; }
  __device__ static uint64_t hash(uint64_t x) { return fmix64(x); }
  __device__ static uint32_t bits(uint64_t x, int shift, int nbits) {
    return (uint32_t)(x >> shift) & ((1u << nbits) - 1u);
  }
  // Canonical key of the window starting at bit offset s (0..62, even) of the
  // little-endian base stream held in words p0, p1 (p2 unused).
  __device__ static uint64_t canon(uint64_t p0, uint64_t p1, uint64_t, int s, int k) {
    uint64_t v = s ? (p0 >> s) | (p1 << (64 - s)) : p0;  // base j of the window at bits 2j
    v &= mask64(k);
    uint64_t rc = ~v & mask64(k);          // complement, base j at 4^j: reverse complement
    uint64_t fwd = rev2(v) >> (64 - 2 * k);  // first base most significant
    return fwd < rc ? fwd : rc;
  }
  __device__ static uint64_t revcomp(uint64_t x, int k) { return rev2(~x & mask64(k)) >> (64 - 2 * k); }
  __device__ static bool in_range(uint64_t x, int k) { return (x & ~mask64(k)) == 0; }
};

template <> struct Key<u128> {
  static constexpr bool kWide = true;
  __device__ static u128 empty() { return ~(u128)0; }
  __device__ static uint64_t hash(u128 x) {
    return fmix64((uint64_t)x ^ fmix64((uint64_t)(x >> 64) + 0x9E3779B97F4A7C15ull));
  }
  __device__ static uint32_t bits(u128 x, int shift, int nbits) {
    return (uint32_t)(x >> shift) & ((1u << nbits) - 1u);
  }
  __device__ static u128 canon(uint64_t p0, uint64_t p1, uint64_t p2, int s, int k) {
    uint64_t lo = s ? (p0 >> s) | (p1 << (64 - s)) : p0;
    uint64_t hi = s ? (p1 >> s) | (p2 << (64 - s)) : p1;
    u128 v = (((u128)hi << 64) | lo) & mask128(k);
    u128 rc = ~v & mask128(k);
    u128 r = ((u128)rev2((uint64_t)v) << 64) | rev2((uint64_t)(v >> 64));
    u128 fwd = r >> (128 - 2 * k);
    return fwd < rc ? fwd : rc;
  }
  __device__ static u128 revcomp(u128 x, int k) {
    u128 c = ~x & mask128(k);
    u128 r = ((u128)rev2((uint64_t)c) << 64) | rev2((uint64_t)(c >> 64));
    return r >> (128 - 2 * k);
  }
  __device__ static bool in_range(u128 x, int k) { return (x & ~mask128(k)) == 0; }
};

// ---------------------------------------------------------------- block scan

// Exclusive scan of one value per thread; returns the prefix, sets *total.
template <int TB>
__device__ __forceinline__ uint32_t block_exscan(uint32_t v, uint32_t* scratch, uint32_t* total) {
  const int tid = threadIdx.x;
  scratch[tid] = v;
  __syncthreads();
  for (int off = 1; off < TB; off <<= 1) {
    uint32_t add = tid >= off ? scratch[tid - off] : 0u;
    __syncthreads();
    scratch[tid] += add;
    __syncthreads();
  }
  uint32_t incl = scratch[tid];
  uint32_t tot = scratch[TB - 1];
  __syncthreads();
  *total = tot;
  return incl - v;
}

// Exclusive scan of an LDS array a[0..n) into out[0..n); returns the total.
template <int TB>
__device__ __forceinline__ uint32_t block_exscan_array(const uint32_t* a, uint32_t* out, int n,
                                                       uint32_t* scratch) {
  const int per = (n + TB - 1) / TB;
  const int b = threadIdx.x * per;
  const int e = min(n, b + per);
  uint32_t s = 0;
  for (int i = b; i < e; ++i) s += a[i];
  uint32_t total;
  uint32_t run = block_exscan<TB>(s, scratch, &total);
  for (int i = b; i < e; ++i) {
    out[i] = run;
    run += a[i];
  }
  __syncthreads();
  return total;
}

// ---------------------------------------------------------------- pack

__device__ __forceinline__ uint32_t base_code(uint32_t b) { return ((b >> 1) ^ (b >> 2)) & 3u; }
__device__ __forceinline__ bool base_valid(uint32_t b) {
  uint32_t u = b | 0x20u;
  return u == 'a' || u == 'c' || u == 'g' || u == 't';
}

// Thread c packs bytes [64c, 64c+64): two packed words, one invalid-mask word
// and one end-mask word (bit j set iff byte 64c+j is the last byte of a read).
__global__ void __launch_bounds__(256) k_pack(const uint8_t* __restrict__ src, uint64_t n_bytes,
                                              const uint64_t* __restrict__ offsets,
                                              uint64_t n_reads, uint64_t off0,
                                              uint64_t* __restrict__ packed,
                                              uint64_t* __restrict__ inv,
                                              uint64_t* __restrict__ endm, uint64_t nchunks,
                                              int aligned) {
  const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nchunks) return;
  const uint64_t g0 = c * 64;
  uint64_t p[2] = {0, 0};
  uint64_t iv = 0;
  if (aligned && g0 + 64 <= n_bytes) {
    const uint4* q = reinterpret_cast<const uint4*>(src + g0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      uint4 x = q[v];
      uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
      for (int d = 0; d < 4; ++d) {
#pragma unroll
        for (int by = 0; by < 4; ++by) {
          const int j = v * 16 + d * 4 + by;
          const uint32_t b = (w[d] >> (8 * by)) & 0xFFu;
          p[j >> 5] |= (uint64_t)base_code(b) << (2 * (j & 31));
          if (!base_valid(b)) iv |= 1ull << j;
        }
      }
    }
  } else {
    for (int j = 0; j < 64; ++j) {
      const uint64_t g = g0 + j;
      if (g < n_bytes) {
        const uint32_t b = src[g];
        p[j >> 5] |= (uint64_t)base_code(b) << (2 * (j & 31));
        if (!base_valid(b)) iv |= 1ull << j;
      } else {
        iv |= 1ull << j;
      }
    }
  }
  packed[2 * c] = p[0];
  packed[2 * c + 1] = p[1];
  inv[c] = iv;
  // Reads whose last byte lies in [g0, g0+64): first the smallest r with
  // offsets[r+1] > off0 + g0 (binary search), then every further end in range.
  uint64_t e = 0;
  if (g0 < n_bytes) {
    uint64_t lo = 0, hi = n_reads;  // search r in [0, n_reads)
    const uint64_t target = off0 + g0;
    while (lo < hi) {
      uint64_t mid = (lo + hi) >> 1;
      if (offsets[mid + 1] > target) hi = mid; else lo = mid + 1;
    }
    for (uint64_t r = lo; r < n_reads; ++r) {
      const uint64_t end = offsets[r + 1];
      if (end > target + 64) break;
      if (end > offsets[r]) e |= 1ull << (end - 1 - target);
    }
  }
  endm[c] = e;
}

// ---------------------------------------------------------------- windows

// Bit i of the result is set iff the window starting at byte g+i (i < S) is
// valid: no invalid byte in [g+i, g+i+k) and no read end in [g+i, g+i+k-1).
// g is a multiple of S; the mask arrays are padded by two words.
__device__ __forceinline__ u128 load_bits(const uint64_t* __restrict__ m, uint64_t g) {
  const uint64_t w = g >> 6;
  const int off = (int)(g & 63);
  const uint64_t a = m[w], b = m[w + 1], c = m[w + 2];
  const uint64_t lo = off ? (a >> off) | (b << (64 - off)) : a;
  const uint64_t hi = off ? (b >> off) | (c << (64 - off)) : b;
  return ((u128)hi << 64) | lo;
}

// r[i] = OR of x[i .. i+len) (len >= 1).
__device__ __forceinline__ u128 smear(u128 x, int len) {
  int l = 1;
  while (2 * l <= len) {
    x |= x >> l;
    l <<= 1;
  }
  if (l < len) x |= x >> (len - l);
  return x;
}

template <int S>
__device__ __forceinline__ uint32_t valid_starts(const uint64_t* __restrict__ inv,
                                                 const uint64_t* __restrict__ endm, uint64_t g,
                                                 int k) {
  u128 bad = smear(load_bits(inv, g), k);
  if (k > 1) bad |= smear(load_bits(endm, g), k - 1);
  return ~(uint32_t)bad & (S >= 32 ? 0xFFFFFFFFu : ((1u << S) - 1u));
}

template <typename K, int S>
__device__ __forceinline__ void load_window_words(const uint64_t* __restrict__ packed, uint64_t g,
                                                  uint64_t& p0, uint64_t& p1, uint64_t& p2) {
  const uint64_t w = g >> 5;
  p0 = packed[w];
  p1 = packed[w + 1];
  p2 = Key<K>::kWide ? packed[w + 2] : 0;
}

template <typename K>
__device__ __forceinline__ uint32_t shard_of(K key, int k, int shard_bits) {
  return (uint32_t)(key >> (2 * k - shard_bits));
}

template <typename K, int S, int TB>
__global__ void __launch_bounds__(TB) k_window_hist(const uint64_t* __restrict__ packed,
                                                    const uint64_t* __restrict__ inv,
                                                    const uint64_t* __restrict__ endm,
                                                    uint64_t n_threads, int k, int shard_bits,
                                                    unsigned long long* __restrict__ hist,
                                                    unsigned long long* __restrict__ wcount) {
  __shared__ uint32_t sh[1 << kMaxShardBits];
  const int nb = 1 << shard_bits;
  for (int i = threadIdx.x; i < nb; i += TB) sh[i] = 0;
  __syncthreads();
  uint32_t w = 0;
  for (uint64_t t = (uint64_t)blockIdx.x * TB + threadIdx.x; t < n_threads;
       t += (uint64_t)gridDim.x * TB) {
    const uint64_t g = t * S;
    uint32_t vm = valid_starts<S>(inv, endm, g, k);
    if (!vm) continue;
    uint64_t p0, p1, p2;
    load_window_words<K, S>(packed, g, p0, p1, p2);
    const int s0 = 2 * (int)(g & 31);
    while (vm) {
      const int i = __builtin_ctz(vm);
      vm &= vm - 1;
      K key = Key<K>::canon(p0, p1, p2, s0 + 2 * i, k);
      atomicAdd(&sh[shard_of(key, k, shard_bits)], 1u);
      ++w;
    }
  }
  // per-wave sum of valid windows, one global atomic per wave
  for (int off = 32; off > 0; off >>= 1) w += __shfl_xor(w, off);
  if ((threadIdx.x & 63) == 0 && w) atomicAdd(wcount, (unsigned long long)w);
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += TB)
    if (sh[i]) atomicAdd(&hist[i], (unsigned long long)sh[i]);
}

// Owner-major scatter of window records into shard slices (cursor[i] starts at
// shard i's slice begin). One tile = TB*S window starts.
template <typename K, int S, int TB>
__global__ void __launch_bounds__(TB) k_window_scatter(const uint64_t* __restrict__ packed,
                                                       const uint64_t* __restrict__ inv,
                                                       const uint64_t* __restrict__ endm,
                                                       uint64_t n_threads, int k, int shard_bits,
                                                       unsigned long long* __restrict__ cursor,
                                                       K* __restrict__ out) {
  constexpr int NBMAX = 1 << kMaxShardBits;
  __shared__ K stage[TB * S];
  __shared__ uint16_t sbin[TB * S];
  __shared__ uint32_t hist[NBMAX];
  __shared__ uint32_t loff[NBMAX];
  __shared__ unsigned long long gbase[NBMAX];
  __shared__ uint32_t scratch[TB];
  const int nb = 1 << shard_bits;
  const uint64_t n_tiles = (n_threads + TB - 1) / TB;
  for (uint64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    for (int i = threadIdx.x; i < nb; i += TB) hist[i] = 0;
    __syncthreads();
    const uint64_t t = tile * TB + threadIdx.x;
    const uint64_t g = t * S;
    uint32_t vm = t < n_threads ? valid_starts<S>(inv, endm, g, k) : 0u;
    K key[S];
    uint32_t bin[S], rank[S];
    if (vm) {
      uint64_t p0, p1, p2;
      load_window_words<K, S>(packed, g, p0, p1, p2);
      const int s0 = 2 * (int)(g & 31);
#pragma unroll
      for (int i = 0; i < S; ++i) {
        if (vm & (1u << i)) {
          key[i] = Key<K>::canon(p0, p1, p2, s0 + 2 * i, k);
          bin[i] = shard_of(key[i], k, shard_bits);
          rank[i] = atomicAdd(&hist[bin[i]], 1u);
        }
      }
    }
    __syncthreads();
    const uint32_t total = block_exscan_array<TB>(hist, loff, nb, scratch);
    for (int i = threadIdx.x; i < nb; i += TB)
      if (hist[i]) gbase[i] = atomicAdd(&cursor[i], (unsigned long long)hist[i]);
#pragma unroll
    for (int i = 0; i < S; ++i) {
      if (vm & (1u << i)) {
        const uint32_t p = loff[bin[i]] + rank[i];
        stage[p] = key[i];
        sbin[p] = (uint16_t)bin[i];
      }
    }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < total; j += TB) {
      const uint32_t b = sbin[j];
      out[gbase[b] + (j - loff[b])] = stage[j];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- split (MSD step)

template <typename K, int TB>
__global__ void __launch_bounds__(TB) k_split_hist(const K* __restrict__ src,
                                                   const SplitItem* __restrict__ items,
                                                   const SplitBin* __restrict__ bins,
                                                   unsigned long long* __restrict__ subhist) {
  __shared__ uint32_t h[1 << kSplitMaxBits];
  const SplitItem it = items[blockIdx.x];
  const SplitBin bn = bins[it.bin];
  const int nsub = 1 << bn.nbits;
  for (int i = threadIdx.x; i < nsub; i += TB) h[i] = 0;
  __syncthreads();
  for (uint64_t r = it.begin + threadIdx.x; r < it.end; r += TB)
    atomicAdd(&h[Key<K>::bits(src[r], bn.shift, bn.nbits)], 1u);
  __syncthreads();
  for (int i = threadIdx.x; i < nsub; i += TB)
    if (h[i]) atomicAdd(&subhist[bn.hist_off + i], (unsigned long long)h[i]);
}

template <typename K, int TB, int R>
__global__ void __launch_bounds__(TB) k_split_scatter(const K* __restrict__ src,
                                                      K* __restrict__ dst,
                                                      const SplitItem* __restrict__ items,
                                                      const SplitBin* __restrict__ bins,
                                                      unsigned long long* __restrict__ cursor) {
  constexpr int NS = 1 << kSplitMaxBits;
  __shared__ K stage[TB * R];
  __shared__ uint8_t ssub[TB * R];
  __shared__ uint32_t hist[NS];
  __shared__ uint32_t loff[NS];
  __shared__ unsigned long long gbase[NS];
  __shared__ uint32_t scratch[TB];
  const SplitItem it = items[blockIdx.x];
  const SplitBin bn = bins[it.bin];
  const int nsub = 1 << bn.nbits;
  for (int i = threadIdx.x; i < nsub; i += TB) hist[i] = 0;
  __syncthreads();
  K key[R];
  uint32_t sub[R], rank[R];
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const uint64_t r = it.begin + threadIdx.x + (uint64_t)j * TB;
    if (r < it.end) {
      key[j] = src[r];
      sub[j] = Key<K>::bits(key[j], bn.shift, bn.nbits);
      rank[j] = atomicAdd(&hist[sub[j]], 1u);
    }
  }
  __syncthreads();
  const uint32_t total = block_exscan_array<TB>(hist, loff, nsub, scratch);
  for (int i = threadIdx.x; i < nsub; i += TB)
    if (hist[i]) gbase[i] = atomicAdd(&cursor[bn.hist_off + i], (unsigned long long)hist[i]);
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const uint64_t r = it.begin + threadIdx.x + (uint64_t)j * TB;
    if (r < it.end) {
      const uint32_t p = loff[sub[j]] + rank[j];
      stage[p] = key[j];
      ssub[p] = (uint8_t)sub[j];
    }
  }
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < total; j += TB) {
    const uint32_t b = ssub[j];
    dst[gbase[b] + (j - loff[b])] = stage[j];
  }
}

// ---------------------------------------------------------------- leaf count

// Bitonic sort of (keys, counts) in LDS, n a power of two.
template <typename K, typename C, int TB>
__device__ __forceinline__ void bitonic_sort(K* keys, C* cnt, uint32_t n) {
  for (uint32_t size = 2; size <= n; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t i = threadIdx.x; i < n / 2; i += TB) {
        const uint32_t lo = (i / stride) * stride * 2 + (i % stride);
        const uint32_t hi = lo + stride;
        const bool asc = (lo & size) == 0;
        const K a = keys[lo], b = keys[hi];
        if ((a > b) == asc) {
          keys[lo] = b;
          keys[hi] = a;
          const C t = cnt[lo];
          cnt[lo] = cnt[hi];
          cnt[hi] = t;
        }
      }
      __syncthreads();
    }
  }
}

__device__ __forceinline__ uint32_t next_pow2(uint32_t x) {
  return x <= 2 ? 2u : 1u << (32 - __builtin_clz(x - 1));
}

// 64-bit keys: EMPTY (all ones) is never a canonical key for k <= 32, so a
// slot is claimed by a 64-bit CAS of the key word itself.
template <int TB, int CMAX>
__global__ void __launch_bounds__(TB) k_leaf_count64(uint64_t* bufA, uint64_t* bufB,
                                                     uint32_t* __restrict__ tmp_cnt,
                                                     const Leaf* __restrict__ leaves,
                                                     uint32_t* __restrict__ d_out,
                                                     int slots_log2) {
  __shared__ unsigned long long tk[CMAX];
  __shared__ uint32_t tc[CMAX];
  __shared__ uint32_t scratch[TB];
  __shared__ uint32_t s_nd;
  __shared__ volatile uint32_t s_ovf;
  const uint32_t C = 1u << slots_log2;
  const uint32_t cmask = C - 1;
  const Leaf lf = leaves[blockIdx.x];
  const uint64_t* src = lf.buf ? bufB : bufA;
  uint64_t* dst = lf.buf ? bufA : bufB;
  const unsigned long long EMPTY = ~0ull;
  for (uint32_t i = threadIdx.x; i < C; i += TB) {
    tk[i] = EMPTY;
    tc[i] = 0;
  }
  if (threadIdx.x == 0) {
    s_nd = 0;
    s_ovf = 0;
  }
  __syncthreads();
  const uint32_t limit = C - (C >> 3);
  for (uint64_t r = lf.begin + threadIdx.x; r < lf.end; r += TB) {
    if (s_ovf) break;
    const unsigned long long key = src[r];
    uint32_t pos = (uint32_t)fmix64(key) & cmask;
    bool done = false;
    for (uint32_t probe = 0; probe < C; ++probe) {
      const unsigned long long prev = atomicCAS(&tk[pos], EMPTY, key);
      if (prev == EMPTY) {
        atomicAdd(&tc[pos], 1u);
        if (atomicAdd(&s_nd, 1u) + 1 >= limit) s_ovf = 1;
        done = true;
        break;
      }
      if (prev == key) {
        atomicAdd(&tc[pos], 1u);
        done = true;
        break;
      }
      pos = (pos + 1) & cmask;
    }
    if (!done) s_ovf = 1;
  }
  __syncthreads();
  if (s_ovf) {
    if (threadIdx.x == 0) d_out[blockIdx.x] = 0xFFFFFFFFu;
    return;
  }
  // compaction to the front of the table (in place, via registers)
  constexpr int PER = CMAX / TB;
  const uint32_t per = C / TB;
  unsigned long long rk[PER];
  uint32_t rc[PER];
  uint32_t mine = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    if ((uint32_t)j < per) {
      rk[j] = tk[threadIdx.x * per + j];
      rc[j] = tc[threadIdx.x * per + j];
      mine += rk[j] != EMPTY;
    }
  }
  uint32_t d;
  uint32_t base = block_exscan<TB>(mine, scratch, &d);
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    if ((uint32_t)j < per && rk[j] != EMPTY) {
      tk[base] = rk[j];
      tc[base] = rc[j];
      ++base;
    }
  }
  __syncthreads();
  const uint32_t n = next_pow2(d);
  for (uint32_t i = d + threadIdx.x; i < n; i += TB) {
    tk[i] = EMPTY;
    tc[i] = 0;
  }
  __syncthreads();
  bitonic_sort<unsigned long long, uint32_t, TB>(tk, tc, n);
  for (uint32_t i = threadIdx.x; i < d; i += TB) {
    dst[lf.begin + i] = tk[i];
    tmp_cnt[lf.begin + i] = tc[i];
  }
  if (threadIdx.x == 0) d_out[blockIdx.x] = d;
}

// 128-bit keys: no 128-bit CAS, so a slot is claimed through its count word:
// 0 = empty, LOCK = being written; the claimer writes the key and then
// publishes the count. Others seeing LOCK retry the same slot; the claimer
// publishes in the same pass without waiting on anyone, so the retry ends.
template <int TB, int CMAX>
__global__ void __launch_bounds__(TB) k_leaf_count128(u128* bufA, u128* bufB,
                                                      uint32_t* __restrict__ tmp_cnt,
                                                      const Leaf* __restrict__ leaves,
                                                      uint32_t* __restrict__ d_out,
                                                      int slots_log2,
                                                      unsigned int* __restrict__ count_overflow) {
  __shared__ u128 tk[CMAX];
  __shared__ unsigned long long tc[CMAX];
  __shared__ uint32_t scratch[TB];
  __shared__ uint32_t s_nd;
  __shared__ volatile uint32_t s_ovf;
  const uint32_t C = 1u << slots_log2;
  const uint32_t cmask = C - 1;
  const Leaf lf = leaves[blockIdx.x];
  const u128* src = lf.buf ? bufB : bufA;
  u128* dst = lf.buf ? bufA : bufB;
  const unsigned long long LOCK = 1ull << 63;
  for (uint32_t i = threadIdx.x; i < C; i += TB) tc[i] = 0;
  if (threadIdx.x == 0) {
    s_nd = 0;
    s_ovf = 0;
  }
  __syncthreads();
  const uint32_t limit = C - (C >> 3);
  for (uint64_t r = lf.begin + threadIdx.x; r < lf.end; r += TB) {
    if (s_ovf) break;
    const u128 key = src[r];
    uint32_t pos = (uint32_t)Key<u128>::hash(key) & cmask;
    uint32_t probe = 0, spins = 0;
    bool done = false;
    while (probe < C) {
      unsigned long long c =
          __hip_atomic_load(&tc[pos], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (c == 0) {
        unsigned long long expect = 0;
        if (__hip_atomic_compare_exchange_strong(&tc[pos], &expect, LOCK, __ATOMIC_ACQ_REL,
                                                 __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP)) {
          tk[pos] = key;
          __hip_atomic_store(&tc[pos], 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
          if (atomicAdd(&s_nd, 1u) + 1 >= limit) s_ovf = 1;
          done = true;
          break;
        }
        c = expect;
      }
      if (c == LOCK) {
        if (++spins > (1u << 22)) break;  // cannot happen; guards against a hang
        continue;
      }
      if (tk[pos] == key) {
        __hip_atomic_fetch_add(&tc[pos], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        done = true;
        break;
      }
      pos = (pos + 1) & cmask;
      ++probe;
    }
    if (!done) s_ovf = 1;
  }
  __syncthreads();
  if (s_ovf) {
    if (threadIdx.x == 0) d_out[blockIdx.x] = 0xFFFFFFFFu;
    return;
  }
  constexpr int PER = CMAX / TB;
  const uint32_t per = C / TB;
  u128 rk[PER];
  unsigned long long rc[PER];
  uint32_t mine = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    if ((uint32_t)j < per) {
      rc[j] = tc[threadIdx.x * per + j];
      rk[j] = tk[threadIdx.x * per + j];
      mine += rc[j] != 0;
    }
  }
  uint32_t d;
  uint32_t base = block_exscan<TB>(mine, scratch, &d);
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    if ((uint32_t)j < per && rc[j] != 0) {
      tk[base] = rk[j];
      tc[base] = rc[j];
      ++base;
    }
  }
  __syncthreads();
  const uint32_t n = next_pow2(d);
  for (uint32_t i = d + threadIdx.x; i < n; i += TB) {
    tk[i] = ~(u128)0;
    tc[i] = 0;
  }
  __syncthreads();
  bitonic_sort<u128, unsigned long long, TB>(tk, tc, n);
  for (uint32_t i = threadIdx.x; i < d; i += TB) {
    dst[lf.begin + i] = tk[i];
    const unsigned long long c = tc[i];
    if (c > 0xFFFFFFFFull) atomicOr(count_overflow, 1u);
    tmp_cnt[lf.begin + i] = (uint32_t)c;
  }
  if (threadIdx.x == 0) d_out[blockIdx.x] = d;
}

// ---------------------------------------------------------------- concat + check

template <typename K>
__global__ void __launch_bounds__(256) k_concat(const K* __restrict__ bufA,
                                                const K* __restrict__ bufB,
                                                const uint32_t* __restrict__ tmp_cnt,
                                                const Leaf* __restrict__ leaves,
                                                const uint32_t* __restrict__ d,
                                                uint64_t* __restrict__ out_keys,
                                                uint32_t* __restrict__ out_counts) {
  const Leaf lf = leaves[blockIdx.x];
  const K* src = lf.buf ? bufA : bufB;  // sorted pairs sit in the other buffer
  const uint32_t n = d[blockIdx.x];
  for (uint32_t i = threadIdx.x; i < n; i += 256) {
    const K key = src[lf.begin + i];
    const uint64_t o = lf.out_off + i;
    if (Key<K>::kWide) {
      out_keys[2 * o] = (uint64_t)key;
      out_keys[2 * o + 1] = (uint64_t)((u128)key >> 64);
    } else {
      out_keys[o] = (uint64_t)key;
    }
    out_counts[o] = tmp_cnt[lf.begin + i];
  }
}

template <typename K>
__device__ __forceinline__ K load_out_key(const uint64_t* keys, uint64_t i) {
  if (Key<K>::kWide) return (K)(((u128)keys[2 * i + 1] << 64) | keys[2 * i]);
  return (K)keys[i];
}

template <typename K>
__global__ void __launch_bounds__(256) k_check(const uint64_t* __restrict__ keys,
                                               const uint32_t* __restrict__ counts, uint64_t n,
                                               int k, CheckResult* res) {
  unsigned long long sum = 0;
  uint32_t ns = 0, nc = 0, nr = 0, nz = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * 256) {
    const K x = load_out_key<K>(keys, i);
    if (i + 1 < n && !(x < load_out_key<K>(keys, i + 1))) ++ns;
    if (!Key<K>::in_range(x, k)) ++nr;
    else if (Key<K>::revcomp(x, k) < x) ++nc;
    if (counts[i] == 0) ++nz;
    sum += counts[i];
  }
  for (int off = 32; off > 0; off >>= 1) {
    sum += __shfl_xor(sum, off);
    ns += __shfl_xor(ns, off);
    nc += __shfl_xor(nc, off);
    nr += __shfl_xor(nr, off);
    nz += __shfl_xor(nz, off);
  }
  if ((threadIdx.x & 63) == 0) {
    if (sum) atomicAdd(&res->sum_counts, sum);
    if (ns) atomicAdd(&res->not_sorted, ns);
    if (nc) atomicAdd(&res->not_canonical, nc);
    if (nr) atomicAdd(&res->out_of_range, nr);
    if (nz) atomicAdd(&res->zero_count, nz);
  }
}

constexpr int kHistTB = 256;
constexpr int kScatterTB64 = 1024;
constexpr int kScatterTB128 = 512;
constexpr int kSplitTB64 = 1024;
constexpr int kSplitTB128 = 512;
constexpr int kSplitR = 8;
constexpr int kLeafTB = 1024;
constexpr int kLeafCmax64 = 8192;
constexpr int kLeafCmax128 = 4096;

inline unsigned grid_for(uint64_t n, unsigned tb, unsigned cap) {
  uint64_t g = (n + tb - 1) / tb;
  if (g > cap) g = cap;
  return g ? (unsigned)g : 1u;
}

}  // namespace

int max_leaf_slots_log2(bool wide) { return wide ? 12 : 13; }
int max_shard_bits() { return kMaxShardBits; }

hipError_t launch_pack(const uint8_t* src, uint64_t n_bytes, const uint64_t* offsets,
                       uint64_t n_reads, uint64_t off0, uint64_t* packed, uint64_t* inv,
                       uint64_t* endm, uint64_t nchunks, hipStream_t s) {
  const int aligned = ((uintptr_t)src & 15) == 0;
  const unsigned grid = (unsigned)((nchunks + 255) / 256);
  hipLaunchKernelGGL(k_pack, dim3(grid), dim3(256), 0, s, src, n_bytes, offsets, n_reads, off0,
                     packed, inv, endm, nchunks, aligned);
  return hipGetLastError();
}

hipError_t launch_window_hist(bool wide, const uint64_t* packed, const uint64_t* inv,
                              const uint64_t* endm, uint64_t n_bytes, int k, int shard_bits,
                              unsigned long long* hist, unsigned long long* wcount,
                              hipStream_t s) {
  const uint64_t nthr = (n_bytes + kWinStarts - 1) / kWinStarts;
  const unsigned grid = grid_for(nthr, kHistTB, 2048);
  if (wide)
    hipLaunchKernelGGL((k_window_hist<u128, kWinStarts, kHistTB>), dim3(grid), dim3(kHistTB), 0,
                       s, packed, inv, endm, nthr, k, shard_bits, hist, wcount);
  else
    hipLaunchKernelGGL((k_window_hist<uint64_t, kWinStarts, kHistTB>), dim3(grid), dim3(kHistTB),
                       0, s, packed, inv, endm, nthr, k, shard_bits, hist, wcount);
  return hipGetLastError();
}

hipError_t launch_window_scatter(bool wide, const uint64_t* packed, const uint64_t* inv,
                                 const uint64_t* endm, uint64_t n_bytes, int k, int shard_bits,
                                 unsigned long long* cursor, void* out, hipStream_t s) {
  const uint64_t nthr = (n_bytes + kWinStarts - 1) / kWinStarts;
  if (wide) {
    const unsigned grid = grid_for(nthr, kScatterTB128, 1u << 20);
    hipLaunchKernelGGL((k_window_scatter<u128, kWinStarts, kScatterTB128>), dim3(grid),
                       dim3(kScatterTB128), 0, s, packed, inv, endm, nthr, k, shard_bits, cursor,
                       (u128*)out);
  } else {
    const unsigned grid = grid_for(nthr, kScatterTB64, 1u << 20);
    hipLaunchKernelGGL((k_window_scatter<uint64_t, kWinStarts, kScatterTB64>), dim3(grid),
                       dim3(kScatterTB64), 0, s, packed, inv, endm, nthr, k, shard_bits, cursor,
                       (uint64_t*)out);
  }
  return hipGetLastError();
}

int split_tile(bool wide) { return wide ? kSplitTB128 * kSplitR : kSplitTB64 * kSplitR; }

hipError_t launch_split_hist(bool wide, const void* src, const SplitItem* items,
                             uint64_t n_items, const SplitBin* bins,
                             unsigned long long* subhist, hipStream_t s) {
  if (!n_items) return hipSuccess;
  if (wide)
    hipLaunchKernelGGL((k_split_hist<u128, 256>), dim3((unsigned)n_items), dim3(256), 0, s,
                       (const u128*)src, items, bins, subhist);
  else
    hipLaunchKernelGGL((k_split_hist<uint64_t, 256>), dim3((unsigned)n_items), dim3(256), 0, s,
                       (const uint64_t*)src, items, bins, subhist);
  return hipGetLastError();
}

hipError_t launch_split_scatter(bool wide, const void* src, void* dst, const SplitItem* items,
                                uint64_t n_items, const SplitBin* bins,
                                unsigned long long* cursor, hipStream_t s) {
  if (!n_items) return hipSuccess;
  if (wide)
    hipLaunchKernelGGL((k_split_scatter<u128, kSplitTB128, kSplitR>), dim3((unsigned)n_items),
                       dim3(kSplitTB128), 0, s, (const u128*)src, (u128*)dst, items, bins, cursor);
  else
    hipLaunchKernelGGL((k_split_scatter<uint64_t, kSplitTB64, kSplitR>), dim3((unsigned)n_items),
                       dim3(kSplitTB64), 0, s, (const uint64_t*)src, (uint64_t*)dst, items, bins,
                       cursor);
  return hipGetLastError();
}

hipError_t launch_leaf_count(bool wide, void* bufA, void* bufB, uint32_t* tmp_cnt,
                             const Leaf* leaves, uint64_t n_leaves, uint32_t* d_out,
                             int slots_log2, unsigned int* count_overflow, hipStream_t s) {
  if (!n_leaves) return hipSuccess;
  if (wide)
    hipLaunchKernelGGL((k_leaf_count128<kLeafTB, kLeafCmax128>), dim3((unsigned)n_leaves),
                       dim3(kLeafTB), 0, s, (u128*)bufA, (u128*)bufB, tmp_cnt, leaves, d_out,
                       slots_log2, count_overflow);
  else
    hipLaunchKernelGGL((k_leaf_count64<kLeafTB, kLeafCmax64>), dim3((unsigned)n_leaves),
                       dim3(kLeafTB), 0, s, (uint64_t*)bufA, (uint64_t*)bufB, tmp_cnt, leaves,
                       d_out, slots_log2);
  return hipGetLastError();
}

hipError_t launch_concat(bool wide, const void* bufA, const void* bufB, const uint32_t* tmp_cnt,
                         const Leaf* leaves, const uint32_t* d, uint64_t n_leaves,
                         uint64_t* out_keys, uint32_t* out_counts, hipStream_t s) {
  if (!n_leaves) return hipSuccess;
  if (wide)
    hipLaunchKernelGGL(k_concat<u128>, dim3((unsigned)n_leaves), dim3(256), 0, s,
                       (const u128*)bufA, (const u128*)bufB, tmp_cnt, leaves, d, out_keys,
                       out_counts);
  else
    hipLaunchKernelGGL(k_concat<uint64_t>, dim3((unsigned)n_leaves), dim3(256), 0, s,
                       (const uint64_t*)bufA, (const uint64_t*)bufB, tmp_cnt, leaves, d, out_keys,
                       out_counts);
  return hipGetLastError();
}

hipError_t launch_check(bool wide, const uint64_t* keys, const uint32_t* counts, uint64_t n,
                        int k, CheckResult* res, hipStream_t s) {
  if (!n) return hipSuccess;
  const unsigned grid = grid_for(n, 256, 4096);
  if (wide)
    hipLaunchKernelGGL(k_check<u128>, dim3(grid), dim3(256), 0, s, keys, counts, n, k, res);
  else
    hipLaunchKernelGGL(k_check<uint64_t>, dim3(grid), dim3(256), 0, s, keys, counts, n, k, res);
  return hipGetLastError();
}

}  // namespace kc
