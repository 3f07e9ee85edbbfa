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

#include <type_traits>

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
  static constexpr int kWords = 1;
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
  __device__ static uint64_t mask(int k) { return mask64(k); }
  __device__ static uint64_t window(uint64_t p0, uint64_t p1, int s, int k) {
    return (s ? (p0 >> s) | (p1 << (64 - s)) : p0) & mask64(k);
  }
  __device__ static uint64_t fwd_of(uint64_t p0, uint64_t p1, uint64_t, int s, int k) {
    return rev2(window(p0, p1, s, k)) >> (64 - 2 * k);
  }
  __device__ static uint64_t rc_of(uint64_t p0, uint64_t p1, uint64_t, int s, int k) {
    return ~window(p0, p1, s, k) & mask64(k);
  }
  __device__ static uint64_t revcomp(uint64_t x, int k) { return rev2(~x & mask64(k)) >> (64 - 2 * k); }
  __device__ static bool in_range(uint64_t x, int k) { return (x & ~mask64(k)) == 0; }
};

// LDS atomics take unsigned long long; same key semantics as uint64_t.
template <> struct Key<unsigned long long> : Key<uint64_t> {};

template <> struct Key<u128> {
  static constexpr bool kWide = true;
  static constexpr int kWords = 2;
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
  __device__ static u128 mask(int k) { return mask128(k); }
  __device__ static u128 window(uint64_t p0, uint64_t p1, uint64_t p2, int s, int k) {
    const uint64_t lo = s ? (p0 >> s) | (p1 << (64 - s)) : p0;
    const uint64_t hi = s ? (p1 >> s) | (p2 << (64 - s)) : p1;
    return (((u128)hi << 64) | lo) & mask128(k);
  }
  __device__ static u128 fwd_of(uint64_t p0, uint64_t p1, uint64_t p2, int s, int k) {
    const u128 v = window(p0, p1, p2, s, k);
    return (((u128)rev2((uint64_t)v) << 64) | rev2((uint64_t)(v >> 64))) >> (128 - 2 * k);
  }
  __device__ static u128 rc_of(uint64_t p0, uint64_t p1, uint64_t p2, int s, int k) {
    return ~window(p0, p1, p2, s, k) & mask128(k);
  }
  __device__ static u128 revcomp(u128 x, int k) {
    u128 c = ~x & mask128(k);
    u128 r = ((u128)rev2((uint64_t)c) << 64) | rev2((uint64_t)(c >> 64));
    return r >> (128 - 2 * k);
  }
  __device__ static bool in_range(u128 x, int k) { return (x & ~mask128(k)) == 0; }
};

// 256-bit keys (k in [65, 128]): two 128-bit halves with the operations the
// key-generic kernels apply to keys (shifts by 0..255, bitwise logic, order).
struct u256 {
  u128 lo, hi;
  u256() = default;
  __device__ constexpr u256(u128 l, u128 h) : lo(l), hi(h) {}
  __device__ constexpr u256(u128 x) : lo(x), hi(0) {}
  __device__ constexpr u256(uint64_t x) : lo(x), hi(0) {}
  __device__ constexpr u256(unsigned long long x) : lo(x), hi(0) {}
  __device__ constexpr u256(uint32_t x) : lo(x), hi(0) {}
  __device__ constexpr u256(int x) : lo((u128)(uint32_t)x), hi(0) {}
  __device__ explicit operator uint32_t() const { return (uint32_t)lo; }
  __device__ explicit operator uint64_t() const { return (uint64_t)lo; }
  __device__ explicit operator unsigned long long() const { return (unsigned long long)lo; }
};
__device__ __forceinline__ u256 operator<<(const u256& a, int s) {
  if (s == 0) return a;
  if (s >= 128) return u256((u128)0, a.lo << (s - 128));
  return u256(a.lo << s, (a.hi << s) | (a.lo >> (128 - s)));
}
__device__ __forceinline__ u256 operator>>(const u256& a, int s) {
  if (s == 0) return a;
  if (s >= 128) return u256(a.hi >> (s - 128), (u128)0);
  return u256((a.lo >> s) | (a.hi << (128 - s)), a.hi >> s);
}
__device__ __forceinline__ u256 operator|(const u256& a, const u256& b) {
  return u256(a.lo | b.lo, a.hi | b.hi);
}
__device__ __forceinline__ u256 operator&(const u256& a, const u256& b) {
  return u256(a.lo & b.lo, a.hi & b.hi);
}
__device__ __forceinline__ u256 operator~(const u256& a) { return u256(~a.lo, ~a.hi); }
__device__ __forceinline__ u256& operator|=(u256& a, const u256& b) { return a = a | b; }
__device__ __forceinline__ bool operator==(const u256& a, const u256& b) {
  return a.lo == b.lo && a.hi == b.hi;
}
__device__ __forceinline__ bool operator!=(const u256& a, const u256& b) { return !(a == b); }
__device__ __forceinline__ bool operator<(const u256& a, const u256& b) {
  return a.hi != b.hi ? a.hi < b.hi : a.lo < b.lo;
}
__device__ __forceinline__ bool operator>(const u256& a, const u256& b) { return b < a; }

// Reverse the order of the 128 two-bit groups.
__device__ __forceinline__ u256 rev2_256(const u256& v) {
  const u128 lo = ((u128)rev2((uint64_t)(v.hi >> 64)) << 0) | ((u128)rev2((uint64_t)v.hi) << 64);
  const u128 hi = ((u128)rev2((uint64_t)(v.lo >> 64)) << 0) | ((u128)rev2((uint64_t)v.lo) << 64);
  return u256(lo, hi);
}

__device__ __forceinline__ u128 low_bits128(int bits) {
  return bits >= 128 ? ~(u128)0 : (((u128)1 << bits) - 1);
}

// Keys of more than 64 bases: built from five packed words (up to 128 bases
// starting anywhere in the first word).
template <> struct Key<u256> {
  static constexpr bool kWide = true;
  static constexpr int kWords = 4;
  __device__ static u256 mask(int k) {
    const int b = 2 * k;
    return b <= 128 ? u256(low_bits128(b), (u128)0) : u256(~(u128)0, low_bits128(b - 128));
  }
  __device__ static uint32_t bits(const u256& x, int shift, int nbits) {
    return (uint32_t)(x >> shift) & ((1u << nbits) - 1u);
  }
  __device__ static uint64_t hash(const u256& x) {
    uint64_t h = fmix64((uint64_t)(x.hi >> 64) + 0x9E3779B97F4A7C15ull);
    h = fmix64((uint64_t)x.hi ^ h);
    h = fmix64((uint64_t)(x.lo >> 64) ^ h);
    return fmix64((uint64_t)x.lo ^ h);
  }
  // Bases [s/2, s/2 + k) of the little-endian base stream in p[0..4] (base j
  // of the window at bits 2j), s even, 0 <= s <= 62.
  __device__ static u256 window(const uint64_t (&p)[5], int s, int k) {
    uint64_t w[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i] = s ? (p[i] >> s) | (p[i + 1] << (64 - s)) : p[i];
    return u256(((u128)w[1] << 64) | w[0], ((u128)w[3] << 64) | w[2]) & mask(k);
  }
  __device__ static u256 fwd_of_window(const u256& v, int k) { return rev2_256(v) >> (256 - 2 * k); }
  __device__ static u256 rc_of_window(const u256& v, int k) { return ~v & mask(k); }
  __device__ static u256 revcomp(const u256& x, int k) {
    return rev2_256(~x & mask(k)) >> (256 - 2 * k);
  }
  __device__ static bool in_range(const u256& x, int k) { return (x & ~mask(k)) == u256(0); }
};

// ---------------------------------------------------------------- block scans

// Exclusive scan of one value per thread (wave shuffles, then one wave over
// the wave totals); returns the prefix and sets *total. wsum holds TB/64 values.
template <int TB, typename T>
__device__ __forceinline__ T block_exscan(T v, T* wsum, T* total) {
  constexpr int NW = TB / 64;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  T x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  if (wid == 0) {
    T w = lane < NW ? wsum[lane] : (T)0;
#pragma unroll
    for (int off = 1; off < NW; off <<= 1) {
      const T y = __shfl_up(w, off);
      if (lane >= off) w += y;
    }
    if (lane < NW) wsum[lane] = w;  // inclusive prefix of the wave totals
  }
  __syncthreads();
  const T before = wid ? wsum[wid - 1] : (T)0;
  *total = wsum[NW - 1];
  __syncthreads();
  return before + x - v;
}

// Exclusive scan of an LDS array a[0..n) into out[0..n); returns the total.
// If maxv is not null it receives the largest a[i].
template <int TB>
__device__ __forceinline__ uint32_t block_exscan_array(const uint32_t* a, uint32_t* out, int n,
                                                       uint32_t* wsum, uint32_t* maxv = nullptr) {
  const int per = (n + TB - 1) / TB;
  const int b = threadIdx.x * per;
  const int e = min(n, b + per);
  uint32_t s = 0, m = 0;
  for (int i = b; i < e; ++i) {
    s += a[i];
    m = max(m, a[i]);
  }
  if (maxv) {
    for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) atomicMax(maxv, m);
  }
  uint32_t total;
  uint32_t run = block_exscan<TB, uint32_t>(s, wsum, &total);
  for (int i = b; i < e; ++i) {
    out[i] = run;
    run += a[i];
  }
  __syncthreads();
  return total;
}

// In-place exclusive scan of a[0..n) (counts become offsets); returns the total.
template <int TB>
__device__ __forceinline__ uint32_t block_exscan_inplace(uint32_t* a, int n, uint32_t* wsum) {
  const int per = (n + TB - 1) / TB;
  const int b = threadIdx.x * per;
  const int e = min(n, b + per);
  uint32_t s = 0;
  for (int i = b; i < e; ++i) s += a[i];
  uint32_t total;
  uint32_t run = block_exscan<TB, uint32_t>(s, wsum, &total);
  for (int i = b; i < e; ++i) {
    const uint32_t x = a[i];
    a[i] = run;
    run += x;
  }
  __syncthreads();
  return total;
}

__global__ void k_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------- pack

__device__ __forceinline__ uint32_t base_code(uint32_t b) { return ((b >> 1) ^ (b >> 2)) & 3u; }
// Top bit of each byte of v set iff that byte is not zero (no carry between bytes).
__device__ __forceinline__ uint32_t nonzero_bytes(uint32_t v) {
  return (((v & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | v) & 0x80808080u;
}
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
        // four bytes at once (SWAR): base_code of each byte, then the four
        // 2-bit codes gathered into 8 bits; a byte is invalid iff its
        // lowercase form differs from each of a, c, g, t (nonzero_bytes sets
        // a byte's top bit iff the byte is not 0), the four top bits gathered
        // into 4 bits by one multiply
        const int j = v * 16 + d * 4;
        const uint32_t c = ((w[d] >> 1) ^ (w[d] >> 2)) & 0x03030303u;
        const uint32_t t = c | (c >> 6);
        p[j >> 5] |= (uint64_t)((t & 0xFu) | ((t >> 12) & 0xF0u)) << (2 * (j & 31));
        const uint32_t l = w[d] | 0x20202020u;
        const uint32_t bad = nonzero_bytes(l ^ 0x61616161u) & nonzero_bytes(l ^ 0x63636363u) &
                             nonzero_bytes(l ^ 0x67676767u) & nonzero_bytes(l ^ 0x74747474u);
        iv |= (uint64_t)(((bad & 0x80808080u) * 0x00204081u) >> 28) << j;
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
  endm[c] = 0;  // read ends are set by k_read_ends, launched after this kernel
}

// Read-end mask: bit of the last byte of every non-empty read (thread per read).
__global__ void __launch_bounds__(256) k_read_ends(const uint64_t* __restrict__ offsets,
                                                   uint64_t n_reads, uint64_t off0,
                                                   unsigned long long* __restrict__ endm) {
  const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_reads) return;
  const uint64_t b = offsets[r], e = offsets[r + 1];
  if (e > b) {
    const uint64_t pos = e - 1 - off0;
    atomicOr(&endm[pos >> 6], 1ull << (pos & 63));
  }
}

// ---------------------------------------------------------------- windows

// Window validity. Bit j of valid[w] is set iff the window of k bytes
// starting at byte 64w + j is valid: no invalid byte in it and no read end
// before its last byte. The mask is built once per k by k_valid_mask, so that
// the window kernels test a start with one shift.

// Bits [64w, 64w + 128) of a bit array (the arrays are padded by two words).
__device__ __forceinline__ u128 load_bits(const uint64_t* __restrict__ m, uint64_t w) {
  return ((u128)m[w + 1] << 64) | m[w];
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

// The same over 256 bits, for keys of more than 64 bases (64 + k - 1 may pass
// 128 bits; the arrays are padded by five words).
__device__ __forceinline__ u256 load_bits256(const uint64_t* __restrict__ m, uint64_t w) {
  return u256(((u128)m[w + 1] << 64) | m[w], ((u128)m[w + 3] << 64) | m[w + 2]);
}

__device__ __forceinline__ u256 smear256(u256 x, int len) {
  int l = 1;
  while (2 * l <= len) {
    x |= x >> l;
    l <<= 1;
  }
  if (l < len) x |= x >> (len - l);
  return x;
}

// One thread per mask word w in [w_begin, w_end).
template <bool WIDE>
__global__ void __launch_bounds__(256) k_valid_mask(const uint64_t* __restrict__ inv,
                                                    const uint64_t* __restrict__ endm,
                                                    uint64_t w_begin, uint64_t w_end, int k,
                                                    uint64_t* __restrict__ valid) {
  const uint64_t w = w_begin + (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (w >= w_end) return;
  uint64_t bad;
  if constexpr (WIDE) {
    u256 b = smear256(load_bits256(inv, w), k);
    if (k > 1) b |= smear256(load_bits256(endm, w), k - 1);
    bad = (uint64_t)b;
  } else {
    u128 b = smear(load_bits(inv, w), k);
    if (k > 1) b |= smear(load_bits(endm, w), k - 1);
    bad = (uint64_t)b;
  }
  valid[w] = ~bad;
}

// Valid starts among the S window starts g .. g+S-1 (g a multiple of S, S
// dividing 64): bit i for start g+i.
template <int S>
__device__ __forceinline__ uint32_t valid_starts(const uint64_t* __restrict__ valid, uint64_t g) {
  return (uint32_t)(valid[g >> 6] >> (g & 63)) & (S >= 32 ? 0xFFFFFFFFu : ((1u << S) - 1u));
}

template <typename K, int S>
__device__ __forceinline__ void load_window_words(const uint64_t* __restrict__ packed, uint64_t g,
                                                  uint64_t& p0, uint64_t& p1, uint64_t& p2) {
  const uint64_t w = g >> 5;
  p0 = packed[w];
  p1 = packed[w + 1];
  p2 = Key<K>::kWide ? packed[w + 2] : 0;
}

// Canonical keys of the S windows starting at bytes g .. g+S-1 (g a multiple
// of S, S dividing 32). The first is built directly from the packed words,
// the others by rolling one base in: fwd = ((fwd << 2) | x) & mask and
// rc = (rc >> 2) | ((3 - x) << 2(k-1)), x being the base at g+i+k-1.
// Keys of invalid starts are computed too (the caller masks them).
template <typename K, int S>
__device__ __forceinline__ void canon_run(uint64_t p0, uint64_t p1, uint64_t p2, uint64_t g, int k,
                                          K (&out)[S]) {
  const int s0 = (int)(g & 31);
  out[0] = Key<K>::canon(p0, p1, p2, 2 * s0, k);
  K fwd = Key<K>::fwd_of(p0, p1, p2, 2 * s0, k);
  K rc = Key<K>::rc_of(p0, p1, p2, 2 * s0, k);
  const K mask = Key<K>::mask(k);
  const int top = 2 * (k - 1);
#pragma unroll
  for (int i = 1; i < S; ++i) {
    const int p = s0 + i + k - 1;  // position of the incoming base within words p0..p2
    const uint64_t w = p < 32 ? p0 : (p < 64 ? p1 : p2);
    const uint32_t x = (uint32_t)(w >> (2 * (p & 31))) & 3u;
    fwd = ((fwd << 2) | (K)x) & mask;
    rc = (rc >> 2) | ((K)(3u - x) << top);
    out[i] = fwd < rc ? fwd : rc;
  }
}

// canon_run for keys of more than 64 bases, from five packed words (the
// incoming base of window i sits at most 158 bases past the first word).
template <int S>
__device__ __forceinline__ void canon_run256(const uint64_t (&p)[5], uint64_t g, int k,
                                             u256 (&out)[S]) {
  const int s0 = (int)(g & 31);
  const u256 v = Key<u256>::window(p, 2 * s0, k);
  u256 fwd = Key<u256>::fwd_of_window(v, k);
  u256 rc = Key<u256>::rc_of_window(v, k);
  out[0] = fwd < rc ? fwd : rc;
  const u256 mask = Key<u256>::mask(k);
  const int top = 2 * (k - 1);
#pragma unroll
  for (int i = 1; i < S; ++i) {
    const int q = s0 + i + k - 1;  // position of the incoming base within p[0..4]
    const int wi = q >> 5;
    const uint64_t w = wi == 0 ? p[0] : wi == 1 ? p[1] : wi == 2 ? p[2] : wi == 3 ? p[3] : p[4];
    const uint32_t x = (uint32_t)(w >> (2 * (q & 31))) & 3u;
    fwd = ((fwd << 2) | u256(x)) & mask;
    rc = (rc >> 2) | (u256(3u - x) << top);
    out[i] = fwd < rc ? fwd : rc;
  }
}

template <typename K>
__device__ __forceinline__ uint32_t shard_of(const K& key, int keybits, int shard_bits) {
  return (uint32_t)(key >> (keybits - shard_bits));
}

// Keys of a thread's S window starts. Plain counting: the canonical k-mer. In
// a batch of read sets, the key of a window is (set id within its k-class <<
// 2k) | canonical k-mer, so that sorting keys sorts by set, then k-mer; windows
// of sets outside the class are dropped from vm. Returns the updated vm.
template <typename K, typename Kc, int S, bool BATCH>
__device__ __forceinline__ uint32_t window_keys(const uint64_t* __restrict__ packed, uint64_t g,
                                                int k, uint32_t vm, const BatchSets& bs,
                                                K (&key)[S]) {
  Kc c[S];
  if constexpr (Key<Kc>::kWords == 4) {
    const uint64_t w = g >> 5;
    uint64_t p[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) p[i] = packed[w + i];
    canon_run256<S>(p, g, k, c);
  } else {
    uint64_t p0, p1, p2;
    load_window_words<Kc, S>(packed, g, p0, p1, p2);
    canon_run<Kc, S>(p0, p1, p2, g, k, c);
  }
  if constexpr (!BATCH) {
#pragma unroll
    for (int i = 0; i < S; ++i) key[i] = (K)c[i];
    return vm;
  } else {
  uint32_t lo = 0, hi = bs.n_sets - 1;  // last set whose first byte is <= g
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (bs.set_byte_off[mid] <= g) lo = mid; else hi = mid - 1;
  }
  uint32_t set = lo;
#pragma unroll
  for (int i = 0; i < S; ++i) {
    if (!(vm & (1u << i))) continue;
    while (set + 1 < bs.n_sets && g + i >= bs.set_byte_off[set + 1]) ++set;
    const uint32_t loc = bs.set_local[set];
    if (loc == kNoSet) vm &= ~(1u << i);
    // (a class of one k = 32 set has no set-id bits: no shift by the key width)
    else key[i] = (2 * k < (int)(8 * sizeof(K)) ? ((K)loc << (2 * k)) : (K)0) | (K)c[i];
  }
  return vm;
  }
}

// 24 bits of the packed stream (p1:p0) from bit q (q < 128 - 24).
__device__ __forceinline__ uint32_t bits24(uint64_t p0, uint64_t p1, int q) {
  const uint64_t lo = q >= 64 ? p1 >> (q - 64) : (p0 >> q) | (q ? p1 << (64 - q) : 0ull);
  return (uint32_t)lo & 0xFFFFFFu;
}

// Shard histogram over the owner scatter's tiles: tile j holds the window
// starts [w_begin + j*tile_starts, w_begin + (j+1)*tile_starts) ∩ [.., w_end),
// taken S per thread. Totals go to hist[0, nb); the counts of the tiles of
// class c = j mod kXcds to hist[(1 + c)*nb, ..) (gridDim.x is a multiple of
// kXcds, so all of a workgroup's tiles are of class blockIdx.x mod kXcds).
template <typename K, typename Kc, int S, int TB, bool BATCH>
__global__ void __launch_bounds__(TB) k_window_hist(const uint64_t* __restrict__ packed,
                                                    const uint64_t* __restrict__ valid,
                                                    uint64_t w_begin, uint64_t w_end,
                                                    uint64_t tile_starts, int k, int keybits,
                                                    int shard_bits, BatchSets bs,
                                                    unsigned long long* __restrict__ hist,
                                                    unsigned long long* __restrict__ wcount) {
  __shared__ uint32_t sh[1 << kMaxShardBits];
  const int nb = 1 << shard_bits;
  for (int i = threadIdx.x; i < nb; i += TB) sh[i] = 0;
  __syncthreads();
  uint32_t w = 0;
  const uint64_t n_tiles = (w_end - w_begin + tile_starts - 1) / tile_starts;
  for (uint64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const uint64_t g_end = min(w_end, w_begin + (tile + 1) * tile_starts);
    for (uint64_t g = w_begin + tile * tile_starts + (uint64_t)threadIdx.x * S; g < g_end;
         g += (uint64_t)TB * S) {
      uint32_t vm = valid_starts<S>(valid, g);
      if (!vm) continue;
      if constexpr (!BATCH && std::is_same<Kc, uint64_t>::value && S <= 8) {
        if (k >= 5) {
          // only the shard is needed: the top bits of min(fwd, rc) are the
          // smaller of the top bits of fwd and of rc (if those are equal, so
          // are both keys' top bits). The top 10 bits of fwd are its first 5
          // bases, those of rc the complements of its last 5 bases, last first.
          const uint64_t w0 = g >> 5;
          const uint64_t p0 = packed[w0], p1 = packed[w0 + 1];
          const int s0 = (int)(g & 31);
          const uint32_t head = bits24(p0, p1, 2 * s0);            // bases g .. g+11
          const uint32_t tail = bits24(p0, p1, 2 * (s0 + k - 5));  // bases g+k-5 .. g+k+6
          // the 12 head bases in reverse order (each base's 2-bit code kept):
          // reverse all bits, then swap the two bits of every base
          const uint32_t hb = __builtin_bitreverse32(head) >> 8;
          const uint32_t hr = ((hb >> 1) & 0x555555u) | ((hb & 0x555555u) << 1);
#pragma unroll
          for (int i = 0; i < S; ++i) {
            if (!(vm & (1u << i))) continue;
            // bases g+i .. g+i+4, the first most significant
            const uint32_t f = (hr >> (2 * (7 - i))) & 0x3FFu;
            const uint32_t r = ((tail >> (2 * i)) & 0x3FFu) ^ 0x3FFu;
            atomicAdd(&sh[min(f, r) >> (10 - shard_bits)], 1u);
          }
          w += __builtin_popcount(vm);
          continue;
        }
      }
      K keys[S];
      vm = window_keys<K, Kc, S, BATCH>(packed, g, k, vm, bs, keys);
#pragma unroll
      for (int i = 0; i < S; ++i)
        if (vm & (1u << i)) atomicAdd(&sh[shard_of(keys[i], keybits, shard_bits)], 1u);
      w += __builtin_popcount(vm);
    }
  }
  // per-wave sum of valid windows, one global atomic per wave
  for (int off = 32; off > 0; off >>= 1) w += __shfl_xor(w, off);
  if ((threadIdx.x & 63) == 0 && w) atomicAdd(wcount, (unsigned long long)w);
  __syncthreads();
  unsigned long long* const hc = hist + (uint64_t)(1 + blockIdx.x % kXcds) * nb;
  for (int i = threadIdx.x; i < nb; i += TB)
    if (sh[i]) {
      atomicAdd(&hist[i], (unsigned long long)sh[i]);
      atomicAdd(&hc[i], (unsigned long long)sh[i]);
    }
}

// Owner-major scatter of window records into shard slices (cursor[x*nb + i]
// starts where tile class x's part of shard i's slice begins). One tile =
// TB*S window starts: the tile's records are ranked per shard in LDS, each
// shard's run reserves its place in its class's part with one global atomic,
// and the runs leave LDS as coalesced writes.
template <typename K, typename Kc, int S, int TB, bool BATCH>
__device__ __forceinline__ void window_scatter_body(const uint64_t* __restrict__ packed,
                                                    const uint64_t* __restrict__ valid,
                                                    uint64_t t_begin, uint64_t t_end, int k,
                                                    int keybits, int shard_bits, BatchSets bs,
                                                    unsigned long long* __restrict__ cursor,
                                                    K* __restrict__ out) {
  constexpr int NBMAX = 1 << kMaxShardBits;
  __shared__ K stage[TB * S];
  __shared__ uint32_t loff[NBMAX];  // per shard: records in the tile, then their run offsets
  __shared__ unsigned long long gbase[NBMAX];
  __shared__ uint32_t wsum[TB / 64];
  const int nb = 1 << shard_bits;
  const uint64_t n_tiles = (t_end - t_begin + TB - 1) / TB;
  for (uint64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    // tiles of class tile mod kXcds take their runs from their own part of
    // each shard slice (cursor[class * nb + shard], sized by k_window_hist):
    // the concurrent tiles of one XCD (workgroups are dealt to the XCDs in
    // turn) then write adjacent runs, whose shared 64-byte segments meet in
    // that XCD's L2 instead of going to memory in halves
    unsigned long long* const cls_cursor = cursor + (tile % kXcds) * (uint64_t)nb;
    for (int i = threadIdx.x; i < nb; i += TB) loff[i] = 0;
    __syncthreads();
    const uint64_t t = t_begin + tile * TB + threadIdx.x;
    const uint64_t g = t * S;
    uint32_t vm = t < t_end ? valid_starts<S>(valid, g) : 0u;
    K key[S];
    uint32_t rank[S];  // (the shard is recomputed from the key: fewer live registers)
    if (vm) {
      vm = window_keys<K, Kc, S, BATCH>(packed, g, k, vm, bs, key);
#pragma unroll
      for (int i = 0; i < S; ++i)
        if (vm & (1u << i)) rank[i] = atomicAdd(&loff[shard_of(key[i], keybits, shard_bits)], 1u);
    }
    __syncthreads();
    const uint32_t total = block_exscan_inplace<TB>(loff, nb, wsum);
    for (int i = threadIdx.x; i < nb; i += TB) {
      const uint32_t cnt = (i + 1 < nb ? loff[i + 1] : total) - loff[i];
      if (cnt) gbase[i] = atomicAdd(&cls_cursor[i], (unsigned long long)cnt);
    }
#pragma unroll
    for (int i = 0; i < S; ++i)
      if (vm & (1u << i)) stage[loff[shard_of(key[i], keybits, shard_bits)] + rank[i]] = key[i];
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < total; j += TB) {
      const K kk = stage[j];  // its shard again from the key: cheaper than staging it
      const uint32_t b = shard_of(kk, keybits, shard_bits);
      out[gbase[b] + (j - loff[b])] = kk;
    }
    __syncthreads();
  }
}

template <typename K, typename Kc, int S, int TB, bool BATCH>
__global__ void __launch_bounds__(TB) k_window_scatter(const uint64_t* __restrict__ packed,
                                                       const uint64_t* __restrict__ valid,
                                                       uint64_t t_begin, uint64_t t_end, int k,
                                                       int keybits, int shard_bits, BatchSets bs,
                                                       unsigned long long* __restrict__ cursor,
                                                       K* __restrict__ out) {
  window_scatter_body<K, Kc, S, TB, BATCH>(packed, valid, t_begin, t_end, k, keybits,
                                           shard_bits, bs, cursor, out);
}

// Plain 64-bit keys: registers capped so that two 1024-thread workgroups
// share a CU (their LDS fits twice), which hides the per-tile barriers and
// atomics. (The batch form keeps more values live and stays uncapped.)
// The same with 16 window starts per thread: a tile of 16,384 records (128 KiB
// of LDS staging, one workgroup per CU) gives each of many shards a run twice
// as long per tile.
template <typename K, typename Kc, int S, int TB, bool BATCH>
__global__ void __launch_bounds__(TB)
k_window_scatter64w(const uint64_t* __restrict__ packed, const uint64_t* __restrict__ valid, uint64_t t_begin, uint64_t t_end, int k,
                    int keybits, int shard_bits, BatchSets bs,
                    unsigned long long* __restrict__ cursor, K* __restrict__ out) {
  window_scatter_body<K, Kc, S, TB, BATCH>(packed, valid, t_begin, t_end, k, keybits,
                                           shard_bits, bs, cursor, out);
}

template <typename K, typename Kc, int S, int TB, bool BATCH>
__global__ void __launch_bounds__(TB) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_window_scatter64(const uint64_t* __restrict__ packed, const uint64_t* __restrict__ valid, uint64_t t_begin, uint64_t t_end, int k,
                   int keybits, int shard_bits, BatchSets bs,
                   unsigned long long* __restrict__ cursor, K* __restrict__ out) {
  window_scatter_body<K, Kc, S, TB, BATCH>(packed, valid, t_begin, t_end, k, keybits,
                                           shard_bits, bs, cursor, out);
}

// ---------------------------------------------------------------- planning (one block)

constexpr int kPlanTB = 1024;

__device__ __forceinline__ int ceil_log2_dev(uint64_t x) {
  return x <= 1 ? 0 : 64 - __builtin_clzll(x - 1);
}

// Shard plan: owner-major record ranges, split decision per shard, split
// work items, leaf slot offsets (leaf slots follow key order).
__global__ void __launch_bounds__(kPlanTB) k_plan_shards(
    const unsigned long long* __restrict__ hist, const int* __restrict__ order, int shard_bits,
    int keybits, uint64_t leaf_target, uint64_t leaf_attempt, int tile,
    unsigned long long* __restrict__ sbegin, unsigned long long* __restrict__ cursor,
    SplitBin* __restrict__ bins, unsigned long long* __restrict__ item_off,
    unsigned long long* __restrict__ subhist, DevState* __restrict__ st) {
  __shared__ unsigned long long wsum[kPlanTB / 64];
  const int nb = 1 << shard_bits;  // <= kPlanTB
  const int t = threadIdx.x;
  unsigned long long total;
  // owner-major exclusive scan: the t-th shard in owner order
  const int co = t < nb ? order[t] : 0;
  const unsigned long long ho = t < nb ? hist[co] : 0ull;
  const unsigned long long b0 = block_exscan<kPlanTB, unsigned long long>(ho, wsum, &total);
  if (t < nb) {
    sbegin[co] = b0;
    // each class's part of the slice: after the earlier classes' records
    unsigned long long c = b0;
    for (int x = 0; x < kXcds; ++x) {
      cursor[(uint64_t)x * nb + co] = c;
      c += hist[(uint64_t)(1 + x) * nb + co];
    }
  }
  // split decision for shard t (key order)
  const unsigned long long h = t < nb ? hist[t] : 0ull;
  int nbits = 0;
  const int remaining = keybits - shard_bits;
  if (h > leaf_attempt && remaining > 0) {
    nbits = ceil_log2_dev((h + leaf_target - 1) / leaf_target);
    nbits = max(1, min(nbits, min(kSplitMaxBits, remaining)));
  }
  const unsigned long long L = h == 0 ? 0ull : (nbits ? (1ull << nbits) : 1ull);
  const unsigned long long loff = block_exscan<kPlanTB, unsigned long long>(L, wsum, &total);
  const unsigned long long n_leaves = total;
  const unsigned long long ni = nbits ? (h + tile - 1) / tile : 0ull;
  const unsigned long long ioff = block_exscan<kPlanTB, unsigned long long>(ni, wsum, &total);
  const unsigned long long n_items = total;
  if (t < nb) {
    bins[t] = SplitBin{loff, (uint32_t)(keybits - shard_bits - nbits), (uint32_t)nbits};
    item_off[t] = ioff;
    if (!nbits && h) subhist[loff] = h;  // split shards' counters were cleared before
  }
  if (t == 0) {
    item_off[nb] = n_items;
    st->n_items = n_items;
    st->n_leaves = n_leaves;
  }
}

// Split work items: item i belongs to the shard c with item_off[c] <= i < item_off[c+1].
__global__ void k_plan_items(const unsigned long long* __restrict__ hist,
                             const unsigned long long* __restrict__ sbegin,
                             const unsigned long long* __restrict__ item_off, int shard_bits,
                             int tile, const DevState* __restrict__ st,
                             SplitItem* __restrict__ items) {
  const int nb = 1 << shard_bits;
  const unsigned long long n = st->n_items;
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (unsigned long long)gridDim.x * blockDim.x) {
    int lo = 0, hi = nb - 1;  // last c with item_off[c] <= i
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (item_off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    const unsigned long long a = sbegin[lo] + (i - item_off[lo]) * (unsigned long long)tile;
    items[i] = SplitItem{a, min(sbegin[lo] + hist[lo], a + (unsigned long long)tile), (uint32_t)lo, 0};
  }
}

// Leaf table (key order) and sub-bin cursors: block c handles shard c.
__global__ void __launch_bounds__(kPlanTB) k_plan_leaves(
    const unsigned long long* __restrict__ hist, const unsigned long long* __restrict__ sbegin,
    const SplitBin* __restrict__ bins, int shard_bits,
    const unsigned long long* __restrict__ subhist, Leaf* __restrict__ leaves,
    unsigned long long* __restrict__ cursor, int merge_cshift, int ncls, uint64_t cls_stride) {
  __shared__ unsigned long long wsum[kPlanTB / 64];
  const int c = blockIdx.x;
  const unsigned long long h = hist[c];
  if (!h) return;
  const SplitBin b = bins[c];
  if (b.nbits == 0) {
    if (threadIdx.x == 0) leaves[b.hist_off] = Leaf{sbegin[c], sbegin[c] + h, 0u, (uint32_t)shard_bits};
    return;
  }
  const uint32_t nsub = 1u << b.nbits;  // <= kPlanTB
  const uint32_t j = threadIdx.x;
  unsigned long long n = 0;
  if (j < nsub)
    for (int x = 0; x < ncls; ++x) n += subhist[x * cls_stride + b.hist_off + j];
  unsigned long long total;
  const unsigned long long off = block_exscan<kPlanTB, unsigned long long>(n, wsum, &total);
  if (j < nsub) {
    const unsigned long long run = sbegin[c] + off;
    leaves[b.hist_off + j] = Leaf{run, run + n, 1u, (uint32_t)(shard_bits + b.nbits),
                                  (uint32_t)merge_cshift, (uint32_t)c};
    // each item class's part of the sub-bin: after the earlier classes' records
    unsigned long long at = run;
    for (int x = 0; x < ncls; ++x) {
      cursor[x * cls_stride + b.hist_off + j] = at;
      at += subhist[x * cls_stride + b.hist_off + j];
    }
  }
}

// ---------------------------------------------------------------- refinement support

// Indices (any order) and entries of the leaves whose tables overflowed.
__global__ void k_list_overflowed(const uint32_t* __restrict__ d, uint64_t n,
                                  const Leaf* __restrict__ leaves, uint32_t* __restrict__ list,
                                  Leaf* __restrict__ out, unsigned long long* __restrict__ count) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x; i0 < n; i0 += stride) {
    const uint64_t i = i0 + threadIdx.x;
    const bool ovf = i < n && d[i] == kLeafOverflow;
    const unsigned long long m = __ballot(ovf);
    if (!m) continue;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)m) - 1;
    unsigned long long base = 0;
    if (lane == leader) base = atomicAdd(count, (unsigned long long)__popcll(m));
    base = __shfl(base, leader);
    if (ovf) {
      const unsigned long long at = base + __popcll(m & ((1ull << lane) - 1));
      list[at] = (uint32_t)i;
      out[at] = leaves[i];
    }
  }
}

// Entries each old leaf occupies in the refined list: 1, or (for an
// overflowed leaf) the number of its parts, set by k_splice_root_counts.
__global__ void k_splice_counts(const uint32_t* __restrict__ d, uint64_t n,
                                uint32_t* __restrict__ cnt) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) cnt[i] = d[i] == kLeafOverflow ? 0u : 1u;
}

__global__ void k_splice_root_counts(const uint32_t* __restrict__ root_leaf,
                                     const uint32_t* __restrict__ nparts, uint32_t R,
                                     uint32_t* __restrict__ cnt) {
  const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < R) cnt[root_leaf[r]] = nparts[r];
}

// Kept leaves move to pos[i]; the parts of root r fill pos[root_leaf[r]] onwards.
__global__ void k_splice_keep(const Leaf* __restrict__ leaves, const uint32_t* __restrict__ d,
                              const unsigned long long* __restrict__ pos, uint64_t n,
                              Leaf* __restrict__ out, uint32_t* __restrict__ out_d) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && d[i] != kLeafOverflow) {
    out[pos[i]] = leaves[i];
    out_d[pos[i]] = d[i];
  }
}

__global__ void k_splice_parts(const uint32_t* __restrict__ root_leaf,
                               const uint32_t* __restrict__ part_begin,
                               const uint32_t* __restrict__ nparts, uint32_t R,
                               const Leaf* __restrict__ parts, const uint32_t* __restrict__ part_d,
                               const unsigned long long* __restrict__ pos, Leaf* __restrict__ out,
                               uint32_t* __restrict__ out_d) {
  for (uint32_t r = blockIdx.x; r < R; r += gridDim.x) {
    const unsigned long long at = pos[root_leaf[r]];
    const uint32_t b = part_begin[r];
    for (uint32_t p = threadIdx.x; p < nparts[r]; p += blockDim.x) {
      out[at + p] = parts[b + p];
      out_d[at + p] = part_d[b + p];
    }
  }
}

// Before a second-chance count of overflowed leaves: the flag is raised again
// by that count's own overflows (and by the output-offset scan, from the leaf
// counts).
__global__ void k_clear_overflow(DevState* __restrict__ st) {
  if (threadIdx.x == 0) st->overflow = 0;
}

// Leaves above the small-leaf size go to a list of their own (order
// irrelevant); with huge != nullptr, leaves of more than huge_min records go
// straight to that list instead (st->n_ovf), for the second count's larger
// table: such leaves are the dense clusters that overflow the first table
// (on 40,000,000 reads at k = 31 the overflowed leaves average 147,000
// records, the others 4,600), and the first count would read part of them
// before giving up.
__global__ void k_classify_leaves(const Leaf* __restrict__ leaves, DevState* __restrict__ st,
                                  uint64_t small_max, uint32_t* __restrict__ large,
                                  uint64_t huge_min, uint32_t* __restrict__ huge) {
  const unsigned long long n = st->n_leaves;
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
  const int lane = threadIdx.x & 63;
  for (unsigned long long i0 = (unsigned long long)blockIdx.x * blockDim.x; i0 < n; i0 += stride) {
    const unsigned long long i = i0 + threadIdx.x;
    const Leaf lf = i < n ? leaves[i] : Leaf{0, 0, 0, 0, 0, 0};
    const uint64_t len = lf.end - lf.begin;
    const bool to_huge = huge && len > huge_min;
    const bool big = !to_huge && len > small_max;
    const unsigned long long m = __ballot(big);
    if (m) {
      const int leader = __ffsll((long long)m) - 1;
      unsigned long long base = 0;
      if (lane == leader) base = atomicAdd(&st->n_large, (unsigned long long)__popcll(m));
      base = __shfl(base, leader);
      if (big) large[base + __popcll(m & ((1ull << lane) - 1))] = (uint32_t)i;
    }
    const unsigned long long mh = __ballot(to_huge);
    if (mh) {
      const int leader = __ffsll((long long)mh) - 1;
      unsigned long long base = 0;
      if (lane == leader) base = atomicAdd(&st->n_ovf, (unsigned long long)__popcll(mh));
      base = __shfl(base, leader);
      if (to_huge) huge[base + __popcll(mh & ((1ull << lane) - 1))] = (uint32_t)i;
    }
  }
}

// Output offsets: exclusive scan of the leaf counts in leaf (= key) order, in
// three steps (tile sums, scan of tile sums, tile scans). Overflowed leaves
// count zero and raise st->overflow.
constexpr int kScanTB = 256, kScanPer = 16, kScanTile = kScanTB * kScanPer;

__global__ void __launch_bounds__(kScanTB) k_scan_reduce(const uint32_t* __restrict__ d,
                                                         DevState* __restrict__ st,
                                                         unsigned long long* __restrict__ bsum) {
  __shared__ unsigned long long wsum[kScanTB / 64];
  const unsigned long long n = st->n_leaves;
  const unsigned long long base = (unsigned long long)blockIdx.x * kScanTile;
  unsigned long long s = 0;
  uint32_t ovf = 0;
  for (int j = 0; j < kScanPer; ++j) {
    const unsigned long long i = base + (unsigned long long)j * kScanTB + threadIdx.x;
    if (i < n) {
      const uint32_t x = d[i];
      if (x == kLeafOverflow) ovf = 1;
      else s += x;
    }
  }
  if (ovf) atomicOr(&st->overflow, 1u);
  unsigned long long total;
  (void)block_exscan<kScanTB, unsigned long long>(s, wsum, &total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kPlanTB) k_scan_top(unsigned long long* __restrict__ bsum,
                                                      uint32_t nblocks, DevState* __restrict__ st) {
  __shared__ unsigned long long wsum[kPlanTB / 64];
  const uint32_t per = (nblocks + kPlanTB - 1) / kPlanTB;
  const uint32_t b = threadIdx.x * per, e = min(nblocks, b + per);
  unsigned long long s = 0;
  for (uint32_t i = b; i < e; ++i) s += bsum[i];
  unsigned long long total;
  unsigned long long run = block_exscan<kPlanTB, unsigned long long>(s, wsum, &total);
  for (uint32_t i = b; i < e; ++i) {
    const unsigned long long x = bsum[i];
    bsum[i] = run;
    run += x;
  }
  if (threadIdx.x == 0) st->D = total;
}

__global__ void __launch_bounds__(kScanTB) k_scan_down(const uint32_t* __restrict__ d,
                                                       const DevState* __restrict__ st,
                                                       const unsigned long long* __restrict__ bsum,
                                                       unsigned long long* __restrict__ out_off) {
  __shared__ unsigned long long wsum[kScanTB / 64];
  const unsigned long long n = st->n_leaves;
  // thread t owns kScanPer consecutive leaves of the tile
  const unsigned long long base = (unsigned long long)blockIdx.x * kScanTile +
                                  (unsigned long long)threadIdx.x * kScanPer;
  uint32_t v[kScanPer];
  unsigned long long s = 0;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    const unsigned long long i = base + j;
    v[j] = i < n ? d[i] : 0u;
    if (v[j] == kLeafOverflow) v[j] = 0;
    s += v[j];
  }
  unsigned long long total;
  unsigned long long run = bsum[blockIdx.x] + block_exscan<kScanTB, unsigned long long>(s, wsum, &total);
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    const unsigned long long i = base + j;
    if (i < n) out_off[i] = run;
    run += v[j];
  }
}

// ---------------------------------------------------------------- split (MSD step)

template <typename K, int TB>
__global__ void __launch_bounds__(TB) k_split_hist(const K* __restrict__ src,
                                                   const SplitItem* __restrict__ items,
                                                   const DevState* __restrict__ st,
                                                   const SplitBin* __restrict__ bins,
                                                   unsigned long long* __restrict__ subhist,
                                                   int ncls, uint64_t cls_stride) {
  __shared__ uint32_t h[1 << kSplitMaxBits];
  const unsigned long long n_items = st->n_items;
  for (unsigned long long w = blockIdx.x; w < n_items; w += gridDim.x) {
    const SplitItem it = items[w];
    // counts of item class w mod ncls (the split scatter's cursor classes)
    unsigned long long* const sh = subhist + (w % ncls) * cls_stride;
    const SplitBin bn = bins[it.bin];
    const int nsub = 1 << bn.nbits;
    for (int i = threadIdx.x; i < nsub; i += TB) h[i] = 0;
    __syncthreads();
    // loads of a batch are issued together, then counted
    constexpr int RB = 8;
    for (uint64_t r0 = it.begin; r0 < it.end; r0 += (uint64_t)TB * RB) {
      K kb[RB];
#pragma unroll
      for (int j = 0; j < RB; ++j) {
        const uint64_t r = r0 + (uint64_t)j * TB + threadIdx.x;
        if (r < it.end) kb[j] = src[r];
      }
#pragma unroll
      for (int j = 0; j < RB; ++j) {
        const uint64_t r = r0 + (uint64_t)j * TB + threadIdx.x;
        if (r < it.end) atomicAdd(&h[Key<K>::bits(kb[j], bn.shift, bn.nbits)], 1u);
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nsub; i += TB)
      if (h[i]) atomicAdd(&sh[bn.hist_off + i], (unsigned long long)h[i]);
    __syncthreads();
  }
}

template <typename K, int TB, int R>
__global__ void __launch_bounds__(TB) k_split_scatter(const K* __restrict__ src,
                                                      K* __restrict__ dst,
                                                      const SplitItem* __restrict__ items,
                                                      const DevState* __restrict__ st,
                                                      const SplitBin* __restrict__ bins,
                                                      unsigned long long* __restrict__ cursor,
                                                      int ncls, uint64_t cls_stride) {
  constexpr int NS = 1 << kSplitMaxBits;
  __shared__ K stage[TB * R];
  __shared__ uint32_t hist[NS];  // per sub-bin: records in the tile, then their run offsets
  uint32_t* const loff = hist;
  __shared__ unsigned long long gbase[NS];
  __shared__ uint32_t wsum[TB / 64];
  const unsigned long long n_items = st->n_items;
  // the records of the workgroup's next item are loaded while the current
  // one's runs leave LDS (its keys' registers are free once it is staged)
  K key[R];
  SplitItem it = blockIdx.x < n_items ? items[blockIdx.x] : SplitItem{0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < R; ++j) {
    const uint64_t r = it.begin + threadIdx.x + (uint64_t)j * TB;
    if (r < it.end) key[j] = src[r];
  }
  for (unsigned long long w = blockIdx.x; w < n_items; w += gridDim.x) {
    const SplitBin bn = bins[it.bin];
    const int nsub = 1 << bn.nbits;
    // items of class w mod ncls take their runs from their own part of each
    // sub-bin (as in the owner scatter: with ncls = kXcds and the workgroups
    // of one class on one XCD, the partial segments of adjacent runs meet in
    // that XCD's L2)
    unsigned long long* const cls_cursor = cursor + (w % ncls) * cls_stride;
    for (int i = threadIdx.x; i < nsub; i += TB) hist[i] = 0;
    __syncthreads();
    uint32_t sub[R], rank[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const uint64_t r = it.begin + threadIdx.x + (uint64_t)j * TB;
      if (r < it.end) {
        sub[j] = Key<K>::bits(key[j], bn.shift, bn.nbits);
        rank[j] = atomicAdd(&hist[sub[j]], 1u);
      }
    }
    __syncthreads();
    const uint32_t total = block_exscan_inplace<TB>(hist, nsub, wsum);
    for (int i = threadIdx.x; i < nsub; i += TB) {
      const uint32_t cnt = (i + 1 < nsub ? loff[i + 1] : total) - loff[i];
      if (cnt) gbase[i] = atomicAdd(&cls_cursor[bn.hist_off + i], (unsigned long long)cnt);
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const uint64_t r = it.begin + threadIdx.x + (uint64_t)j * TB;
      if (r < it.end) {
        const uint32_t p = loff[sub[j]] + rank[j];
        stage[p] = key[j];
      }
    }
    __syncthreads();
    const unsigned long long wn = w + gridDim.x;
    const SplitItem nx = wn < n_items ? items[wn] : SplitItem{0, 0, 0, 0};
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const uint64_t r = nx.begin + threadIdx.x + (uint64_t)j * TB;
      if (r < nx.end) key[j] = src[r];
    }
    for (uint32_t j = threadIdx.x; j < total; j += TB) {
      const K kk = stage[j];
      const uint32_t b = Key<K>::bits(kk, bn.shift, bn.nbits);
      dst[gbase[b] + (j - loff[b])] = kk;
    }
    it = nx;
    __syncthreads();
  }
}

// Split scatter with pre-aggregation of equal keys (the heavy-hitter
// aggregation of Section IV-D, on one tile of one shard's records: keys that
// occur many times in the input are concentrated in one shard and one
// sub-bin, where their copies meet in the tile). After the tile is staged by
// sub-bin in LDS, each thread takes R consecutive staged records; a run of
// equal keys among them (always inside one sub-bin) leaves as one record with
// its length minus one in bits [cshift, 64), where the key's top bits (the
// shard, common to the leaf) were. The first record of each thread's segment
// starts a run, so a run never exceeds R. The tile's cursors advance by the
// records written.
template <int TB, int R>
__global__ void __launch_bounds__(TB) k_split_scatter_merge(const uint64_t* __restrict__ src,
                                                            uint64_t* __restrict__ dst,
                                                            const SplitItem* __restrict__ items,
                                                            const DevState* __restrict__ st,
                                                            const SplitBin* __restrict__ bins,
                                                            unsigned long long* __restrict__ cursor,
                                                            int cshift) {
  constexpr int NS = 1 << kSplitMaxBits;
  __shared__ uint64_t stage[TB * R];
  __shared__ uint32_t loff[NS];        // per sub-bin: records of the tile, then their offsets
  __shared__ uint32_t mstart[NS + 1];  // per sub-bin: offset of its first merged record
  __shared__ uint32_t tbase[TB];       // per thread: merged records before its segment
  __shared__ unsigned long long gbase[NS];
  __shared__ uint32_t wsum[TB / 64];
  const uint64_t low = (1ull << cshift) - 1;
  const unsigned long long n_items = st->n_items;
  for (unsigned long long w = blockIdx.x; w < n_items; w += gridDim.x) {
    const SplitItem it = items[w];
    const SplitBin bn = bins[it.bin];
    const int nsub = 1 << bn.nbits;
    for (int i = threadIdx.x; i < nsub; i += TB) loff[i] = 0;
    __syncthreads();
    uint64_t key[R];
    uint32_t sub[R], rank[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const uint64_t r = it.begin + threadIdx.x + (uint64_t)j * TB;
      if (r < it.end) {
        key[j] = src[r];
        sub[j] = Key<uint64_t>::bits(key[j], bn.shift, bn.nbits);
        rank[j] = atomicAdd(&loff[sub[j]], 1u);
      }
    }
    __syncthreads();
    const uint32_t total = block_exscan_inplace<TB>(loff, nsub, wsum);
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const uint64_t r = it.begin + threadIdx.x + (uint64_t)j * TB;
      if (r < it.end) stage[loff[sub[j]] + rank[j]] = key[j];
    }
    __syncthreads();
    // runs of equal keys in this thread's segment [R*t, R*t + R) of the stage
    const uint32_t s0 = (uint32_t)threadIdx.x * R;
    uint64_t seg[R];
    uint32_t heads = 0;  // bit j: a run starts at s0 + j
#pragma unroll
    for (int j = 0; j < R; ++j) {
      const uint32_t i = s0 + j;
      seg[j] = i < total ? stage[i] : 0;
      if (i < total && (j == 0 || seg[j] != seg[j - 1])) heads |= 1u << j;
    }
    uint32_t nh_all;
    const uint32_t base = block_exscan<TB, uint32_t>(__builtin_popcount(heads), wsum, &nh_all);
    tbase[threadIdx.x] = base;
    __syncthreads();
    // merged records before each sub-bin: heads before its first staged record
    for (int b = threadIdx.x; b <= nsub; b += TB) {
      const uint32_t i = b < nsub ? loff[b] : total;
      if (i >= total) {
        mstart[b] = nh_all;
        continue;
      }
      const uint32_t t = i / R, j0 = t * R;
      uint32_t h = tbase[t];
      for (uint32_t q = j0; q < i; ++q) h += (q == j0 || stage[q] != stage[q - 1]) ? 1u : 0u;
      mstart[b] = h;
    }
    __syncthreads();  // every staged record has been read: the stage is rewritten below
    {
      uint32_t at = base;
#pragma unroll
      for (int j = 0; j < R; ++j) {
        if (!(heads & (1u << j))) continue;
        const uint32_t rest = heads >> (j + 1);
        const uint32_t next = rest ? (uint32_t)(j + 1 + __builtin_ctz(rest)) : (uint32_t)R;
        const uint32_t end = min(next, total - s0);
        const uint64_t len = end - (uint32_t)j;
        stage[at++] = ((len - 1) << cshift) | (seg[j] & low);
      }
    }
    for (int b = threadIdx.x; b < nsub; b += TB) {
      const uint32_t cnt = mstart[b + 1] - mstart[b];
      if (cnt) gbase[b] = atomicAdd(&cursor[bn.hist_off + b], (unsigned long long)cnt);
    }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < nh_all; j += TB) {
      const uint64_t kk = stage[j];
      const uint32_t b = Key<uint64_t>::bits(kk, bn.shift, bn.nbits);
      dst[gbase[b] + (j - mstart[b])] = kk;
    }
    __syncthreads();
  }
}

// Records of pre-aggregated leaves end where the split scatter's cursor
// stopped (fewer records than windows).
__global__ void k_leaf_ends(Leaf* __restrict__ leaves, const unsigned long long* __restrict__ cursor,
                            const DevState* __restrict__ st) {
  const unsigned long long n = st->n_leaves;
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (unsigned long long)gridDim.x * blockDim.x)
    if (leaves[i].cshift) leaves[i].end = cursor[i];
}

// ---------------------------------------------------------------- leaf count

// Bitonic sort of (keys, counts) in LDS, n a power of two (fallback sort).
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

// Table slot of a 64-bit key: multiply-shift (Knuth) of a 32-bit fold of the
// key; collisions are resolved by linear probing, so only speed depends on it.
__device__ __forceinline__ uint32_t slot_hash(uint64_t key, int bits) {
  const uint32_t f = (uint32_t)key * 0x9E3779B1u + (uint32_t)(key >> 32) * 0x85EBCA77u;
  return (f ^ (f >> 15)) * 0x2C1B3C6Du >> (32 - bits);
}

// Workgroup-scope flag in LDS (a volatile LDS variable would be accessed with
// flat instructions that also wait for all outstanding global memory operations).
__device__ __forceinline__ uint32_t ovf_get(uint32_t* f) {
  return __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void ovf_set(uint32_t* f) {
  __hip_atomic_store(f, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t next_pow2(uint32_t x) {
  return x <= 2 ? 2u : 1u << (32 - __builtin_clz(x - 1));
}

// Table slots for a leaf of n records: enough that n distinct keys stay below
// 7/8 load, at least TB, at most CMAX.
template <int TB, int CMAX>
__device__ __forceinline__ uint32_t leaf_slots(uint64_t n, uint32_t cmax_rt) {
  const uint64_t want = n + n / 7 + 1;
  uint32_t c = want >= cmax_rt ? cmax_rt : next_pow2((uint32_t)want);
  return c < (uint32_t)TB ? (uint32_t)TB : c;
}

// Epilogue shared by both key widths: the table (tk, tc) has been filled with
// Cn slots. The distinct keys are grouped by a counting sort on the key bits
// just below the leaf's common prefix; each key then finds its place inside
// its group by counting the smaller keys of the group, and the pair is written
// to dst/tmp_cnt at [begin, begin + d) in key order. Keys of one group share a
// long prefix when sequencing errors sit near the k-mer's end (the erroneous
// copies of one k-mer), so groups are not always tiny; a group larger than
// kRankMax switches the leaf to a bitonic sort. Cn >> GSHIFT groups: aux holds
// 2 * Cn >> GSHIFT counters. Returns d.
constexpr uint32_t kRankMax = 256;

template <typename K, typename C, int TB, int PER, int GSHIFT>
__device__ __forceinline__ uint32_t leaf_sort_write(K* tk, C* tc, uint32_t* aux, uint32_t* wsum,
                                                    uint32_t* s_max, uint32_t Cn, int keybits,
                                                    int prefix_bits, K* __restrict__ dst,
                                                    uint32_t* __restrict__ tmp_cnt,
                                                    uint64_t begin, bool (*occupied)(C)) {
  K rk[PER];
  C rc[PER];
  uint32_t rank[PER], bk[PER];
#pragma unroll
  for (int j = 0; j < PER; ++j) {  // slot j*TB + tid: consecutive lanes, consecutive slots
    const uint32_t s = (uint32_t)j * TB + threadIdx.x;
    rc[j] = 0;
    if (s < Cn) {
      rk[j] = tk[s];
      rc[j] = tc[s];
    }
  }
  int nbk_bits = 31 - __builtin_clz(Cn) - GSHIFT;
  if (nbk_bits > keybits - prefix_bits) nbk_bits = keybits - prefix_bits;
  const uint32_t nbk = 1u << nbk_bits;
  const int shift = keybits - prefix_bits - nbk_bits;
  for (uint32_t i = threadIdx.x; i < nbk; i += TB) aux[i] = 0;
  if (threadIdx.x == 0) *s_max = 0;
  __syncthreads();  // table copied to registers; group counters cleared
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    if ((uint32_t)j * TB >= Cn) break;  // uniform: Cn is a multiple of TB
    // every slot adds 0 or 1 (empty slots add 0 to a spread-out counter), so
    // no branch per slot
    const bool o = occupied(rc[j]);
    const uint32_t s = (uint32_t)j * TB + threadIdx.x;
    bk[j] = o ? (nbk_bits ? Key<K>::bits(rk[j], shift, nbk_bits) : 0u) : (s & (nbk - 1));
    rank[j] = atomicAdd(&aux[bk[j]], o ? 1u : 0u);
  }
  __syncthreads();
  const uint32_t d = block_exscan_array<TB>(aux, aux + nbk, (int)nbk, wsum, s_max);
  const uint32_t maxb = *s_max;
  const uint32_t* boff = aux + nbk;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    if (occupied(rc[j])) {
      const uint32_t p = boff[bk[j]] + rank[j];
      tk[p] = rk[j];
      tc[p] = rc[j];
    }
  }
  __syncthreads();
  if (maxb <= kRankMax) {
    for (uint32_t i = threadIdx.x; i < d; i += TB) {
      const K x = tk[i];
      const uint32_t b = nbk_bits ? Key<K>::bits(x, shift, nbk_bits) : 0u;
      const uint32_t a = boff[b], m = aux[b];
      uint32_t r = 0;
      uint32_t t = a;
      for (; t + 4 <= a + m; t += 4)
        r += (uint32_t)(tk[t] < x) + (uint32_t)(tk[t + 1] < x) + (uint32_t)(tk[t + 2] < x) +
             (uint32_t)(tk[t + 3] < x);
      for (; t < a + m; ++t) r += tk[t] < x;
      dst[begin + a + r] = x;
      tmp_cnt[begin + a + r] = (uint32_t)tc[i];
    }
    return d;
  }
  const uint32_t n2 = next_pow2(d);
  for (uint32_t i = d + threadIdx.x; i < n2; i += TB) {
    tk[i] = ~(K)0;
    tc[i] = 0;
  }
  __syncthreads();
  bitonic_sort<K, C, TB>(tk, tc, n2);
  for (uint32_t i = threadIdx.x; i < d; i += TB) {
    dst[begin + i] = tk[i];
    tmp_cnt[begin + i] = (uint32_t)tc[i];
  }
  return d;
}

__device__ bool occ32(uint32_t c) { return c != 0; }
__device__ bool occ64(unsigned long long c) { return c != 0; }

// One-word leaf tables: the epilogue's counting sort uses Cn/8 groups (8 KiB
// of group counters for 4,096 slots instead of 32 KiB with Cn/2), so that
// three 512-thread workgroups, 24 waves, share a CU (53 KB of LDS each, and
// registers capped for 6 waves per SIMD: 79 VGPRs, no spills): 27.1 -> 25.7
// ms for the large leaves of 40,000,000 reads at k = 31, 23.8 -> 21.9 ms at
// k = 21, against two workgroups per CU.
constexpr int kLeafGroupShift = 3;
constexpr int kLeafOccTB = 512;
constexpr int kLeafOccWaves = 6;

// 64-bit keys: EMPTY (all ones) is never a canonical key for k <= 32, so a
// slot is claimed by a 64-bit CAS of the key word itself; the count is then
// added with an atomic add. FULL_FIRST: the first table is the full one (the
// parts of a leaf that overflowed are rich in distinct keys: a half table
// would mostly fill up and be retried).
// MERGED: some leaves may hold pre-aggregated records (Leaf::cshift); the
// plain instantiation has no decoding in its insert loop.
// list != nullptr: the leaves listed there, *n_list of them (large ones, or
// those whose table overflowed in an earlier launch), with the records and
// distinct keys of the leaves counted added to acc[0] and acc[1]; else every
// leaf of at most small_max records. ovf_list != nullptr: the leaves whose
// table overflows are also appended there (count in st->n_ovf) for a second
// launch with a larger table.
template <int TB, int CMAX, int R, bool FULL_FIRST, bool MERGED>
__global__ void __launch_bounds__(TB)
__attribute__((amdgpu_waves_per_eu(TB == kLeafOccTB ? kLeafOccWaves : 1)))
k_leaf_count64(int keybits, uint64_t* bufA, uint64_t* bufB,
                                                     uint32_t* __restrict__ tmp_cnt,
                                                     const Leaf* __restrict__ leaves,
                                                     DevState* __restrict__ st,
                                                     uint32_t* __restrict__ d_out,
                                                     int slots_log2,
                                                     const uint32_t* __restrict__ list,
                                                     const unsigned long long* __restrict__ n_list,
                                                     uint32_t* __restrict__ ovf_list,
                                                     unsigned long long* __restrict__ acc,
                                                     uint64_t small_max) {
  __shared__ unsigned long long tk[CMAX];
  __shared__ uint32_t tc[CMAX];
  __shared__ uint32_t aux[(2 * CMAX) >> kLeafGroupShift];
  __shared__ uint32_t wsum[TB / 64];
  __shared__ uint32_t s_nd, s_max, s_cov;
  __shared__ unsigned long long s_sum, s_windows;
  __shared__ uint32_t s_ovf;  // accessed only through ovf_get / ovf_set
  const unsigned long long EMPTY = ~0ull;
  const uint32_t cmax_rt = 1u << slots_log2;
  const unsigned long long count = list ? *n_list : st->n_leaves;
  unsigned long long my_records = 0, my_distinct = 0;  // thread 0: this workgroup's totals
  for (unsigned long long it = blockIdx.x; it < count; it += gridDim.x) {
    const unsigned long long l = list ? (unsigned long long)list[it] : it;
    const Leaf lf = leaves[l];
    const uint64_t n = lf.end - lf.begin;
    if (n == 0) {
      if (threadIdx.x == 0) d_out[l] = 0;
      continue;
    }
    if (!list && n > small_max) continue;
    const uint64_t* src = lf.buf ? bufB : bufA;
    uint64_t* dst = lf.buf ? bufA : bufB;
    // First try a table sized for half the records being distinct; if it
    // fills up, count the leaf again with a table large enough for all.
    const uint32_t Cfull = leaf_slots<TB, CMAX>(n, cmax_rt);
    uint32_t Cn = FULL_FIRST ? Cfull : leaf_slots<TB, CMAX>(n / 2, cmax_rt);
    // pre-aggregated records: (count - 1) in bits [cshift, 64), the shard above
    const uint32_t cshift = MERGED ? lf.cshift : 0u;
    const uint64_t low = cshift ? (1ull << cshift) - 1 : ~0ull;
    const uint64_t top = cshift ? (uint64_t)lf.shard << cshift : 0ull;
    unsigned long long my_windows = 0;  // this thread's share of the leaf's windows
    for (;;) {
    const uint32_t cmask = Cn - 1;
    const int slot_bits = 31 - __builtin_clz(Cn);
    for (uint32_t i = threadIdx.x; i < Cn; i += TB) {
      tk[i] = EMPTY;
      tc[i] = 0;
    }
    if (threadIdx.x == 0) {
      s_nd = 0;
      s_cov = 0;
      s_windows = 0;
      __hip_atomic_store(&s_ovf, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    __syncthreads();
    const uint32_t limit = Cn - (Cn >> 3);
    const bool track = n >= limit;  // fewer records than the limit cannot overflow
    my_windows = 0;
    // records are loaded R per thread before inserting, so that the loads of a
    // batch are in flight together instead of one round trip per insert. The
    // probe loop has a single exit flag (always-CAS: a CAS on a slot holding
    // another key just returns that key), which keeps divergent control flow,
    // and its scalar bookkeeping, small.
    for (uint64_t base = lf.begin; base < lf.end; base += (uint64_t)TB * R) {
      if (ovf_get(&s_ovf)) break;
      unsigned long long kb[R];
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const uint64_t r = base + (uint64_t)j * TB + threadIdx.x;
        kb[j] = r < lf.end ? src[r] : EMPTY;
      }
      // one probe loop over the thread's R records: a lane moves on to its
      // next record as soon as the current one is placed, so a wave runs
      // about as many iterations as its slowest lane's probes in total, not
      // the sum over the R records of the slowest lane's probes (records past
      // the leaf's end, EMPTY, come last)
      unsigned long long key = EMPTY;
      uint32_t cnt = 1, pos = 0, probes = 0;
      int j = 0;
      auto take = [&](unsigned long long x) {
        key = x;
        cnt = 1;
        if constexpr (MERGED) {
          if (cshift) {  // uniform per leaf
            cnt = (uint32_t)(x >> cshift) + 1u;
            key = top | (x & low);
            my_windows += cnt;
          }
        }
        pos = slot_hash(key, slot_bits);
        probes = 0;
      };
      bool todo = kb[0] != EMPTY;
      if (todo) take(kb[0]);
      while (todo) {
        const unsigned long long prev = atomicCAS(&tk[pos], EMPTY, key);
        const bool hit = (prev == EMPTY) | (prev == key);
        if (hit) {
          atomicAdd(&tc[pos], cnt);
          if (track && prev == EMPTY && atomicAdd(&s_nd, 1u) + 1 >= limit) ovf_set(&s_ovf);
          ++j;
          unsigned long long nx = EMPTY;
#pragma unroll
          for (int q = 1; q < R; ++q)
            if (j == q) nx = kb[q];
          todo = nx != EMPTY;
          if (todo) take(nx);
        } else {
          pos = (pos + 1) & cmask;
          todo = ++probes < Cn;
          if (!todo) ovf_set(&s_ovf);  // table full: the leaf overflows
        }
      }
    }
    __syncthreads();
    if (ovf_get(&s_ovf) && Cn < Cfull) {
      Cn = Cfull;
      __syncthreads();
      continue;  // retry this leaf with the full table
    }
    break;
    }
    if (ovf_get(&s_ovf)) {
      if (threadIdx.x == 0) {
        d_out[l] = kLeafOverflow;
        atomicOr(&st->overflow, 1u);
        if (ovf_list) ovf_list[atomicAdd(&st->n_ovf, 1ull)] = (uint32_t)l;
      }
      __syncthreads();
      continue;
    }
    // windows of the leaf: its records, or the sum of pre-aggregated counts
    unsigned long long windows = n;
    if (MERGED && cshift) {
      if (my_windows) atomicAdd(&s_windows, my_windows);
      __syncthreads();
      windows = s_windows;
    }
    if (windows > 0xFFFFFFFFull) {
      // a leaf of 2^32 windows or more may hold a count that wrapped past 32
      // bits; the counts then sum to less than the windows
      if (threadIdx.x == 0) s_sum = 0;
      __syncthreads();
      unsigned long long part = 0;
      for (uint32_t i = threadIdx.x; i < Cn; i += TB) part += tc[i];
      atomicAdd(&s_sum, part);
      __syncthreads();
      if (threadIdx.x == 0 && s_sum != windows) s_cov = 1;
    }
    const uint32_t d = leaf_sort_write<unsigned long long, uint32_t, TB, CMAX / TB, kLeafGroupShift>(
        tk, tc, aux, wsum, &s_max, Cn, keybits, (int)lf.bits, (unsigned long long*)dst, tmp_cnt,
        lf.begin, occ32);
    if (threadIdx.x == 0) {
      d_out[l] = d;
      if (s_cov) atomicOr(&st->count_overflow, 1u);
      my_records += n;
      my_distinct += d;
    }
    __syncthreads();
  }
  // one update of the shared totals per workgroup (not per leaf: same-address
  // atomics from every workgroup would serialise)
  if (list && threadIdx.x == 0 && my_records) {
    atomicAdd(&acc[0], my_records);
    atomicAdd(&acc[1], my_distinct);
  }
}

// 128-bit keys: there is no 128-bit CAS.
// HI = true (k <= 63): the high word of a key is then never all ones, so a
//   slot is claimed by a CAS of its high word (all ones = empty); the claimer
//   writes the low word and publishes it with the count (release). A lane
//   that finds its high word in a slot whose count is still 0 waits for that
//   publication (made in the claimer's same pass), then compares the low
//   word. Counts are 32-bit.
// HI = false (k = 64, where one key has an all-ones high word): a slot is
//   claimed through its 64-bit count word: 0 = empty, LOCK = being written;
//   the claimer writes the key and then publishes the count; others seeing
//   LOCK retry the same slot.
// FULL_FIRST only names the launches that count refined parts apart (two-word
// and wider keys always start with the full table).
template <typename K, int TB, int CMAX, int R, bool HI, bool FULL_FIRST>
__global__ void __launch_bounds__(TB) k_leaf_countw(int keybits, K* bufA, K* bufB,
                                                      uint32_t* __restrict__ tmp_cnt,
                                                      const Leaf* __restrict__ leaves,
                                                      DevState* __restrict__ st,
                                                      uint32_t* __restrict__ d_out,
                                                      int slots_log2,
                                                      const uint32_t* __restrict__ list,
                                                      uint64_t small_max) {
  static_assert(!HI || std::is_same<K, u128>::value, "high-word claims need 128-bit keys");
  typedef typename std::conditional<HI, uint32_t, unsigned long long>::type C;
  __shared__ K tk[CMAX];
  __shared__ C tc[CMAX];
  __shared__ uint32_t aux[CMAX];
  __shared__ uint32_t wsum[TB / 64];
  __shared__ uint32_t s_nd, s_max, s_cov;
  __shared__ unsigned long long s_sum;
  __shared__ uint32_t s_ovf;  // accessed only through ovf_get / ovf_set
  const unsigned long long LOCK = 1ull << 63;
  const uint32_t cmax_rt = 1u << slots_log2;
  // list != nullptr: the leaves listed there (large ones); else every leaf of
  // at most small_max records.
  const unsigned long long count = list ? st->n_large : st->n_leaves;
  unsigned long long my_records = 0, my_distinct = 0;  // thread 0: this workgroup's totals
  for (unsigned long long it = blockIdx.x; it < count; it += gridDim.x) {
    const unsigned long long l = list ? (unsigned long long)list[it] : it;
    const Leaf lf = leaves[l];
    const uint64_t n = lf.end - lf.begin;
    if (n == 0) {
      if (threadIdx.x == 0) d_out[l] = 0;
      continue;
    }
    if (!list && n > small_max) continue;
    const K* src = lf.buf ? bufB : bufA;
    K* dst = lf.buf ? bufA : bufB;
    const uint32_t Cfull = leaf_slots<TB, CMAX>(n, cmax_rt);
    // keys of more than 64 bases are mostly distinct: their first table is the
    // full one (a half table would fill to its limit, with long probe runs,
    // before the retry)
    uint32_t Cn = (sizeof(K) >= 16 || FULL_FIRST) ? Cfull : leaf_slots<TB, CMAX>(n / 2, cmax_rt);
    for (;;) {
    const uint32_t cmask = Cn - 1;
    for (uint32_t i = threadIdx.x; i < Cn; i += TB) {
      tc[i] = 0;
      if constexpr (HI) reinterpret_cast<unsigned long long*>(&tk[i])[1] = ~0ull;
    }
    if (threadIdx.x == 0) {
      s_nd = 0;
      __hip_atomic_store(&s_ovf, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      s_cov = 0;
    }
    __syncthreads();
    const uint32_t limit = Cn - (Cn >> 3);
    const bool track = n >= limit;  // fewer records than the limit cannot overflow
    for (uint64_t base = lf.begin; base < lf.end; base += (uint64_t)TB * R) {
      if (ovf_get(&s_ovf)) break;
      K kb[R];
      bool kv[R];
#pragma unroll
      for (int j = 0; j < R; ++j) {
        const uint64_t r = base + (uint64_t)j * TB + threadIdx.x;
        kv[j] = r < lf.end;
        kb[j] = kv[j] ? src[r] : (K)0;
      }
#pragma unroll
      for (int j = 0; j < R; ++j) {
      if (!kv[j]) continue;
      const K key = kb[j];
      uint32_t pos = (uint32_t)Key<K>::hash(key) & cmask;
      uint32_t probe = 0, spins = 0;
      bool done = false;
      if constexpr (HI) {
        const unsigned long long khi = (unsigned long long)(key >> 64);
        const unsigned long long klo = (unsigned long long)key;
        bool todo = true;
        while (todo) {
          unsigned long long* w = reinterpret_cast<unsigned long long*>(&tk[pos]);
          const unsigned long long prev = atomicCAS(&w[1], ~0ull, khi);
          bool hit = false, wait = false;
          if (prev == ~0ull) {
            w[0] = klo;
            __hip_atomic_store(&tc[pos], (C)1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (track && atomicAdd(&s_nd, 1u) + 1 >= limit) ovf_set(&s_ovf);
            hit = true;
          } else if (prev == khi) {
            const C c = __hip_atomic_load(&tc[pos], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (c == 0) {
              // the bound only guards against a hang; giving up marks the
              // leaf overflowed, so it is counted again by refinement
              wait = ++spins <= (1u << 22);
              if (!wait) probe = Cn;
            } else if (w[0] == klo) {
              __hip_atomic_fetch_add(&tc[pos], (C)1, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_WORKGROUP);
              hit = true;
            }
          }
          done |= hit;
          if (!hit && !wait && probe < Cn) {
            pos = (pos + 1) & cmask;
            ++probe;
          }
          todo = !hit && probe < Cn;
        }
      } else {
      while (probe < Cn) {
        C c = __hip_atomic_load(&tc[pos], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (c == 0) {
          C expect = 0;
          if (__hip_atomic_compare_exchange_strong(&tc[pos], &expect, (C)LOCK, __ATOMIC_ACQ_REL,
                                                   __ATOMIC_ACQUIRE,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP)) {
            tk[pos] = key;
            __hip_atomic_store(&tc[pos], (C)1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (track && atomicAdd(&s_nd, 1u) + 1 >= limit) ovf_set(&s_ovf);
            done = true;
            break;
          }
          c = expect;
        }
        if (c == (C)LOCK) {
          if (++spins > (1u << 22)) break;  // cannot happen; guards against a hang
          continue;
        }
        if (tk[pos] == key) {
          __hip_atomic_fetch_add(&tc[pos], (C)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          done = true;
          break;
        }
        pos = (pos + 1) & cmask;
        ++probe;
      }
      }
      if (!done) ovf_set(&s_ovf);
      }
    }
    __syncthreads();
    if (ovf_get(&s_ovf) && Cn < Cfull) {
      Cn = Cfull;
      __syncthreads();
      continue;  // retry this leaf with the full table
    }
    break;
    }
    if (ovf_get(&s_ovf)) {
      if (threadIdx.x == 0) {
        d_out[l] = kLeafOverflow;
        atomicOr(&st->overflow, 1u);
      }
      __syncthreads();
      continue;
    }
    if constexpr (HI) {
      if (n > 0xFFFFFFFFull) {
        // 32-bit counts may have wrapped: they then sum to less than the records
        if (threadIdx.x == 0) s_sum = 0;
        __syncthreads();
        unsigned long long part = 0;
        for (uint32_t i = threadIdx.x; i < Cn; i += TB) part += tc[i];
        atomicAdd(&s_sum, part);
        __syncthreads();
        if (threadIdx.x == 0 && s_sum != n) s_cov = 1;
      }
    } else {
      for (uint32_t i = threadIdx.x; i < Cn; i += TB)
        if ((unsigned long long)tc[i] > 0xFFFFFFFFull) s_cov = 1;
    }
    const uint32_t d = leaf_sort_write<K, C, TB, CMAX / TB, 1>(
        tk, tc, aux, wsum, &s_max, Cn, keybits, (int)lf.bits, dst, tmp_cnt, lf.begin,
        HI ? (bool (*)(C))occ32 : (bool (*)(C))occ64);
    if (threadIdx.x == 0) {
      d_out[l] = d;
      if (s_cov) atomicOr(&st->count_overflow, 1u);
      my_records += n;
      my_distinct += d;
    }
    __syncthreads();
  }
  if (list && threadIdx.x == 0 && my_records) {
    atomicAdd(&st->large_records, my_records);
    atomicAdd(&st->large_distinct, my_distinct);
  }
}

// ---------------------------------------------------------------- sort-based leaf count

// The paper's own way to count an owner's k-mers (counting by sorting, as in
// Algorithm 1 and by every owner in Algorithm 3), applied to a leaf: its
// records are sorted in LDS and each run of equal keys becomes one pair. A
// leaf of more records than fit is marked overflowed and cut further by key
// (refinement); a leaf whose key range is a single key is counted without
// sorting.
template <typename K, int TB>
__device__ __forceinline__ void bitonic_keys(K* keys, uint32_t n) {
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
        }
      }
      __syncthreads();
    }
  }
}

template <typename K, int TB, int SMAX>
__global__ void __launch_bounds__(TB) k_leaf_sort(int keybits, K* bufA, K* bufB,
                                                  uint32_t* __restrict__ tmp_cnt,
                                                  const Leaf* __restrict__ leaves,
                                                  DevState* __restrict__ st,
                                                  uint32_t* __restrict__ d_out,
                                                  const uint32_t* __restrict__ list) {
  __shared__ K sk[SMAX];
  __shared__ uint32_t sp[SMAX + 1];  // positions of the run starts, then n
  __shared__ uint32_t wsum[TB / 64];
  const unsigned long long count = st->n_large;
  unsigned long long my_records = 0, my_distinct = 0;
  for (unsigned long long it = blockIdx.x; it < count; it += gridDim.x) {
    const uint32_t l = list[it];
    const Leaf lf = leaves[l];
    const uint64_t n = lf.end - lf.begin;
    const K* src = lf.buf ? bufB : bufA;
    K* dst = lf.buf ? bufA : bufB;
    if ((int)lf.bits >= keybits) {  // the leaf's range is one key
      if (threadIdx.x == 0) {
        dst[lf.begin] = src[lf.begin];
        tmp_cnt[lf.begin] = (uint32_t)n;
        if (n > 0xFFFFFFFFull) atomicOr(&st->count_overflow, 1u);
        d_out[l] = 1;
        my_records += n;
        my_distinct += 1;
      }
      continue;
    }
    if (n > SMAX) {
      if (threadIdx.x == 0) {
        d_out[l] = kLeafOverflow;
        atomicOr(&st->overflow, 1u);
      }
      continue;
    }
    const uint32_t m = (uint32_t)n;
    const uint32_t n2 = next_pow2(m);
    for (uint32_t i = threadIdx.x; i < n2; i += TB) sk[i] = i < m ? src[lf.begin + i] : ~(K)0;
    __syncthreads();
    bitonic_keys<K, TB>(sk, n2);
    // run starts: thread t looks at positions [t*per, t*per + per)
    const uint32_t per = (m + TB - 1) / TB;
    const uint32_t b = threadIdx.x * per, e = min(m, b + per);
    uint32_t c = 0;
    for (uint32_t i = b; i < e; ++i) c += (i == 0 || sk[i] != sk[i - 1]) ? 1u : 0u;
    uint32_t d = 0;
    uint32_t at = block_exscan<TB, uint32_t>(c, wsum, &d);
    for (uint32_t i = b; i < e; ++i)
      if (i == 0 || sk[i] != sk[i - 1]) sp[at++] = i;
    if (threadIdx.x == 0) sp[d] = m;
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < d; q += TB) {
      const uint32_t i = sp[q];
      dst[lf.begin + q] = sk[i];
      tmp_cnt[lf.begin + q] = sp[q + 1] - i;
    }
    if (threadIdx.x == 0) {
      d_out[l] = d;
      my_records += n;
      my_distinct += d;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && my_records) {
    atomicAdd(&st->large_records, my_records);
    atomicAdd(&st->large_distinct, my_distinct);
  }
}

// Lanes of this wave whose digit d (nb bits) equals this lane's, among the
// lanes with v set (ballots over the digit's bits).
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool v, int nb) {
  uint64_t m = __ballot(v);
  for (int bit = 0; bit < nb; ++bit) {
    const bool on = (d >> bit) & 1u;
    const uint64_t set = __ballot(v && on);
    m &= on ? set : ~set;
  }
  return m;
}

// Stable LSD radix sort in LDS of n one-word keys (and their counts) by bits
// [0, nbits), 8-bit digits. Per pass, wave w walks its contiguous chunk of
// the elements 64 at a time: lanes holding the same digit find each other by
// ballots, so each digit's count per wave and each element's rank among the
// wave's equal digits come without atomics; a block scan of the counts in
// digit-major order gives every (digit, wave) its first position, and a
// second walk places the elements there in order (stable). Ping-pong between
// (ka, ca) and (kb, cb); returns true if the result ended in (kb, cb).
template <int TB>
__device__ bool lds_radix_sort64(uint64_t* ka, uint32_t* ca, uint64_t* kb, uint32_t* cb,
                                 uint32_t n, int nbits, uint32_t* whist, uint32_t* wsum) {
  constexpr int NW = TB / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t chunk = (n + NW - 1) / NW;
  const uint32_t c0 = min(n, (uint32_t)w * chunk), c1 = min(n, c0 + chunk);
  const uint64_t below = (1ull << lane) - 1;
  bool flipped = false;
  for (int shift = 0; shift < nbits; shift += 8) {
    const int nb = min(8, nbits - shift);
    for (int i = threadIdx.x; i < 256 * NW; i += TB) whist[i] = 0;
    __syncthreads();
    for (uint32_t r0 = c0; r0 < c1; r0 += 64) {
      const uint32_t i = r0 + lane;
      const bool v = i < c1;
      const uint32_t d = v ? (uint32_t)(ka[i] >> shift) & ((1u << nb) - 1u) : 0u;
      const uint64_t peers = digit_peers(d, v, nb);
      if (v && lane == __ffsll((long long)peers) - 1) whist[d * NW + w] += __popcll(peers);
    }
    __syncthreads();
    (void)block_exscan_inplace<TB>(whist, 256 * NW, wsum);
    for (uint32_t r0 = c0; r0 < c1; r0 += 64) {
      const uint32_t i = r0 + lane;
      const bool v = i < c1;
      const uint64_t key = v ? ka[i] : 0ull;
      const uint32_t d = (uint32_t)(key >> shift) & ((1u << nb) - 1u);
      const uint64_t peers = digit_peers(d, v, nb);
      if (v) {
        const uint32_t pos = whist[d * NW + w] + (uint32_t)__popcll(peers & below);
        kb[pos] = key;
        cb[pos] = ca[i];
      }
      // every lane has read its digit's base before the leader advances it
      if (v && lane == __ffsll((long long)peers) - 1) whist[d * NW + w] += __popcll(peers);
    }
    __syncthreads();
    uint64_t* tk = ka;
    ka = kb;
    kb = tk;
    uint32_t* tc = ca;
    ca = cb;
    cb = tc;
    flipped = !flipped;
  }
  return flipped;
}

// The paper's counting step on one-word keys, with a radix sort: a leaf's
// records (up to SMAX; pre-aggregated ones carry their counts) are loaded into
// LDS, radix-sorted by the key bits below the leaf's common prefix, and each
// run of equal keys becomes one pair whose count is the sum of its records'
// counts (the Sort and Accumulate of Algorithm 1, run by each owner in
// Algorithm 3, on records shaped like the HEAVY (k-mer, count) and NORMAL
// (k-mer) messages of Section IV-D). A larger leaf is marked overflowed and cut
// further by key; a leaf whose range is one key is summed without sorting.
template <int TB, int SMAX>
__global__ void __launch_bounds__(TB) k_leaf_radix64(int keybits, uint64_t* bufA, uint64_t* bufB,
                                                     uint32_t* __restrict__ tmp_cnt,
                                                     const Leaf* __restrict__ leaves,
                                                     DevState* __restrict__ st,
                                                     uint32_t* __restrict__ d_out,
                                                     const uint32_t* __restrict__ list) {
  __shared__ uint64_t ka[SMAX], kb[SMAX];
  __shared__ uint32_t ca[SMAX], cb[SMAX];
  __shared__ uint32_t sp[SMAX + 1];  // run starts; then their count prefix sums
  __shared__ uint32_t whist[256 * (TB / 64)];
  __shared__ uint32_t wsum[TB / 64];
  __shared__ unsigned long long s_sum;
  const unsigned long long count = st->n_large;
  unsigned long long my_records = 0, my_distinct = 0;
  for (unsigned long long it = blockIdx.x; it < count; it += gridDim.x) {
    const uint32_t l = list[it];
    const Leaf lf = leaves[l];
    const uint64_t n = lf.end - lf.begin;
    const uint64_t* src = lf.buf ? bufB : bufA;
    uint64_t* dst = lf.buf ? bufA : bufB;
    const uint32_t cshift = lf.cshift;
    const uint64_t low = cshift ? (1ull << cshift) - 1 : ~0ull;
    const uint64_t top = cshift ? (uint64_t)lf.shard << cshift : 0ull;
    if ((int)lf.bits >= keybits) {  // the leaf's range is one key: sum its records' counts
      if (threadIdx.x == 0) s_sum = 0;
      __syncthreads();
      unsigned long long part = 0;
      for (uint64_t r = lf.begin + threadIdx.x; r < lf.end; r += TB)
        part += cshift ? (src[r] >> cshift) + 1 : 1;
      if (part) atomicAdd(&s_sum, part);
      __syncthreads();
      if (threadIdx.x == 0) {
        const uint64_t w0 = src[lf.begin];
        dst[lf.begin] = cshift ? top | (w0 & low) : w0;
        tmp_cnt[lf.begin] = (uint32_t)s_sum;
        if (s_sum > 0xFFFFFFFFull) atomicOr(&st->count_overflow, 1u);
        d_out[l] = 1;
        my_records += n;
        my_distinct += 1;
      }
      __syncthreads();
      continue;
    }
    if (n > SMAX) {
      if (threadIdx.x == 0) {
        d_out[l] = kLeafOverflow;
        atomicOr(&st->overflow, 1u);
      }
      continue;
    }
    const uint32_t m = (uint32_t)n;
    for (uint32_t i = threadIdx.x; i < m; i += TB) {
      const uint64_t x = src[lf.begin + i];
      ka[i] = cshift ? top | (x & low) : x;
      ca[i] = cshift ? (uint32_t)(x >> cshift) + 1u : 1u;
    }
    __syncthreads();
    const bool in_b = lds_radix_sort64<TB>(ka, ca, kb, cb, m, keybits - (int)lf.bits, whist, wsum);
    const uint64_t* sk = in_b ? kb : ka;
    uint32_t* sc = in_b ? cb : ca;
    // run starts: thread t looks at positions [t*per, t*per + per)
    const uint32_t per = (m + TB - 1) / TB;
    const uint32_t b = threadIdx.x * per, e = min(m, b + per);
    uint32_t c = 0;
    for (uint32_t i = b; i < e; ++i) c += (i == 0 || sk[i] != sk[i - 1]) ? 1u : 0u;
    uint32_t d = 0;
    uint32_t at = block_exscan<TB, uint32_t>(c, wsum, &d);
    for (uint32_t i = b; i < e; ++i)
      if (i == 0 || sk[i] != sk[i - 1]) sp[at++] = i;
    if (threadIdx.x == 0) sp[d] = m;
    __syncthreads();
    // counts of the runs: exclusive prefix sums of the sorted records' counts
    const uint32_t all = block_exscan_inplace<TB>(sc, m, wsum);
    for (uint32_t q = threadIdx.x; q < d; q += TB) {
      const uint32_t i = sp[q], j = sp[q + 1];
      dst[lf.begin + q] = sk[i];
      tmp_cnt[lf.begin + q] = (j < m ? sc[j] : all) - sc[i];
    }
    if (threadIdx.x == 0) {
      d_out[l] = d;
      my_records += n;
      my_distinct += d;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && my_records) {
    atomicAdd(&st->large_records, my_records);
    atomicAdd(&st->large_distinct, my_distinct);
  }
}

// Empty leaves of the sort-based count (the others are all in the list).
__global__ void k_empty_leaves(const Leaf* __restrict__ leaves, const DevState* __restrict__ st,
                               uint32_t* __restrict__ d_out) {
  const unsigned long long n = st->n_leaves;
  const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += stride)
    if (leaves[i].end == leaves[i].begin) d_out[i] = 0;
}

// ---------------------------------------------------------------- concat + check

template <typename K>
__global__ void __launch_bounds__(256) k_concat(const K* __restrict__ bufA,
                                                const K* __restrict__ bufB,
                                                const uint32_t* __restrict__ tmp_cnt,
                                                const Leaf* __restrict__ leaves,
                                                const uint32_t* __restrict__ d,
                                                const unsigned long long* __restrict__ out_off,
                                                const DevState* __restrict__ st, uint64_t cap,
                                                uint64_t* __restrict__ out_keys,
                                                uint32_t* __restrict__ out_counts) {
  // a leaf overflowed: the host refines it and concatenates afterwards, so
  // this launch (enqueued before the host could know) has nothing to do
  if (st->overflow) return;
  // one wave per leaf, many leaves in flight per CU
  const unsigned long long n_leaves = st->n_leaves;
  const unsigned lane = threadIdx.x & 63;
  const unsigned long long nw = (unsigned long long)gridDim.x * 4;
  for (unsigned long long l = (unsigned long long)blockIdx.x * 4 + (threadIdx.x >> 6); l < n_leaves;
       l += nw) {
    const uint32_t n = d[l];
    if (n == 0 || n == kLeafOverflow) continue;
    const Leaf lf = leaves[l];
    const K* src = lf.buf ? bufA : bufB;  // sorted pairs sit in the other buffer
    const unsigned long long base = out_off[l];
    // U pairs per lane per step, all loaded before any is stored (more bytes
    // in flight per wave)
    constexpr uint32_t U = Key<K>::kWords == 4 ? 1 : 4;
    const uint64_t lim = base >= cap ? 0 : min((uint64_t)n, cap - base);
    for (uint32_t i0 = 0; i0 < lim; i0 += 64 * U) {
      K key[U];
      uint32_t cnt[U];
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) {
        const uint32_t i = i0 + u * 64 + lane;
        if (i < lim) {
          key[u] = src[lf.begin + i];
          cnt[u] = tmp_cnt[lf.begin + i];
        }
      }
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) {
        const uint32_t i = i0 + u * 64 + lane;
        if (i >= lim) break;
        const uint64_t o = base + i;
        if constexpr (Key<K>::kWords == 4) {
          out_keys[4 * o] = (uint64_t)key[u].lo;
          out_keys[4 * o + 1] = (uint64_t)(key[u].lo >> 64);
          out_keys[4 * o + 2] = (uint64_t)key[u].hi;
          out_keys[4 * o + 3] = (uint64_t)(key[u].hi >> 64);
        } else if constexpr (Key<K>::kWords == 2) {
          out_keys[2 * o] = (uint64_t)key[u];
          out_keys[2 * o + 1] = (uint64_t)((u128)key[u] >> 64);
        } else {
          out_keys[o] = (uint64_t)key[u];
        }
        out_counts[o] = cnt[u];
      }
    }
  }
}

// Batch form of concat: writes the k-mer (low 2k bits) and the set id within
// the class (the bits above) of every pair, in key order.
template <typename K>
__global__ void __launch_bounds__(256) k_concat_batch(
    const K* __restrict__ bufA, const K* __restrict__ bufB, const uint32_t* __restrict__ tmp_cnt,
    const Leaf* __restrict__ leaves, const uint32_t* __restrict__ d,
    const unsigned long long* __restrict__ out_off, const DevState* __restrict__ st, uint64_t cap,
    int k, uint64_t* __restrict__ out_keys, uint32_t* __restrict__ out_counts,
    uint32_t* __restrict__ out_set) {
  if (st->overflow) return;  // the class is recounted set by set
  const unsigned long long n_leaves = st->n_leaves;
  const unsigned lane = threadIdx.x & 63;
  const unsigned long long nw = (unsigned long long)gridDim.x * 4;
  const bool has_set_bits = 2 * k < (int)(8 * sizeof(K));
  const K kmask = has_set_bits ? ((K)1 << (2 * k)) - 1 : ~(K)0;
  for (unsigned long long l = (unsigned long long)blockIdx.x * 4 + (threadIdx.x >> 6); l < n_leaves;
       l += nw) {
    const uint32_t n = d[l];
    if (n == 0 || n == kLeafOverflow) continue;
    const Leaf lf = leaves[l];
    const K* src = lf.buf ? bufA : bufB;
    const unsigned long long base = out_off[l];
    constexpr uint32_t U = 4;  // as in k_concat
    const uint64_t lim = base >= cap ? 0 : min((uint64_t)n, cap - base);
    for (uint32_t i0 = 0; i0 < lim; i0 += 64 * U) {
      K key[U];
      uint32_t cnt[U];
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) {
        const uint32_t i = i0 + u * 64 + lane;
        if (i < lim) {
          key[u] = src[lf.begin + i];
          cnt[u] = tmp_cnt[lf.begin + i];
        }
      }
#pragma unroll
      for (uint32_t u = 0; u < U; ++u) {
        const uint32_t i = i0 + u * 64 + lane;
        if (i >= lim) break;
        const uint64_t o = base + i;
        out_keys[o] = (uint64_t)(key[u] & kmask);
        out_set[o] = has_set_bits ? (uint32_t)(key[u] >> (2 * k)) : 0u;
        out_counts[o] = cnt[u];
      }
    }
  }
}

// start[s] = index of the first pair of set s (within a class output sorted
// by set); sets without pairs get the index of the next pair. start has
// n_local + 1 entries; start[n_local] = number of pairs. A class whose leaf
// overflowed has no output (its concat returned at once, so the set ids hold
// whatever the buffer held before): all its bounds are 0, and the host counts
// the wave's sets one by one.
__global__ void k_set_bounds(const uint32_t* __restrict__ set, const DevState* __restrict__ st,
                             uint32_t n_local, unsigned long long* __restrict__ start) {
  const unsigned long long n = st->D;
  if (n == 0 || st->overflow) {
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t <= n_local; t += gridDim.x * blockDim.x)
      start[t] = 0;
    return;
  }
  for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (unsigned long long)gridDim.x * blockDim.x) {
    const uint32_t s = set[i];
    const uint32_t from = i == 0 ? 0u : set[i - 1] + 1;
    for (uint32_t t = from; t <= s; ++t) start[t] = i;
    if (i == n - 1)
      for (uint32_t t = s + 1; t <= n_local; ++t) start[t] = n;
  }
}

// Global output offsets of the sets (one block): set g is set_local[g] of
// class set_class[g], whose bounds start at start_base[class] in starts[].
__global__ void __launch_bounds__(kPlanTB) k_batch_offsets(
    const uint32_t* __restrict__ set_class, const uint32_t* __restrict__ set_local,
    const unsigned long long* __restrict__ starts, const unsigned long long* __restrict__ start_base,
    uint32_t n_sets, unsigned long long* __restrict__ set_off) {
  __shared__ unsigned long long wsum[kPlanTB / 64];
  const uint32_t per = (n_sets + kPlanTB - 1) / kPlanTB;
  const uint32_t b = threadIdx.x * per, e = min(n_sets, b + per);
  unsigned long long s = 0;
  for (uint32_t g = b; g < e; ++g) {
    const unsigned long long* st = starts + start_base[set_class[g]];
    s += st[set_local[g] + 1] - st[set_local[g]];
  }
  unsigned long long total;
  unsigned long long run = block_exscan<kPlanTB, unsigned long long>(s, wsum, &total);
  for (uint32_t g = b; g < e; ++g) {
    set_off[g] = run;
    const unsigned long long* st = starts + start_base[set_class[g]];
    run += st[set_local[g] + 1] - st[set_local[g]];
  }
  if (threadIdx.x == 0) set_off[n_sets] = total;
}

// Copy each set's pairs from its class output to its place in the batch
// output. Waves take chunks of consecutive output positions (coalesced
// reads and writes); the set of a chunk's first position is found by binary
// search in set_off, later positions move to the next set when they pass its
// start.
__global__ void __launch_bounds__(256) k_batch_gather(
    const uint32_t* __restrict__ set_class, const uint32_t* __restrict__ set_local,
    const unsigned long long* __restrict__ starts, const unsigned long long* __restrict__ start_base,
    const unsigned long long* __restrict__ class_base, const uint64_t* __restrict__ cls_keys,
    const uint32_t* __restrict__ cls_counts, const unsigned long long* __restrict__ set_off,
    uint32_t n_sets, uint64_t cap, uint64_t* __restrict__ out_keys,
    uint32_t* __restrict__ out_counts) {
  constexpr int kChunk = 64 * 16;
  const unsigned lane = threadIdx.x & 63;
  const unsigned long long D = min((unsigned long long)cap, set_off[n_sets]);
  const unsigned long long nchunks = (D + kChunk - 1) / kChunk;
  for (unsigned long long ch = (unsigned long long)blockIdx.x * 4 + (threadIdx.x >> 6);
       ch < nchunks; ch += (unsigned long long)gridDim.x * 4) {
    const unsigned long long o0 = ch * kChunk;
    uint32_t lo = 0, hi = n_sets - 1;  // last set starting at or before o0
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (set_off[mid] <= o0) lo = mid; else hi = mid - 1;
    }
    uint32_t g = lo;
    unsigned long long src0 = class_base[set_class[g]] +
                              starts[start_base[set_class[g]] + set_local[g]] - set_off[g];
    for (int j = 0; j < 16; ++j) {
      const unsigned long long o = o0 + (unsigned long long)j * 64 + lane;
      if (o >= D) break;
      bool moved = false;
      while (g + 1 < n_sets && o >= set_off[g + 1]) {
        ++g;
        moved = true;
      }
      if (moved)
        src0 = class_base[set_class[g]] + starts[start_base[set_class[g]] + set_local[g]] -
               set_off[g];
      out_keys[o] = cls_keys[src0 + o];
      out_counts[o] = cls_counts[src0 + o];
    }
  }
}

template <typename K>
__device__ __forceinline__ K load_out_key(const uint64_t* keys, uint64_t i) {
  if constexpr (Key<K>::kWords == 4)
    return K(((u128)keys[4 * i + 1] << 64) | keys[4 * i], ((u128)keys[4 * i + 3] << 64) | keys[4 * i + 2]);
  else if constexpr (Key<K>::kWords == 2)
    return (K)(((u128)keys[2 * i + 1] << 64) | keys[2 * i]);
  else
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
constexpr unsigned kHistGrid = 2048;  // a multiple of kXcds
constexpr int kScatterTB64 = 1024;
constexpr int kScatterTB128 = 512;
constexpr int kSplitTB64 = 1024;
constexpr int kSplitTB128 = 512;
constexpr int kScatterTB256 = 256;  // 256-bit keys: LDS staging of 64 KiB per tile
constexpr int kSplitTB256 = 256;
constexpr int kSplitR = 8;
constexpr int kLeafTB = 512;
constexpr int kLeafCmax64 = 4096;
// second-chance count of overflowed one-word leaves: 8,192 slots (128 KiB of
// LDS with the epilogue's counters: one 1,024-thread workgroup per CU)
constexpr int kRescueTB = 1024;
constexpr int kRescueCmax64 = 8192;
constexpr int kRescueSlotsLog2 = 13;
constexpr unsigned kRescueGrid = 256;
constexpr int kLeafCmax128 = 2048;
constexpr int kLeafCmax256 = 2048;  // 44 bytes a slot: key, 64-bit count, sort aux
constexpr unsigned kPersistentGrid = 1024;  // blocks of the persistent kernels
constexpr int kSmallCmax64 = 1024;  // one-wave leaf kernel: slots of its private table
constexpr int kSmallCmax128 = 512;
constexpr unsigned kSmallGrid = 256 * 20;
constexpr int kSortMax64 = 5120;   // records per leaf of the sort-based count (radix: 148 KiB LDS)
constexpr int kSortMax128 = 4096;
constexpr int kSortMax256 = 2048;

inline unsigned grid_for(uint64_t n, unsigned tb, unsigned cap) {
  uint64_t g = (n + tb - 1) / tb;
  if (g > cap) g = cap;
  return g ? (unsigned)g : 1u;
}

inline unsigned persistent(uint64_t max_n, unsigned cap) {
  return (unsigned)(max_n == 0 ? 1 : (max_n < cap ? max_n : cap));
}

}  // namespace

int max_leaf_slots_log2(int words) { return words > 1 ? 11 : 12; }
int max_shard_bits() { return kMaxShardBits; }
int split_tile(int words, int records_per_thread) {
  const int r = words == 1 && records_per_thread == 16 ? 16 : kSplitR;
  return (words == 4 ? kSplitTB256 : words == 2 ? kSplitTB128 : kSplitTB64) * r;
}

hipError_t launch_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v,
                           hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_pack(const uint8_t* src, uint64_t n_bytes, const uint64_t* offsets,
                       uint64_t n_reads, uint64_t off0, uint64_t* packed, uint64_t* inv,
                       uint64_t* endm, uint64_t nchunks, hipStream_t s) {
  const int aligned = ((uintptr_t)src & 15) == 0;
  const unsigned grid = (unsigned)((nchunks + 255) / 256);
  hipLaunchKernelGGL(k_pack, dim3(grid), dim3(256), 0, s, src, n_bytes, offsets, n_reads, off0,
                     packed, inv, endm, nchunks, aligned);
  if (n_reads)
    hipLaunchKernelGGL(k_read_ends, dim3((unsigned)((n_reads + 255) / 256)), dim3(256), 0, s,
                       offsets, n_reads, off0, (unsigned long long*)endm);
  return hipGetLastError();
}

#define KC_WINDOW_LAUNCH(KERNEL, K, KC, TB, BATCH, GRID)                                    \
  hipLaunchKernelGGL((KERNEL<K, KC, kWinStarts, TB, BATCH>), dim3(GRID), dim3(TB), 0, s, packed, \
                     valid, t_begin, t_end, k, keybits, shard_bits, bs, ARG0, ARG1)
#define KC_WINDOW_LAUNCH_S(KERNEL, K, KC, S, TB, BATCH, GRID)                                  \
  hipLaunchKernelGGL((KERNEL<K, KC, S, TB, BATCH>), dim3(GRID), dim3(TB), 0, s, packed, valid,     \
                     t_begin, t_end, k, keybits, shard_bits, bs, ARG0, ARG1)

hipError_t launch_valid_mask(int words, const uint64_t* inv, const uint64_t* endm,
                             uint64_t byte_begin, uint64_t byte_end, int k, uint64_t* valid,
                             hipStream_t s) {
  // the words the window kernels read: starts [byte_begin, byte_end) rounded
  // out to whole threads, which stay inside whole words
  const uint64_t w_begin = byte_begin >> 6, w_end = (byte_end + 63) >> 6;
  if (w_end <= w_begin) return hipSuccess;
  const unsigned grid = (unsigned)((w_end - w_begin + 255) / 256);
  if (words == 4)
    hipLaunchKernelGGL(k_valid_mask<true>, dim3(grid), dim3(256), 0, s, inv, endm, w_begin, w_end,
                       k, valid);
  else
    hipLaunchKernelGGL(k_valid_mask<false>, dim3(grid), dim3(256), 0, s, inv, endm, w_begin,
                       w_end, k, valid);
  return hipGetLastError();
}

#define KC_HIST_LAUNCH(K, KC, BATCH)                                                            \
  hipLaunchKernelGGL((k_window_hist<K, KC, kWinStarts, kHistTB, BATCH>), dim3(grid),            \
                     dim3(kHistTB), 0, s, packed, valid, w_begin, w_end, tile_starts, k, keybits, \
                     shard_bits, bs, hist, wcount)

hipError_t launch_window_hist(int words, const uint64_t* packed, const uint64_t* valid,
                              uint64_t byte_begin, uint64_t byte_end, int k,
                              int keybits, int shard_bits, const BatchSets* batch,
                              unsigned long long* hist, unsigned long long* wcount,
                              int starts_per_thread, hipStream_t s) {
  // the owner scatter's tiles (see launch_window_scatter)
  const int S = words == 1 && starts_per_thread == 16 ? 16 : kWinStarts;
  const int TBs = words == 4 ? kScatterTB256 : words == 2 ? kScatterTB128 : kScatterTB64;
  const uint64_t w_begin = byte_begin / S * S;
  const uint64_t w_end = (byte_end + S - 1) / S * S;
  const uint64_t tile_starts = (uint64_t)TBs * S;
  const uint64_t n_tiles = (w_end - w_begin + tile_starts - 1) / tile_starts;
  // a multiple of kXcds workgroups (every workgroup's tiles share a class)
  const unsigned grid = (unsigned)std::min<uint64_t>((n_tiles + kXcds - 1) / kXcds * kXcds,
                                                     kHistGrid);
  if (grid == 0) return hipSuccess;
  const BatchSets bs = batch ? *batch : BatchSets{nullptr, nullptr, 0};
  const bool wide = words == 2;
  if (batch) {
    if (words == 4) return hipErrorInvalidValue;
    if (wide) KC_HIST_LAUNCH(u128, uint64_t, true);
    else KC_HIST_LAUNCH(uint64_t, uint64_t, true);
  } else {
    if (words == 4) KC_HIST_LAUNCH(u256, u256, false);
    else if (wide) KC_HIST_LAUNCH(u128, u128, false);
    else KC_HIST_LAUNCH(uint64_t, uint64_t, false);
  }
  return hipGetLastError();
}
#undef KC_HIST_LAUNCH

hipError_t launch_window_scatter(int words, const uint64_t* packed, const uint64_t* valid,
                                 uint64_t byte_begin, uint64_t byte_end,
                                 int k, int keybits, int shard_bits, const BatchSets* batch,
                                 unsigned long long* cursor, void* out, int starts_per_thread,
                                 hipStream_t s) {
  const BatchSets bs0 = batch ? *batch : BatchSets{nullptr, nullptr, 0};
  if (words == 1 && starts_per_thread == 16) {
    // byte_begin is a multiple of 32 (batch classes) or 0
    constexpr int S = 16;
    const uint64_t t_begin = byte_begin / S;
    const uint64_t t_end = (byte_end + S - 1) / S;
    const BatchSets bs = bs0;
    const unsigned grid = grid_for(t_end - t_begin, kScatterTB64, 1u << 20);
#define ARG0 cursor
#define ARG1 (uint64_t*)out
    if (batch) KC_WINDOW_LAUNCH_S(k_window_scatter64w, uint64_t, uint64_t, S, kScatterTB64, true, grid);
    else KC_WINDOW_LAUNCH_S(k_window_scatter64w, uint64_t, uint64_t, S, kScatterTB64, false, grid);
#undef ARG1
#undef ARG0
    return hipGetLastError();
  }
  const uint64_t t_begin = byte_begin / kWinStarts;
  const uint64_t t_end = (byte_end + kWinStarts - 1) / kWinStarts;
  const BatchSets bs = batch ? *batch : BatchSets{nullptr, nullptr, 0};
#define ARG0 cursor
  if (words == 4) {
    if (batch) return hipErrorInvalidValue;
    const unsigned grid = grid_for(t_end - t_begin, kScatterTB256, 1u << 20);
#define ARG1 (u256*)out
    KC_WINDOW_LAUNCH(k_window_scatter, u256, u256, kScatterTB256, false, grid);
#undef ARG1
  } else if (words == 2) {
    const unsigned grid = grid_for(t_end - t_begin, kScatterTB128, 1u << 20);
#define ARG1 (u128*)out
    if (batch) KC_WINDOW_LAUNCH(k_window_scatter, u128, uint64_t, kScatterTB128, true, grid);
    else KC_WINDOW_LAUNCH(k_window_scatter, u128, u128, kScatterTB128, false, grid);
#undef ARG1
  } else {
    const unsigned grid = grid_for(t_end - t_begin, kScatterTB64, 1u << 20);
#define ARG1 (uint64_t*)out
    if (batch) KC_WINDOW_LAUNCH(k_window_scatter, uint64_t, uint64_t, kScatterTB64, true, grid);
    else KC_WINDOW_LAUNCH(k_window_scatter64, uint64_t, uint64_t, kScatterTB64, false, grid);
#undef ARG1
  }
#undef ARG0
  return hipGetLastError();
}
#undef KC_WINDOW_LAUNCH
#undef KC_WINDOW_LAUNCH_S

hipError_t launch_plan_shards(const unsigned long long* hist, const int* order, int shard_bits,
                              int keybits, uint64_t leaf_target, uint64_t leaf_attempt,
                              int tile, unsigned long long* sbegin, unsigned long long* cursor,
                              SplitBin* bins, SplitItem* items, unsigned long long* item_off,
                              unsigned long long* subhist, uint64_t max_leaves,
                              uint64_t max_items, int ncls, DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(max_leaves * ncls, 256, 1024)), dim3(256), 0, s,
                     subhist, max_leaves * ncls, 0ull);
  hipLaunchKernelGGL(k_plan_shards, dim3(1), dim3(kPlanTB), 0, s, hist, order, shard_bits,
                     keybits, leaf_target, leaf_attempt, tile, sbegin, cursor, bins, item_off,
                     subhist, st);
  hipLaunchKernelGGL(k_plan_items, dim3(grid_for(max_items, 256, 2048)), dim3(256), 0, s, hist,
                     sbegin, item_off, shard_bits, tile, st, items);
  return hipGetLastError();
}

hipError_t launch_plan_leaves(const unsigned long long* hist, const unsigned long long* sbegin,
                              const SplitBin* bins, int shard_bits,
                              const unsigned long long* subhist, Leaf* leaves,
                              unsigned long long* cursor, int merge_cshift, int ncls,
                              uint64_t cls_stride, hipStream_t s) {
  hipLaunchKernelGGL(k_plan_leaves, dim3(1u << shard_bits), dim3(kPlanTB), 0, s, hist, sbegin,
                     bins, shard_bits, subhist, leaves, cursor, merge_cshift, ncls, cls_stride);
  return hipGetLastError();
}

hipError_t launch_leaf_ends(Leaf* leaves, const unsigned long long* cursor, const DevState* st,
                            uint64_t max_leaves, hipStream_t s) {
  hipLaunchKernelGGL(k_leaf_ends, dim3(grid_for(max_leaves, 256, 2048)), dim3(256), 0, s, leaves,
                     cursor, st);
  return hipGetLastError();
}

hipError_t launch_split_hist(int words, const void* src, const SplitItem* items,
                             const DevState* st, uint64_t max_items, const SplitBin* bins,
                             unsigned long long* subhist, int ncls, uint64_t cls_stride,
                             hipStream_t s) {
  const unsigned grid = persistent(max_items, 4096);
  if (words == 4)
    hipLaunchKernelGGL((k_split_hist<u256, 256>), dim3(grid), dim3(256), 0, s, (const u256*)src,
                       items, st, bins, subhist, ncls, cls_stride);
  else if (words == 2)
    hipLaunchKernelGGL((k_split_hist<u128, 256>), dim3(grid), dim3(256), 0, s, (const u128*)src,
                       items, st, bins, subhist, ncls, cls_stride);
  else
    hipLaunchKernelGGL((k_split_hist<uint64_t, 256>), dim3(grid), dim3(256), 0, s,
                       (const uint64_t*)src, items, st, bins, subhist, ncls, cls_stride);
  return hipGetLastError();
}

hipError_t launch_split_scatter(int words, const void* src, void* dst, const SplitItem* items,
                                const DevState* st, uint64_t max_items, const SplitBin* bins,
                                unsigned long long* cursor, int records_per_thread,
                                int merge_cshift, int ncls, uint64_t cls_stride, hipStream_t s) {
  const unsigned grid = persistent(max_items, 2048);
  if (merge_cshift) {
    // one cursor per leaf: its final value is the leaf's end
    if (words != 1 || records_per_thread != 16 || ncls != 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_split_scatter_merge<kSplitTB64, 16>), dim3(grid), dim3(kSplitTB64), 0,
                       s, (const uint64_t*)src, (uint64_t*)dst, items, st, bins, cursor,
                       merge_cshift);
    return hipGetLastError();
  }
  if (words == 1 && records_per_thread == 16) {
    // 16,384-record tiles: 128 KiB of LDS staging, one workgroup per CU
    hipLaunchKernelGGL((k_split_scatter<uint64_t, kSplitTB64, 16>), dim3(grid), dim3(kSplitTB64),
                       0, s, (const uint64_t*)src, (uint64_t*)dst, items, st, bins, cursor,
                       ncls, cls_stride);
    return hipGetLastError();
  }
  if (words == 4)
    hipLaunchKernelGGL((k_split_scatter<u256, kSplitTB256, kSplitR>), dim3(grid),
                       dim3(kSplitTB256), 0, s, (const u256*)src, (u256*)dst, items, st, bins,
                       cursor, ncls, cls_stride);
  else if (words == 2)
    hipLaunchKernelGGL((k_split_scatter<u128, kSplitTB128, kSplitR>), dim3(grid),
                       dim3(kSplitTB128), 0, s, (const u128*)src, (u128*)dst, items, st, bins,
                       cursor, ncls, cls_stride);
  else
    hipLaunchKernelGGL((k_split_scatter<uint64_t, kSplitTB64, kSplitR>), dim3(grid),
                       dim3(kSplitTB64), 0, s, (const uint64_t*)src, (uint64_t*)dst, items, st,
                       bins, cursor, ncls, cls_stride);
  return hipGetLastError();
}

uint64_t small_leaf_max(int words) {
  // n + n/7 + 1 <= slots of the one-wave kernel (256-bit keys: sort-based only)
  return words == 4 ? 0 : words == 2 ? 447 : 895;
}

hipError_t launch_leaf_small(int words, int keybits, void* bufA, void* bufB, uint32_t* tmp_cnt,
                             const Leaf* leaves, DevState* st, uint64_t max_leaves,
                             uint32_t* d_out, uint32_t* large_list, uint32_t* ovf_list,
                             int slots_log2, hipStream_t s, int mode, bool refine, bool merged) {
  const bool wide = words == 2;
  const uint64_t small_max = mode == 1 ? 0 : small_leaf_max(words);
  // leaves of more than 8 first tables of records go straight to the second
  // count (where it runs: launch_leaf_second)
  const bool second = words == 1 && mode != 1 && slots_log2 < kRescueSlotsLog2 && ovf_list;
  const uint64_t huge_min = 8ull << slots_log2;
  // n_large and n_ovf
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, &st->n_large, (uint64_t)2, 0ull);
  hipLaunchKernelGGL(k_classify_leaves, dim3(grid_for(max_leaves, 256, 2048)), dim3(256), 0, s,
                     leaves, st, small_max, large_list, huge_min, second ? ovf_list : nullptr);
  if (mode == 1 || words == 4) {  // every non-empty leaf is in the list
    hipLaunchKernelGGL(k_empty_leaves, dim3(grid_for(max_leaves, 256, 2048)), dim3(256), 0, s,
                       leaves, st, d_out);
    return hipGetLastError();
  }
  const unsigned gsmall = persistent(max_leaves, kSmallGrid);
#define KC_SMALLW(HI, FF)                                                                        \
  hipLaunchKernelGGL((k_leaf_countw<u128, 64, kSmallCmax128, 8, HI, FF>), dim3(gsmall), dim3(64), \
                     0, s, keybits, (u128*)bufA, (u128*)bufB, tmp_cnt, leaves, st, d_out,        \
                     __builtin_ctz(kSmallCmax128), (const uint32_t*)nullptr, small_max)
#define KC_SMALL64(FF, MG)                                                                       \
  hipLaunchKernelGGL((k_leaf_count64<64, kSmallCmax64, 8, FF, MG>), dim3(gsmall), dim3(64), 0, s, \
                     keybits, (uint64_t*)bufA, (uint64_t*)bufB, tmp_cnt, leaves, st, d_out,      \
                     __builtin_ctz(kSmallCmax64), (const uint32_t*)nullptr,                      \
                     (const unsigned long long*)nullptr, (uint32_t*)nullptr, &st->large_records, \
                     small_max)
  if (wide) {
    if (keybits <= 126) {
      if (refine) KC_SMALLW(true, true); else KC_SMALLW(true, false);
    } else {
      if (refine) KC_SMALLW(false, true); else KC_SMALLW(false, false);
    }
  } else {
    if (merged) {
      if (refine) KC_SMALL64(true, true); else KC_SMALL64(false, true);
    } else {
      if (refine) KC_SMALL64(true, false); else KC_SMALL64(false, false);
    }
  }
#undef KC_SMALLW
#undef KC_SMALL64
  return hipGetLastError();
}

hipError_t launch_leaf_large(int words, int keybits, void* bufA, void* bufB, uint32_t* tmp_cnt,
                             const Leaf* leaves, DevState* st, uint64_t max_leaves,
                             uint32_t* d_out, int slots_log2, const uint32_t* large_list,
                             uint32_t* ovf_list, hipStream_t s, int mode, bool refine,
                             bool merged) {
  const bool wide = words == 2;
  const uint64_t small_max = small_leaf_max(words);
  const unsigned glarge = persistent(max_leaves, kPersistentGrid);
  if (mode == 1) {
    if (words == 4)
      hipLaunchKernelGGL((k_leaf_sort<u256, kLeafTB, kSortMax256>), dim3(glarge), dim3(kLeafTB),
                         0, s, keybits, (u256*)bufA, (u256*)bufB, tmp_cnt, leaves, st, d_out,
                         large_list);
    else if (wide)
      hipLaunchKernelGGL((k_leaf_sort<u128, kLeafTB, kSortMax128>), dim3(glarge), dim3(kLeafTB),
                         0, s, keybits, (u128*)bufA, (u128*)bufB, tmp_cnt, leaves, st, d_out,
                         large_list);
    else
      hipLaunchKernelGGL((k_leaf_radix64<kLeafTB, kSortMax64>), dim3(glarge), dim3(kLeafTB), 0, s,
                         keybits, (uint64_t*)bufA, (uint64_t*)bufB, tmp_cnt, leaves, st, d_out,
                         large_list);
    return hipGetLastError();
  }
#define KC_LARGEW(KT, CM, HI, FF)                                                               \
  hipLaunchKernelGGL((k_leaf_countw<KT, kLeafTB, CM, 4, HI, FF>), dim3(glarge), dim3(kLeafTB), 0, \
                     s, keybits, (KT*)bufA, (KT*)bufB, tmp_cnt, leaves, st, d_out, slots_log2,   \
                     large_list, small_max)
  // one-word keys: the leaves whose table overflows are listed for
  // launch_leaf_second
  uint32_t* const second = words == 1 && slots_log2 < kRescueSlotsLog2 ? ovf_list : nullptr;
#define KC_LARGE64(FF, MG)                                                                      \
  hipLaunchKernelGGL((k_leaf_count64<kLeafTB, kLeafCmax64, 4, FF, MG>), dim3(glarge),            \
                     dim3(kLeafTB), 0, s, keybits, (uint64_t*)bufA, (uint64_t*)bufB, tmp_cnt,    \
                     leaves, st, d_out, slots_log2, large_list, &st->n_large, second,            \
                     &st->large_records, small_max)
  if (words == 4) {
    if (refine) KC_LARGEW(u256, kLeafCmax256, false, true);
    else KC_LARGEW(u256, kLeafCmax256, false, false);
  } else if (wide) {
    if (keybits <= 126) {
      if (refine) KC_LARGEW(u128, kLeafCmax128, true, true);
      else KC_LARGEW(u128, kLeafCmax128, true, false);
    } else {
      if (refine) KC_LARGEW(u128, kLeafCmax128, false, true);
      else KC_LARGEW(u128, kLeafCmax128, false, false);
    }
  } else {
    if (merged) {
      if (refine) KC_LARGE64(true, true); else KC_LARGE64(false, true);
    } else {
      if (refine) KC_LARGE64(true, false); else KC_LARGE64(false, false);
    }
  }
#undef KC_LARGEW
#undef KC_LARGE64
  return hipGetLastError();
}

hipError_t launch_leaf_second(int words, int keybits, void* bufA, void* bufB, uint32_t* tmp_cnt,
                              const Leaf* leaves, DevState* st, uint32_t* d_out, int slots_log2,
                              const uint32_t* ovf_list, hipStream_t s, int mode, bool merged) {
  if (words != 1 || mode == 1 || slots_log2 >= kRescueSlotsLog2 || !ovf_list) return hipSuccess;
  // the leaves whose table overflowed are counted again at once by a
  // workgroup per CU with a table twice as large (a leaf overflows because of
  // its distinct keys: clusters of keys that share a long prefix, the
  // erroneous and diverged copies of frequent k-mers, which a split on the
  // next key bits barely thins out)
  hipLaunchKernelGGL(k_clear_overflow, dim3(1), dim3(64), 0, s, st);
  if (merged)
    hipLaunchKernelGGL((k_leaf_count64<kRescueTB, kRescueCmax64, 4, true, true>),
                       dim3(kRescueGrid), dim3(kRescueTB), 0, s, keybits, (uint64_t*)bufA,
                       (uint64_t*)bufB, tmp_cnt, leaves, st, d_out, slots_log2 + 1, ovf_list,
                       &st->n_ovf, (uint32_t*)nullptr, &st->second_records, (uint64_t)0);
  else
    hipLaunchKernelGGL((k_leaf_count64<kRescueTB, kRescueCmax64, 4, true, false>),
                       dim3(kRescueGrid), dim3(kRescueTB), 0, s, keybits, (uint64_t*)bufA,
                       (uint64_t*)bufB, tmp_cnt, leaves, st, d_out, slots_log2 + 1, ovf_list,
                       &st->n_ovf, (uint32_t*)nullptr, &st->second_records, (uint64_t)0);
  return hipGetLastError();
}

hipError_t launch_list_overflowed(const uint32_t* d, uint64_t n, const Leaf* leaves,
                                  uint32_t* list, Leaf* out, unsigned long long* count,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, count, (uint64_t)1, 0ull);
  if (n)
    hipLaunchKernelGGL(k_list_overflowed, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, d, n,
                       leaves, list, out, count);
  return hipGetLastError();
}

hipError_t launch_splice(const Leaf* leaves, const uint32_t* d, uint64_t n,
                         const uint32_t* root_leaf, const uint32_t* part_begin,
                         const uint32_t* nparts, uint32_t R, const Leaf* parts,
                         const uint32_t* part_d, uint32_t* cnt, DevState* st,
                         unsigned long long* bsum, unsigned long long* pos, Leaf* out,
                         uint32_t* out_d, hipStream_t s) {
  const unsigned g = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_splice_counts, dim3(g), dim3(256), 0, s, d, n, cnt);
  if (R)
    hipLaunchKernelGGL(k_splice_root_counts, dim3((R + 255) / 256), dim3(256), 0, s, root_leaf,
                       nparts, R, cnt);
  // st->n_leaves == n here: the scan gives every old leaf its first new slot
  hipError_t e = launch_plan_out(cnt, st, bsum, n, pos, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_splice_keep, dim3(g), dim3(256), 0, s, leaves, d, pos, n, out, out_d);
  if (R)
    hipLaunchKernelGGL(k_splice_parts, dim3(R < 4096u ? R : 4096u), dim3(64), 0, s, root_leaf,
                       part_begin, nparts, R, parts, part_d, pos, out, out_d);
  return hipGetLastError();
}

uint64_t scan_blocks(uint64_t max_leaves) { return (max_leaves + kScanTile - 1) / kScanTile; }

hipError_t launch_plan_out(const uint32_t* d, DevState* st, unsigned long long* bsum,
                           uint64_t max_leaves, unsigned long long* out_off, hipStream_t s) {
  const uint64_t nb = scan_blocks(max_leaves);
  if (nb > 65536u * kPlanTB) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanTB), 0, s, d, st, bsum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kPlanTB), 0, s, bsum, (uint32_t)nb, st);
  hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanTB), 0, s, d, st, bsum, out_off);
  return hipGetLastError();
}

hipError_t launch_concat(int words, const void* bufA, const void* bufB, const uint32_t* tmp_cnt,
                         const Leaf* leaves, const uint32_t* d, const unsigned long long* out_off,
                         const DevState* st, uint64_t max_leaves, uint64_t cap,
                         uint64_t* out_keys, uint32_t* out_counts, hipStream_t s) {
  const unsigned grid = persistent((max_leaves + 3) / 4, 16384);
  if (words == 4)
    hipLaunchKernelGGL(k_concat<u256>, dim3(grid), dim3(256), 0, s, (const u256*)bufA,
                       (const u256*)bufB, tmp_cnt, leaves, d, out_off, st, cap, out_keys,
                       out_counts);
  else if (words == 2)
    hipLaunchKernelGGL(k_concat<u128>, dim3(grid), dim3(256), 0, s, (const u128*)bufA,
                       (const u128*)bufB, tmp_cnt, leaves, d, out_off, st, cap, out_keys,
                       out_counts);
  else
    hipLaunchKernelGGL(k_concat<uint64_t>, dim3(grid), dim3(256), 0, s, (const uint64_t*)bufA,
                       (const uint64_t*)bufB, tmp_cnt, leaves, d, out_off, st, cap, out_keys,
                       out_counts);
  return hipGetLastError();
}

hipError_t launch_check(int words, const uint64_t* keys, const uint32_t* counts, uint64_t n,
                        int k, CheckResult* res, hipStream_t s) {
  if (!n) return hipSuccess;
  const unsigned grid = grid_for(n, 256, 4096);
  if (words == 4)
    hipLaunchKernelGGL(k_check<u256>, dim3(grid), dim3(256), 0, s, keys, counts, n, k, res);
  else if (words == 2)
    hipLaunchKernelGGL(k_check<u128>, dim3(grid), dim3(256), 0, s, keys, counts, n, k, res);
  else
    hipLaunchKernelGGL(k_check<uint64_t>, dim3(grid), dim3(256), 0, s, keys, counts, n, k, res);
  return hipGetLastError();
}

}  // namespace kc

namespace kc {

hipError_t launch_concat_batch(int words, const void* bufA, const void* bufB,
                               const uint32_t* tmp_cnt, const Leaf* leaves, const uint32_t* d,
                               const unsigned long long* out_off, const DevState* st,
                               uint64_t max_leaves, uint64_t cap, int k, uint64_t* out_keys,
                               uint32_t* out_counts, uint32_t* out_set, hipStream_t s) {
  const unsigned grid = persistent((max_leaves + 3) / 4, 16384);
  if (words == 4) return hipErrorInvalidValue;
  if (words == 2)
    hipLaunchKernelGGL(k_concat_batch<u128>, dim3(grid), dim3(256), 0, s, (const u128*)bufA,
                       (const u128*)bufB, tmp_cnt, leaves, d, out_off, st, cap, k, out_keys,
                       out_counts, out_set);
  else
    hipLaunchKernelGGL(k_concat_batch<uint64_t>, dim3(grid), dim3(256), 0, s,
                       (const uint64_t*)bufA, (const uint64_t*)bufB, tmp_cnt, leaves, d, out_off,
                       st, cap, k, out_keys, out_counts, out_set);
  return hipGetLastError();
}

hipError_t launch_set_bounds(const uint32_t* set, const DevState* st, uint64_t max_pairs,
                             uint32_t n_local, unsigned long long* start, hipStream_t s) {
  hipLaunchKernelGGL(k_set_bounds, dim3(grid_for(max_pairs + n_local + 1, 256, 4096)), dim3(256),
                     0, s, set, st, n_local, start);
  return hipGetLastError();
}

hipError_t launch_batch_offsets(const uint32_t* set_class, const uint32_t* set_local,
                                const unsigned long long* starts,
                                const unsigned long long* start_base, uint32_t n_sets,
                                unsigned long long* set_off, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_offsets, dim3(1), dim3(kPlanTB), 0, s, set_class, set_local, starts,
                     start_base, n_sets, set_off);
  return hipGetLastError();
}

hipError_t launch_batch_gather(const uint32_t* set_class, const uint32_t* set_local,
                               const unsigned long long* starts,
                               const unsigned long long* start_base,
                               const unsigned long long* class_base, const uint64_t* cls_keys,
                               const uint32_t* cls_counts, const unsigned long long* set_off,
                               uint32_t n_sets, uint64_t cap, uint64_t* out_keys,
                               uint32_t* out_counts, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_gather, dim3(2048), dim3(256), 0, s, set_class,
                     set_local, starts, start_base, class_base, cls_keys, cls_counts, set_off,
                     n_sets, cap, out_keys, out_counts);
  return hipGetLastError();
}

}  // namespace kc
