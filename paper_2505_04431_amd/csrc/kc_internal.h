// Internal interface between the host runtime (kc_runtime.cpp) and the
// device kernels (kc_kernels.hip). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kc {

// A tile of records [begin, end) of split-list bin `bin`.
struct SplitItem {
  uint64_t begin, end;
  uint32_t bin, pad;
};

// Per bin being split: its sub-bin counters start at hist_off; the sub-bin of
// a key is (key >> shift) & ((1 << nbits) - 1).
struct SplitBin {
  uint64_t hist_off;
  uint32_t shift, nbits;
};

// A leaf partition: records [begin, end) of buffer `buf` (0 = A, 1 = B);
// its sorted (key, count) pairs go to the other buffer at [begin, begin + d)
// and, at the end, to the output at out_off.
struct Leaf {
  uint64_t begin, end;
  uint64_t out_off;
  uint32_t buf, pad;
};

// Device-side result flags of the output self-check.
struct CheckResult {
  unsigned long long sum_counts;
  unsigned int not_sorted, not_canonical, out_of_range, zero_count;
};

constexpr int kMaxShardBits = 10;  // first-level shards (owner buckets are unions of them)
constexpr int kSplitMaxBits = 8;   // sub-bins per split step: up to 256
constexpr int kSplitTile = 8192;   // records per split work item
constexpr int kWinStarts = 8;      // window starts per thread in the window kernels

// `wide` selects 128-bit keys (33 <= k <= 64) instead of 64-bit keys.
hipError_t launch_pack(const uint8_t* src, uint64_t n_bytes, const uint64_t* offsets,
                       uint64_t n_reads, uint64_t off0, uint64_t* packed, uint64_t* inv,
                       uint64_t* endm, uint64_t nchunks, hipStream_t s);

hipError_t launch_window_hist(bool wide, const uint64_t* packed, const uint64_t* inv,
                              const uint64_t* endm, uint64_t n_bytes, int k, int shard_bits,
                              unsigned long long* hist, unsigned long long* wcount,
                              hipStream_t s);

hipError_t launch_window_scatter(bool wide, const uint64_t* packed, const uint64_t* inv,
                                 const uint64_t* endm, uint64_t n_bytes, int k, int shard_bits,
                                 unsigned long long* cursor, void* out, hipStream_t s);

hipError_t launch_split_hist(bool wide, const void* src, const SplitItem* items,
                             uint64_t n_items, const SplitBin* bins,
                             unsigned long long* subhist, hipStream_t s);

hipError_t launch_split_scatter(bool wide, const void* src, void* dst, const SplitItem* items,
                                uint64_t n_items, const SplitBin* bins,
                                unsigned long long* cursor, hipStream_t s);

// Count each leaf in an LDS open-addressing table; write sorted pairs next to it.
// d_out[i] = distinct keys of leaf i, or 0xFFFFFFFF if its table overflowed.
hipError_t launch_leaf_count(bool wide, void* bufA, void* bufB, uint32_t* tmp_cnt,
                             const Leaf* leaves, uint64_t n_leaves, uint32_t* d_out,
                             int slots_log2, unsigned int* count_overflow, hipStream_t s);

hipError_t launch_concat(bool wide, const void* bufA, const void* bufB, const uint32_t* tmp_cnt,
                         const Leaf* leaves, const uint32_t* d, uint64_t n_leaves,
                         uint64_t* out_keys, uint32_t* out_counts, hipStream_t s);

hipError_t launch_check(bool wide, const uint64_t* keys, const uint32_t* counts, uint64_t n,
                        int k, CheckResult* res, hipStream_t s);

int max_leaf_slots_log2(bool wide);
int max_shard_bits();
int split_tile(bool wide);  // records per split work item

}  // namespace kc
