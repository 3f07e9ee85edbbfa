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

// Per bin being split: its sub-bin counters (and cursors, and leaf slots in the
// device-planned path) start at hist_off; the sub-bin of a key is
// (key >> shift) & ((1 << nbits) - 1). nbits == 0: the bin is not split.
struct SplitBin {
  uint64_t hist_off;
  uint32_t shift, nbits;
};

// A leaf partition: records [begin, end) of buffer `buf` (0 = A, 1 = B) whose
// keys share their top `bits` key bits. Its sorted (key, count) pairs are
// written to the other buffer (and the pair-count array) at [begin, begin + d).
// cshift != 0: the records are pre-aggregated (one-word keys only): bits
// [cshift, 64) of a record hold its count minus one in place of the key's top
// bits, which are `shard` (the key is (shard << cshift) | (record & (2^cshift - 1))).
struct Leaf {
  uint64_t begin, end;
  uint32_t buf, bits;
  uint32_t cshift, shard;
};

// Device-side result flags of the output self-check.
struct CheckResult {
  unsigned long long sum_counts;
  unsigned int not_sorted, not_canonical, out_of_range, zero_count;
};

// Per-call device state: counters written by the planning kernels and flags.
struct DevState {
  unsigned long long W;         // valid windows
  unsigned long long n_items;   // split work items
  unsigned long long n_leaves;  // leaf slots
  unsigned long long D;         // distinct keys (sum of leaf counts)
  unsigned long long n_large;   // leaves handled by the block-wide leaf kernel
  unsigned long long n_ovf;     // of those, leaves whose table overflowed (second-chance list)
  unsigned long long large_records, large_distinct;  // work of the block-wide leaf kernel
  unsigned long long second_records, second_distinct;  // work of its second count
  unsigned int overflow;        // a leaf table overflowed (device-planned path cannot finish)
  unsigned int count_overflow;  // a count exceeds 2^32-1
  unsigned int pad[2];
  CheckResult check;
};

// Read sets of a batch, for the window kernels: set_byte_off[s] is the first
// byte of set s relative to the packed stream (n_sets + 1 entries), and
// set_local[s] its id within the k-class being counted (kNoSet if the set
// belongs to another class).
struct BatchSets {
  const unsigned long long* set_byte_off;
  const uint32_t* set_local;
  uint32_t n_sets;
};
constexpr uint32_t kNoSet = 0xFFFFFFFFu;

constexpr int kMaxShardBits = 10;  // first-level shards (owner buckets are unions of them)
constexpr int kSplitMaxBits = 10;  // sub-bins per split step: up to 1024
constexpr int kWinStarts = 8;      // window starts per thread in the window kernels
constexpr int kXcds = 8;           // XCDs of the chip: classes of owner-scatter tiles
constexpr uint32_t kLeafOverflow = 0xFFFFFFFFu;

int max_leaf_slots_log2(int words);
int max_shard_bits();
// records per split work item (records_per_thread: 8, or 16 for one-word keys)
int split_tile(int words, int records_per_thread);

hipError_t launch_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v, hipStream_t s);

hipError_t launch_pack(const uint8_t* src, uint64_t n_bytes, const uint64_t* offsets,
                       uint64_t n_reads, uint64_t off0, uint64_t* packed, uint64_t* inv,
                       uint64_t* endm, uint64_t nchunks, hipStream_t s);

// Valid-start mask of the windows of k bytes starting in [byte_begin,
// byte_end), from the invalid-byte and read-end masks of launch_pack: bit j of
// valid[w] is set iff the window starting at byte 64w + j is valid. Writes the
// words the window kernels below read for the same byte range (valid holds as
// many words as inv).
hipError_t launch_valid_mask(int words, const uint64_t* inv, const uint64_t* endm,
                             uint64_t byte_begin, uint64_t byte_end, int k, uint64_t* valid,
                             hipStream_t s);

// Window kernels over the bytes [byte_begin, byte_end) of the packed stream,
// with the valid-start mask of launch_valid_mask for the same range and k.
// keybits = 2k (plain) or 2k + set id bits (batch: batch != nullptr).
// hist: (1 + kXcds) << shard_bits entries, zeroed: per-shard totals, then
// per class of the owner scatter's tiles (tile index mod kXcds; the scatter's
// shape follows from words and starts_per_thread).
hipError_t launch_window_hist(int words, const uint64_t* packed, const uint64_t* valid,
                              uint64_t byte_begin, uint64_t byte_end, int k,
                              int keybits, int shard_bits, const BatchSets* batch,
                              unsigned long long* hist, unsigned long long* wcount,
                              int starts_per_thread, hipStream_t s);

// starts_per_thread: 8, or 16 for one-word keys (16,384-record LDS tiles).
// cursor[]: the class cursors of launch_plan_shards; a tile of class x takes
// its runs from cursor[x << shard_bits + shard].
hipError_t launch_window_scatter(int words, const uint64_t* packed, const uint64_t* valid,
                                 uint64_t byte_begin, uint64_t byte_end,
                                 int k, int keybits, int shard_bits, const BatchSets* batch,
                                 unsigned long long* cursor, void* out, int starts_per_thread,
                                 hipStream_t s);

// Device planning of the first split level. order[] lists shards
// owner-major; sbegin[] receives each shard's record range start, cursor[]
// (kXcds << shard_bits entries) where each tile class's part of each shard
// slice starts (from the class counts of hist[]); bins[] the split of each shard; items[] the tiles of
// the split shards (item_off[] holds nb+1 prefix offsets of them); subhist[]
// (ncls * max_leaves entries: one part per item class of the split) is
// prepared: zeros, but the shard size at the leaf of each unsplit shard in
// the first part; st->n_items and st->n_leaves are set.
hipError_t launch_plan_shards(const unsigned long long* hist, const int* order, int shard_bits,
                              int keybits, uint64_t leaf_target, uint64_t leaf_attempt,
                              int tile, unsigned long long* sbegin, unsigned long long* cursor,
                              SplitBin* bins, SplitItem* items, unsigned long long* item_off,
                              unsigned long long* subhist, uint64_t max_leaves,
                              uint64_t max_items, int ncls, DevState* st, hipStream_t s);

// Device planning of the leaves (one block): leaf table in key order and the
// sub-bin cursors of the split shards.
// merge_cshift != 0: the split scatter pre-aggregates (the leaves of split
// shards get cshift = merge_cshift and their shard).
// Item classes: item w of the split is of class w mod ncls; the sub-bin
// counts of class x are at subhist[x * cls_stride + leaf], and the split
// scatter's cursors of class x at cursor[x * cls_stride + leaf] (each class
// writes its own part of every sub-bin, the classes in order).
hipError_t launch_plan_leaves(const unsigned long long* hist, const unsigned long long* sbegin,
                              const SplitBin* bins, int shard_bits,
                              const unsigned long long* subhist, Leaf* leaves,
                              unsigned long long* cursor, int merge_cshift, int ncls,
                              uint64_t cls_stride, hipStream_t s);

// Split kernels loop over st->n_items items (persistent grid of at most max_items blocks).
hipError_t launch_split_hist(int words, const void* src, const SplitItem* items,
                             const DevState* st, uint64_t max_items, const SplitBin* bins,
                             unsigned long long* subhist, int ncls, uint64_t cls_stride,
                             hipStream_t s);

// merge_cshift != 0 (one-word keys, 16 records per thread): equal keys next
// to each other in a tile's LDS staging (same sub-bin) leave as one record
// carrying its count minus one in bits [merge_cshift, 64); the cursors then
// advance by the records written, and launch_leaf_ends records where each
// split leaf's records end (ncls must then be 1).
hipError_t launch_split_scatter(int words, const void* src, void* dst, const SplitItem* items,
                                const DevState* st, uint64_t max_items, const SplitBin* bins,
                                unsigned long long* cursor, int records_per_thread,
                                int merge_cshift, int ncls, uint64_t cls_stride, hipStream_t s);
hipError_t launch_leaf_ends(Leaf* leaves, const unsigned long long* cursor, const DevState* st,
                            uint64_t max_leaves, hipStream_t s);

// Count each of the st->n_leaves leaves, write its sorted pairs next to it.
// d_out[i] = distinct keys of leaf i, or kLeafOverflow (and st->overflow = 1)
// if it could not be counted whole. mode 0: LDS open-addressing tables, then
// an in-LDS sort of the distinct keys; leaves of at most small_leaf_max()
// records go to one-wave workgroups with private tables, larger ones (listed
// in large_list, which holds max_leaves entries) to 512-thread workgroups.
// mode 1: every non-empty leaf's records are sorted in LDS and run-length
// accumulated (the launch_leaf_small call then only lists the leaves).
// refine: the leaves are parts of overflowed leaves (first table full size;
// the launches are separate kernel instantiations, so profiles tell them apart).
// merged: leaves may hold pre-aggregated records (one-word keys).
// ovf_list (max_leaves entries, or nullptr): one-word keys in mode 0 list
// there the leaves whose table overflows, for launch_leaf_second.
// launch_leaf_small also classifies the leaves: large ones into large_list;
// for one-word keys in mode 0 with ovf_list (and the second count running,
// slots_log2 below its table), leaves of more than 8 << slots_log2 records
// straight into ovf_list for launch_leaf_second.
hipError_t launch_leaf_small(int words, int keybits, void* bufA, void* bufB, uint32_t* tmp_cnt,
                             const Leaf* leaves, DevState* st, uint64_t max_leaves,
                             uint32_t* d_out, uint32_t* large_list, uint32_t* ovf_list,
                             int slots_log2, hipStream_t s, int mode, bool refine, bool merged);
hipError_t launch_leaf_large(int words, int keybits, void* bufA, void* bufB, uint32_t* tmp_cnt,
                             const Leaf* leaves, DevState* st, uint64_t max_leaves,
                             uint32_t* d_out, int slots_log2, const uint32_t* large_list,
                             uint32_t* ovf_list, hipStream_t s, int mode, bool refine,
                             bool merged);
// Second count of the leaves launch_leaf_large listed in ovf_list, with a
// table twice as large (one 1,024-thread workgroup per CU); only what
// overflows that table too stays marked overflowed (st->overflow is raised
// again by those, and by launch_plan_out from the leaf counts). A no-op
// where launch_leaf_large lists nothing.
hipError_t launch_leaf_second(int words, int keybits, void* bufA, void* bufB, uint32_t* tmp_cnt,
                              const Leaf* leaves, DevState* st, uint32_t* d_out, int slots_log2,
                              const uint32_t* ovf_list, hipStream_t s, int mode, bool merged);
uint64_t small_leaf_max(int words);

// Exclusive scan of leaf counts into output offsets; st->D = total. bsum
// holds scan_blocks(max_leaves) values.
hipError_t launch_plan_out(const uint32_t* d, DevState* st, unsigned long long* bsum,
                           uint64_t max_leaves, unsigned long long* out_off, hipStream_t s);
uint64_t scan_blocks(uint64_t max_leaves);

// Overflow refinement: list the overflowed leaves (indices and entries; *count
// receives their number), and splice refined parts into the leaf list:
// old leaf i (of n, st->n_leaves == n) keeps one slot, or nparts[r] slots if it
// is root_leaf[r]; parts of root r are parts[part_begin[r] ..] with counts
// part_d. Writes the new list to out / out_d (st->D receives its length).
hipError_t launch_list_overflowed(const uint32_t* d, uint64_t n, const Leaf* leaves,
                                  uint32_t* list, Leaf* out, unsigned long long* count,
                                  hipStream_t s);
hipError_t launch_splice(const Leaf* leaves, const uint32_t* d, uint64_t n,
                         const uint32_t* root_leaf, const uint32_t* part_begin,
                         const uint32_t* nparts, uint32_t R, const Leaf* parts,
                         const uint32_t* part_d, uint32_t* cnt, DevState* st,
                         unsigned long long* bsum, unsigned long long* pos, Leaf* out,
                         uint32_t* out_d, hipStream_t s);

// Output of the leaves in key order (up to cap pairs). Does nothing while
// st->overflow is set: the host refines the overflowed leaves first and
// launches it again (the concat of a batch class likewise: the class is
// recounted set by set).
hipError_t launch_concat(int words, const void* bufA, const void* bufB, const uint32_t* tmp_cnt,
                         const Leaf* leaves, const uint32_t* d, const unsigned long long* out_off,
                         const DevState* st, uint64_t max_leaves, uint64_t cap,
                         uint64_t* out_keys, uint32_t* out_counts, hipStream_t s);

// Batch helpers: class concat (k-mer, count, set id within the class), set
// bounds in a class output, global set offsets and the final gather.
hipError_t launch_concat_batch(int words, const void* bufA, const void* bufB,
                               const uint32_t* tmp_cnt, const Leaf* leaves, const uint32_t* d,
                               const unsigned long long* out_off, const DevState* st,
                               uint64_t max_leaves, uint64_t cap, int k, uint64_t* out_keys,
                               uint32_t* out_counts, uint32_t* out_set, hipStream_t s);
hipError_t launch_set_bounds(const uint32_t* set, const DevState* st, uint64_t max_pairs,
                             uint32_t n_local, unsigned long long* start, hipStream_t s);
hipError_t launch_batch_offsets(const uint32_t* set_class, const uint32_t* set_local,
                                const unsigned long long* starts,
                                const unsigned long long* start_base, uint32_t n_sets,
                                unsigned long long* set_off, hipStream_t s);
hipError_t launch_batch_gather(const uint32_t* set_class, const uint32_t* set_local,
                               const unsigned long long* starts,
                               const unsigned long long* start_base,
                               const unsigned long long* class_base, const uint64_t* cls_keys,
                               const uint32_t* cls_counts, const unsigned long long* set_off,
                               uint32_t n_sets, uint64_t cap, uint64_t* out_keys,
                               uint32_t* out_counts, hipStream_t s);

hipError_t launch_check(int words, const uint64_t* keys, const uint32_t* counts, uint64_t n,
                        int k, CheckResult* res, hipStream_t s);

}  // namespace kc
