// CPU ORACLE FOR CANONICAL k-MER COUNTING — TEST INFRASTRUCTURE ONLY.
//
// Plain, slow, obviously-correct reference for what the GPU path computes.
// Only the tests, the smoke check and the benchmark's CPU-baseline leg use it;
// the product library never links, loads or calls it, and it shares no code,
// header, table or constant with the GPU kernels.
//
// What is computed (the k-mer histogram of Section II; serial sort-based
// counting of Algorithm 1, "Serial Algorithm"):
//   * Encode: A/a=0, C/c=1, G/g=2, T/t=3; any other byte is invalid and no
//     window covering it is counted (the paper only states that ASCII is
//     turned into a 2-bit code, Section V, Phase 1).
//   * GetFirstKmer builds the first k bases of a run of valid bases with the
//     first base most significant; each further base rolls in with
//     kmer = (kmer << 2) | Encode(base), masked to 2k bits (Algorithm 1 omits
//     the mask; without it older bases would pile up above bit 2k).
//   * The reverse complement rolls alongside:
//     rc = (rc >> 2) | ((3 - x) << 2(k-1)); the counted key is the canonical
//     form min(kmer, rc) as an unsigned integer.
//   * All keys are appended to T, T is sorted, and Accumulate sweeps the sorted
//     T into (k-mer, count) pairs in ascending key order (Algorithm 1).
// Keys are held as unsigned __int128 for k in [1, 64] and as a pair of them
// (U256 below) for k in [65, 128]; they are written out as 1 (k <= 32), 2
// (k <= 64) or 4 (k <= 128) little-endian 64-bit words. Counts are summed in
// 64 bits and reported as uint32 (an error is returned above 2^32-1).
//
// Multi-threading: T threads each run the steps above on a contiguous range of
// reads; the per-thread sorted (k-mer, count) lists are merged with a k-way
// merge that sums equal keys. This is Algorithm 1 applied to a partition of
// the reads, followed by the sum over parts that makes the result independent
// of the partition.
//
// A second, independent counter (oracle_count_map) uses std::unordered_map in
// place of sort-and-accumulate, as a cross-check of the first.
//
// parity pinned: see the oracle tests (hand-worked examples, brute force over
// strings, de Bruijn closed form, homopolymers, invariants).
#include <cstdint>
#include <cstring>
#include <algorithm>
#include <functional>
#include <queue>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <utility>
#include <vector>

typedef unsigned __int128 u128;

namespace {

// 256-bit unsigned integer for k-mers of more than 64 bases: only the
// operations the counting steps use (shifts by 0..255, OR, AND, order).
struct U256 {
  u128 lo = 0, hi = 0;
  U256() {}
  explicit U256(u128 x) : lo(x), hi(0) {}
  U256(u128 l, u128 h) : lo(l), hi(h) {}
  U256 operator<<(int s) const {
    if (s == 0) return *this;
    if (s >= 128) return U256(0, lo << (s - 128));
    return U256(lo << s, (hi << s) | (lo >> (128 - s)));
  }
  U256 operator>>(int s) const {
    if (s == 0) return *this;
    if (s >= 128) return U256(hi >> (s - 128), 0);
    return U256((lo >> s) | (hi << (128 - s)), hi >> s);
  }
  U256 operator|(const U256& o) const { return U256(lo | o.lo, hi | o.hi); }
  U256 operator&(const U256& o) const { return U256(lo & o.lo, hi & o.hi); }
  bool operator<(const U256& o) const { return hi != o.hi ? hi < o.hi : lo < o.lo; }
  bool operator==(const U256& o) const { return hi == o.hi && lo == o.lo; }
  bool operator!=(const U256& o) const { return !(*this == o); }
};

inline int key_words(int k) { return k <= 32 ? 1 : (k <= 64 ? 2 : 4); }

inline uint64_t word_of(const u128& x, int i) { return i < 2 ? (uint64_t)(x >> (64 * i)) : 0; }
inline uint64_t word_of(const U256& x, int i) {
  return i < 2 ? (uint64_t)(x.lo >> (64 * i)) : (uint64_t)(x.hi >> (64 * (i - 2)));
}
template <typename K> K key_from_words(const uint64_t* w, int words);
template <> u128 key_from_words<u128>(const uint64_t* w, int words) {
  return (u128)w[0] | (words > 1 ? (u128)w[1] << 64 : (u128)0);
}
template <> U256 key_from_words<U256>(const uint64_t* w, int words) {
  return U256((u128)w[0] | ((u128)w[1] << 64), (u128)w[2] | ((u128)w[3] << 64));
}

// Encode (Algorithm 1): 2-bit code of a base, -1 for a byte that is not a base.
inline int Encode(uint8_t c) {
  switch (c) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return -1;
  }
}

// 4^k - 1: the low 2k bits set.
inline u128 mask_bits128(int bits) { return bits >= 128 ? ~(u128)0 : (((u128)1 << bits) - 1); }
template <typename K> K kmer_mask(int k);
template <> u128 kmer_mask<u128>(int k) { return mask_bits128(2 * k); }
template <> U256 kmer_mask<U256>(int k) {
  return 2 * k <= 128 ? U256(mask_bits128(2 * k), 0) : U256(~(u128)0, mask_bits128(2 * k - 128));
}

// GetFirstKmer (Algorithm 1): the first k bases of s, first base most significant.
template <typename K>
K GetFirstKmer(const uint8_t* s, int k) {
  K kmer(0);
  for (int i = 0; i < k; ++i) kmer = (kmer << 2) | K((u128)Encode(s[i]));
  return kmer;
}

// Reverse complement of the first k bases of s, built directly from its definition:
// base j of the window contributes (3 - x_j) * 4^j.
template <typename K>
K FirstRevComp(const uint8_t* s, int k) {
  K rc(0);
  for (int j = 0; j < k; ++j) rc = rc | (K((u128)(3 - Encode(s[j]))) << (2 * j));
  return rc;
}

// Emit the canonical k-mer of every valid window of one read into T.
// A read is cut into maximal runs of valid bases; each run of length >= k is
// processed as Algorithm 1 processes a read: GetFirstKmer, then one rolling
// update per further base.
template <typename K>
void ParseRead(const uint8_t* R, uint64_t m, int k, const std::function<void(const K&)>& add) {
  const K mask = kmer_mask<K>(k);
  uint64_t i = 0;
  while (i < m) {
    while (i < m && Encode(R[i]) < 0) ++i;  // skip invalid bytes
    uint64_t a = i;
    while (i < m && Encode(R[i]) >= 0) ++i;
    uint64_t len = i - a;  // run [a, i) of valid bases
    if (len < (uint64_t)k) continue;
    const uint8_t* s = R + a;
    K kmer = GetFirstKmer<K>(s, k);
    K rc = FirstRevComp<K>(s, k);
    add(kmer < rc ? kmer : rc);
    for (uint64_t j = k; j < len; ++j) {
      const u128 x = (u128)Encode(s[j]);
      kmer = ((kmer << 2) | K(x)) & mask;
      rc = (rc >> 2) | (K(3 - x) << (2 * (k - 1)));
      add(kmer < rc ? kmer : rc);
    }
  }
}

template <typename K>
using Counts = std::vector<std::pair<K, uint64_t>>;

// Accumulate (Algorithm 1): sweep a sorted array, emit (k-mer, count).
template <typename K>
Counts<K> Accumulate(const std::vector<K>& T) {
  Counts<K> C;
  for (size_t i = 0; i < T.size();) {
    size_t j = i;
    while (j < T.size() && T[j] == T[i]) ++j;
    C.emplace_back(T[i], (uint64_t)(j - i));
    i = j;
  }
  return C;
}

// KmerCounting (Algorithm 1) over reads [r0, r1).
template <typename K>
Counts<K> KmerCountingRange(const uint8_t* reads, const uint64_t* off, uint64_t r0, uint64_t r1,
                            int k) {
  std::vector<K> T;
  for (uint64_t r = r0; r < r1; ++r)
    ParseRead<K>(reads + (off[r] - off[0]), off[r + 1] - off[r], k,
                 [&](const K& x) { T.push_back(x); });
  std::sort(T.begin(), T.end());
  return Accumulate(T);
}

// Contiguous read ranges with about the same number of bases each.
std::vector<uint64_t> SplitReads(const uint64_t* off, uint64_t n, int parts) {
  std::vector<uint64_t> cut(parts + 1, n);
  cut[0] = 0;
  uint64_t total = off[n] - off[0];
  uint64_t r = 0;
  for (int p = 1; p < parts; ++p) {
    uint64_t target = off[0] + (total * (uint64_t)p) / (uint64_t)parts;
    while (r < n && off[r] < target) ++r;
    cut[p] = r;
  }
  for (int p = 1; p <= parts; ++p) cut[p] = std::max(cut[p], cut[p - 1]);
  return cut;
}

// k-way merge of sorted count lists, summing equal keys.
template <typename K>
Counts<K> MergeSum(std::vector<Counts<K>>& parts) {
  typedef std::pair<K, size_t> Head;  // (key, part)
  auto later = [](const Head& a, const Head& b) {
    return b.first < a.first || (a.first == b.first && b.second < a.second);
  };
  std::priority_queue<Head, std::vector<Head>, decltype(later)> pq(later);
  std::vector<size_t> pos(parts.size(), 0);
  for (size_t p = 0; p < parts.size(); ++p)
    if (!parts[p].empty()) pq.push({parts[p][0].first, p});
  Counts<K> out;
  while (!pq.empty()) {
    Head h = pq.top(); pq.pop();
    uint64_t c = parts[h.second][pos[h.second]].second;
    if (++pos[h.second] < parts[h.second].size()) pq.push({parts[h.second][pos[h.second]].first, h.second});
    if (!out.empty() && out.back().first == h.first) out.back().second += c;
    else out.emplace_back(h.first, c);
  }
  return out;
}

// Keys as `words` 64-bit words each (row i at out_keys[i * words]).
template <typename K>
int Emit(const Counts<K>& C, int words, uint64_t* out_keys, uint32_t* cnt, uint64_t cap,
         uint64_t* n_out) {
  *n_out = C.size();
  if (C.size() > cap) return -3;
  for (size_t i = 0; i < C.size(); ++i) {
    if (C[i].second > 0xFFFFFFFFull) return -4;
    for (int w = 0; w < words; ++w) out_keys[i * words + w] = word_of(C[i].first, w);
    cnt[i] = (uint32_t)C[i].second;
  }
  return 0;
}

int CheckArgs(const uint8_t* reads, const uint64_t* off, uint64_t n, int k) {
  if (k < 1 || k > 128 || !off || (n && !reads)) return -1;
  for (uint64_t i = 0; i < n; ++i) if (off[i + 1] < off[i]) return -1;
  return 0;
}

struct KeyHash {
  static size_t mix(uint64_t a, uint64_t b) {
    return (size_t)(a * 0x9E3779B97F4A7C15ULL ^ (b + 0x7F4A7C159E3779B9ULL + (a >> 29)));
  }
  size_t operator()(const u128& x) const { return mix((uint64_t)x, (uint64_t)(x >> 64)); }
  size_t operator()(const U256& x) const {
    return mix((uint64_t)x.lo ^ (uint64_t)(x.hi >> 64) * 31, (uint64_t)(x.lo >> 64) ^ (uint64_t)x.hi);
  }
};

template <typename K>
int CountSort(const uint8_t* reads, const uint64_t* off, uint64_t n, int k, int threads,
              uint64_t* out_keys, uint32_t* out_cnt, uint64_t cap, uint64_t* n_out) {
  std::vector<uint64_t> cut = SplitReads(off, n, threads);
  std::vector<Counts<K>> parts(threads);
  std::vector<std::thread> ts;
  for (int t = 0; t < threads; ++t)
    ts.emplace_back([&, t] { parts[t] = KmerCountingRange<K>(reads, off, cut[t], cut[t + 1], k); });
  for (auto& t : ts) t.join();
  Counts<K> C = threads == 1 ? std::move(parts[0]) : MergeSum(parts);
  return Emit(C, key_words(k), out_keys, out_cnt, cap, n_out);
}

template <typename K>
int CountMap(const uint8_t* reads, const uint64_t* off, uint64_t n, int k, uint64_t* out_keys,
             uint32_t* out_cnt, uint64_t cap, uint64_t* n_out) {
  std::unordered_map<K, uint64_t, KeyHash> M;
  for (uint64_t r = 0; r < n; ++r)
    ParseRead<K>(reads + (off[r] - off[0]), off[r + 1] - off[r], k, [&](const K& x) { ++M[x]; });
  Counts<K> C(M.begin(), M.end());
  std::sort(C.begin(), C.end());
  return Emit(C, key_words(k), out_keys, out_cnt, cap, n_out);
}

template <typename K>
int CountSelected(const uint8_t* reads, const uint64_t* off, uint64_t n, int k, int threads,
                  const uint64_t* keys, uint64_t nkeys, uint64_t* out_cnt) {
  const int words = key_words(k);
  std::unordered_map<K, uint64_t, KeyHash> idx;
  for (uint64_t i = 0; i < nkeys; ++i) idx[key_from_words<K>(keys + i * words, words)] = i;
  std::vector<uint64_t> cut = SplitReads(off, n, threads);
  std::vector<std::vector<uint64_t>> acc(threads, std::vector<uint64_t>(nkeys, 0));
  std::vector<std::thread> ts;
  for (int t = 0; t < threads; ++t)
    ts.emplace_back([&, t] {
      for (uint64_t r = cut[t]; r < cut[t + 1]; ++r)
        ParseRead<K>(reads + (off[r] - off[0]), off[r + 1] - off[r], k, [&](const K& x) {
          auto it = idx.find(x);
          if (it != idx.end()) ++acc[t][it->second];
        });
    });
  for (auto& t : ts) t.join();
  for (uint64_t i = 0; i < nkeys; ++i) {
    uint64_t s = 0;
    for (int t = 0; t < threads; ++t) s += acc[t][i];
    out_cnt[i] = s;
  }
  return 0;
}

}  // namespace

extern "C" {

// Number of valid windows: positions whose k bases are all A/C/G/T (either case).
uint64_t oracle_valid_windows(const uint8_t* reads, const uint64_t* off, uint64_t n, int k) {
  uint64_t w = 0;
  for (uint64_t r = 0; r < n; ++r) {
    const uint8_t* R = reads + (off[r] - off[0]);
    uint64_t run = 0, m = off[r + 1] - off[r];
    for (uint64_t i = 0; i < m; ++i) {
      run = Encode(R[i]) >= 0 ? run + 1 : 0;
      if (run >= (uint64_t)k) ++w;
    }
  }
  return w;
}

// Sorted (k-mer, count) output of Algorithm 1 (canonical, masked, N skipped).
// Key i is written to out_keys[i * w .. i * w + w), w = 1 (k <= 32), 2
// (k <= 64) or 4 (k <= 128) 64-bit words, least significant first. Returns 0,
// -1 bad args, -3 capacity (n_out set), -4 count overflow.
int oracle_count_sort(const uint8_t* reads, const uint64_t* off, uint64_t n, int k, int threads,
                      uint64_t* out_keys, uint32_t* out_cnt, uint64_t cap, uint64_t* n_out) {
  if (CheckArgs(reads, off, n, k)) return -1;
  if (threads < 1) threads = 1;
  return k <= 64 ? CountSort<u128>(reads, off, n, k, threads, out_keys, out_cnt, cap, n_out)
                 : CountSort<U256>(reads, off, n, k, threads, out_keys, out_cnt, cap, n_out);
}

// Cross-check counter: hash map instead of sort-and-accumulate, then sort the keys.
int oracle_count_map(const uint8_t* reads, const uint64_t* off, uint64_t n, int k,
                     uint64_t* out_keys, uint32_t* out_cnt, uint64_t cap, uint64_t* n_out) {
  if (CheckArgs(reads, off, n, k)) return -1;
  return k <= 64 ? CountMap<u128>(reads, off, n, k, out_keys, out_cnt, cap, n_out)
                 : CountMap<U256>(reads, off, n, k, out_keys, out_cnt, cap, n_out);
}

// Counts of selected keys only (for inputs too large to count in full):
// every window is parsed as above, and its canonical key is looked up in the
// set of requested keys (nkeys keys of w words each, as written above).
// out_cnt[i] receives the count of key i (0 if absent).
int oracle_count_selected(const uint8_t* reads, const uint64_t* off, uint64_t n, int k, int threads,
                          const uint64_t* keys, uint64_t nkeys, uint64_t* out_cnt) {
  if (CheckArgs(reads, off, n, k)) return -1;
  if (threads < 1) threads = 1;
  return k <= 64 ? CountSelected<u128>(reads, off, n, k, threads, keys, nkeys, out_cnt)
                 : CountSelected<U256>(reads, off, n, k, threads, keys, nkeys, out_cnt);
}

}  // extern "C"
