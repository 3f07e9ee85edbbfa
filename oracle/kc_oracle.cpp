// CPU ORACLE FOR CANONICAL k-MER COUNTING — TEST INFRASTRUCTURE ONLY.
//
// Plain, slow, obviously-correct reference for what the GPU path computes.
// Only the tests, the smoke check and the benchmark's CPU-baseline leg use it;
// the product library never links, loads or calls it, and it shares no code
// or header with the GPU kernels (it needs no hash function at all).
//
// What is computed: the k-mer histogram of Section II (counted serially by
// sorting in Algorithm 1), written out from its definition:
//   * a byte is a base iff it is A, C, G or T in either case, with codes
//     A=0, C=1, G=2, T=3 (the paper only says ASCII becomes a 2-bit code,
//     Section V, Phase 1);
//   * window (read i, start p) is valid iff its k bytes are all bases;
//   * its forward value is sum_j code(p+j) * 4^(k-1-j) (first base most
//     significant, as in Algorithm 1), its reverse-complement value
//     sum_j (3 - code(p+j)) * 4^j, and its key the smaller of the two as an
//     unsigned 2k-bit integer (the canonical k-mer);
//   * the result lists every key that occurs with its number of valid windows,
//     in ascending key order.
// Each valid window's two values are decoded directly from its k bytes (no
// value is carried from one window to the next); keys are gathered, sorted
// with std::sort and tallied run by run. Keys are uint64_t for k <= 32,
// unsigned __int128 for k <= 64 and a pair of 128-bit halves (Wide below) for
// 65 <= k <= 128, written out as
// 1 (k <= 32), 2 (k <= 64) or 4 (k <= 128) 64-bit words, least significant
// first. Counts are summed in 64 bits and reported as uint32 (an error is
// returned above 2^32 - 1).
//
// Threads: keys are filed by their top bits while the reads are decoded in
// parallel, and each range of top bits is then sorted and tallied on its own
// (the ranges are disjoint and ascending, so their tallies concatenate to the
// whole histogram). A second counter (oracle_count_map) tallies in a std::map
// instead, as a cross-check. oracle_count_range restricts the tally to keys
// whose top bits lie in a range, so that inputs too large to tally at once
// are compared slice by slice.
//
// parity pinned: see tests/test_oracle_pins.py (hand-worked examples, brute
// force over strings, de Bruijn closed form, homopolymers, invariants, range
// slices against the full tally).
#include <cstdint>
#include <cstring>
#include <algorithm>
#include <atomic>
#include <map>
#include <thread>
#include <utility>
#include <vector>

typedef unsigned __int128 u128;

namespace {

// 256-bit unsigned integer for k-mers of more than 64 bases: only what the
// decoding and ordering use (times 4 plus a digit, order).
struct Wide {
  u128 lo = 0, hi = 0;
  Wide() {}
  explicit Wide(u128 x) : lo(x), hi(0) {}
  Wide(u128 l, u128 h) : lo(l), hi(h) {}
  Wide times4_plus(unsigned v) const {  // this * 4 + v, v < 4 (the caller keeps 2k <= 256)
    return Wide((lo << 2) | v, (hi << 2) | (lo >> 126));
  }
  bool operator<(const Wide& o) const { return hi != o.hi ? hi < o.hi : lo < o.lo; }
  bool operator==(const Wide& o) const { return hi == o.hi && lo == o.lo; }
};

inline uint64_t times4_plus(uint64_t x, unsigned v) { return (x << 2) | v; }
inline u128 times4_plus(u128 x, unsigned v) { return (x << 2) | v; }
inline Wide times4_plus(const Wide& x, unsigned v) { return x.times4_plus(v); }

// The top `nbits` bits of a key of `total` bits (1 <= nbits <= 16).
inline unsigned top_of(uint64_t x, int total, int nbits) { return (unsigned)(x >> (total - nbits)); }
inline unsigned top_of(u128 x, int total, int nbits) { return (unsigned)(x >> (total - nbits)); }
inline unsigned top_of(const Wide& x, int total, int nbits) {
  const int s = total - nbits;  // >= 0
  if (s >= 128) return (unsigned)(x.hi >> (s - 128));
  if (s == 0) return (unsigned)x.lo;
  return (unsigned)((x.lo >> s) | (x.hi << (128 - s)));
}

inline int words_per_key(int k) { return k <= 32 ? 1 : (k <= 64 ? 2 : 4); }
inline uint64_t out_word(uint64_t x, int i) { return i == 0 ? x : 0; }
inline uint64_t out_word(const u128& x, int i) { return i < 2 ? (uint64_t)(x >> (64 * i)) : 0; }
inline uint64_t out_word(const Wide& x, int i) {
  return i < 2 ? (uint64_t)(x.lo >> (64 * i)) : (uint64_t)(x.hi >> (64 * (i - 2)));
}

// Code of a byte: 0..3 for a base, 4 for anything else.
struct CodeTable {
  uint8_t c[256];
  CodeTable() {
    for (int i = 0; i < 256; ++i) c[i] = 4;
    const char* up = "ACGT";
    const char* lo = "acgt";
    for (int v = 0; v < 4; ++v) {
      c[(uint8_t)up[v]] = (uint8_t)v;
      c[(uint8_t)lo[v]] = (uint8_t)v;
    }
  }
};
const CodeTable kCode;

// Optional restriction to keys whose top `bits` bits (of the 2k-bit key) lie
// in [lo, hi). The top bits of the smaller of two numbers are the smaller of
// their top bits, and the top digits of the forward value are the window's
// first bases while those of the reverse complement are the complements of
// its last bases, last first: so whether a window's key is in the range is
// known from d = ceil(bits / 2) bases at each of its ends, and only the
// windows inside the range are decoded in full.
struct Range {
  int bits = 0;
  uint64_t lo = 0, hi = 0;
  bool keeps_window(const uint8_t* w, int k) const {
    if (bits == 0) return true;
    const int d = (bits + 1) / 2;
    uint64_t tf = 0, tr = 0;
    for (int j = 0; j < d; ++j) tf = tf * 4 + kCode.c[w[j]];
    for (int j = k - 1; j >= k - d; --j) tr = tr * 4 + (3u - kCode.c[w[j]]);
    const uint64_t t = std::min(tf, tr) >> (2 * d - bits);
    return t >= lo && t < hi;
  }
};

// Calls f(key) for every valid window of read R (m bytes) that `range` keeps,
// in window order. The validity of a window is read off the run of bases
// that ends at each byte; its forward and reverse-complement values are
// decoded from its own k bytes.
template <typename K, typename F>
void for_each_window_key(const uint8_t* R, uint64_t m, int k, const Range& range, F&& f) {
  uint64_t run = 0;  // bases ending at byte i (inclusive)
  for (uint64_t i = 0; i < m; ++i) {
    run = kCode.c[R[i]] < 4 ? run + 1 : 0;
    if (run < (uint64_t)k) continue;
    const uint8_t* w = R + (i + 1 - k);  // window [i+1-k, i]
    if (!range.keeps_window(w, k)) continue;
    K fwd(0), rc(0);
    for (int j = 0; j < k; ++j) fwd = times4_plus(fwd, kCode.c[w[j]]);       // first base most significant
    for (int j = k - 1; j >= 0; --j) rc = times4_plus(rc, 3u - kCode.c[w[j]]);  // base j weighs 4^j
    f(rc < fwd ? rc : fwd);
  }
}

template <typename K>
using Tally = std::vector<std::pair<K, uint64_t>>;

// Sorted keys -> (key, number of copies) for each run of equal keys.
template <typename K>
Tally<K> tally_sorted(const std::vector<K>& keys) {
  Tally<K> out;
  size_t i = 0;
  while (i < keys.size()) {
    size_t j = i + 1;
    while (j < keys.size() && keys[j] == keys[i]) ++j;
    out.push_back({keys[i], (uint64_t)(j - i)});
    i = j;
  }
  return out;
}

// Contiguous read ranges holding about the same number of bytes each.
std::vector<uint64_t> read_ranges(const uint64_t* off, uint64_t n, int parts) {
  std::vector<uint64_t> cut(parts + 1, n);
  cut[0] = 0;
  const uint64_t total = off[n] - off[0];
  uint64_t r = 0;
  for (int p = 1; p < parts; ++p) {
    const uint64_t target = off[0] + (total * (uint64_t)p) / (uint64_t)parts;
    while (r < n && off[r] < target) ++r;
    cut[p] = r;
  }
  for (int p = 1; p <= parts; ++p) cut[p] = std::max(cut[p], cut[p - 1]);
  return cut;
}

// Writes the tallies of consecutive key ranges, in order, as one output.
template <typename K>
int write_out(const std::vector<Tally<K>>& parts, int words, uint64_t* out_keys, uint32_t* cnt,
              uint64_t cap, uint64_t* n_out) {
  uint64_t total = 0;
  for (const Tally<K>& t : parts) total += t.size();
  *n_out = total;
  if (total > cap) return -3;
  uint64_t i = 0;
  for (const Tally<K>& t : parts)
    for (const auto& kc : t) {
      if (kc.second > 0xFFFFFFFFull) return -4;
      for (int w = 0; w < words; ++w) out_keys[i * words + w] = out_word(kc.first, w);
      cnt[i++] = (uint32_t)kc.second;
    }
  return 0;
}

int bad_args(const uint8_t* reads, const uint64_t* off, uint64_t n, int k) {
  if (k < 1 || k > 128 || !off || (n && !reads)) return -1;
  for (uint64_t i = 0; i < n; ++i)
    if (off[i + 1] < off[i]) return -1;
  return 0;
}

// The histogram is tallied per range of top key bits: the ranges are
// disjoint and ascending, so the tallies of the ranges, concatenated in order,
// are the whole histogram. Step 1: each thread decodes the windows of a
// contiguous range of reads and files every key by its top bits. Step 2:
// threads take key ranges one at a time, gather that range's keys from every
// thread, sort them (std::sort) and tally equal neighbours.
template <typename K>
int count_sorted(const uint8_t* reads, const uint64_t* off, uint64_t n, int k, int threads,
                 const Range& range, uint64_t* out_keys, uint32_t* out_cnt, uint64_t cap,
                 uint64_t* n_out) {
  const int nbits = std::min(2 * k, 8);
  const unsigned nb = 1u << nbits;
  const std::vector<uint64_t> cut = read_ranges(off, n, threads);
  std::vector<std::vector<std::vector<K>>> filed(threads, std::vector<std::vector<K>>(nb));
  {
    std::vector<std::thread> ts;
    for (int t = 0; t < threads; ++t)
      ts.emplace_back([&, t] {
        for (uint64_t r = cut[t]; r < cut[t + 1]; ++r)
          for_each_window_key<K>(reads + (off[r] - off[0]), off[r + 1] - off[r], k, range,
                                 [&](const K& key) {
            filed[t][top_of(key, 2 * k, nbits)].push_back(key);
          });
      });
    for (auto& t : ts) t.join();
  }
  std::vector<Tally<K>> parts(nb);
  std::atomic<unsigned> next{0};
  {
    std::vector<std::thread> ts;
    for (int t = 0; t < threads; ++t)
      ts.emplace_back([&] {
        for (unsigned b = next++; b < nb; b = next++) {
          std::vector<K> keys;
          size_t m = 0;
          for (int u = 0; u < threads; ++u) m += filed[u][b].size();
          keys.reserve(m);
          for (int u = 0; u < threads; ++u) {
            keys.insert(keys.end(), filed[u][b].begin(), filed[u][b].end());
            std::vector<K>().swap(filed[u][b]);
          }
          std::sort(keys.begin(), keys.end());
          parts[b] = tally_sorted(keys);
        }
      });
    for (auto& t : ts) t.join();
  }
  return write_out(parts, words_per_key(k), out_keys, out_cnt, cap, n_out);
}

template <typename K>
int count_in_map(const uint8_t* reads, const uint64_t* off, uint64_t n, int k, uint64_t* out_keys,
                 uint32_t* out_cnt, uint64_t cap, uint64_t* n_out) {
  std::map<K, uint64_t> m;  // ordered: its iteration order is the output order
  for (uint64_t r = 0; r < n; ++r)
    for_each_window_key<K>(reads + (off[r] - off[0]), off[r + 1] - off[r], k, Range(),
                           [&](const K& key) { ++m[key]; });
  const std::vector<Tally<K>> all(1, Tally<K>(m.begin(), m.end()));
  return write_out(all, words_per_key(k), out_keys, out_cnt, cap, n_out);
}

template <typename K>
K key_from_words(const uint64_t* w, int words);
template <>
uint64_t key_from_words<uint64_t>(const uint64_t* w, int) {
  return w[0];
}
template <>
u128 key_from_words<u128>(const uint64_t* w, int words) {
  return (u128)w[0] | (words > 1 ? (u128)w[1] << 64 : (u128)0);
}
template <>
Wide key_from_words<Wide>(const uint64_t* w, int) {
  return Wide((u128)w[0] | ((u128)w[1] << 64), (u128)w[2] | ((u128)w[3] << 64));
}

template <typename K>
int count_chosen(const uint8_t* reads, const uint64_t* off, uint64_t n, int k, int threads,
                 const uint64_t* keys, uint64_t nkeys, uint64_t* out_cnt) {
  const int words = words_per_key(k);
  // the chosen keys, sorted, each with its position in the caller's list
  std::vector<std::pair<K, uint64_t>> chosen(nkeys);
  for (uint64_t i = 0; i < nkeys; ++i) chosen[i] = {key_from_words<K>(keys + i * words, words), i};
  std::sort(chosen.begin(), chosen.end());
  const std::vector<uint64_t> cut = read_ranges(off, n, threads);
  std::vector<std::vector<uint64_t>> acc(threads, std::vector<uint64_t>(nkeys, 0));
  std::vector<std::thread> ts;
  for (int t = 0; t < threads; ++t)
    ts.emplace_back([&, t] {
      for (uint64_t r = cut[t]; r < cut[t + 1]; ++r)
        for_each_window_key<K>(reads + (off[r] - off[0]), off[r + 1] - off[r], k, Range(),
                               [&](const K& key) {
          auto it = std::lower_bound(chosen.begin(), chosen.end(), std::make_pair(key, (uint64_t)0));
          // every entry equal to key (the list may hold a key twice)
          for (; it != chosen.end() && it->first == key; ++it) ++acc[t][it->second];
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

// Number of valid windows: positions whose k bytes are all bases.
uint64_t oracle_valid_windows(const uint8_t* reads, const uint64_t* off, uint64_t n, int k) {
  uint64_t w = 0;
  for (uint64_t r = 0; r < n; ++r) {
    const uint8_t* R = reads + (off[r] - off[0]);
    uint64_t run = 0;
    const uint64_t m = off[r + 1] - off[r];
    for (uint64_t i = 0; i < m; ++i) {
      run = kCode.c[R[i]] < 4 ? run + 1 : 0;
      if (run >= (uint64_t)k) ++w;
    }
  }
  return w;
}

// The sorted (k-mer, count) histogram. Key i is written to
// out_keys[i * w .. i * w + w), w = 1 (k <= 32), 2 (k <= 64) or 4 (k <= 128)
// 64-bit words, least significant first. Returns 0, -1 bad arguments, -3
// capacity too small (n_out set), -4 a count above 2^32 - 1.
int oracle_count_sort(const uint8_t* reads, const uint64_t* off, uint64_t n, int k, int threads,
                      uint64_t* out_keys, uint32_t* out_cnt, uint64_t cap, uint64_t* n_out) {
  if (bad_args(reads, off, n, k)) return -1;
  if (threads < 1) threads = 1;
  const Range all;
  if (k <= 32)
    return count_sorted<uint64_t>(reads, off, n, k, threads, all, out_keys, out_cnt, cap, n_out);
  return k <= 64 ? count_sorted<u128>(reads, off, n, k, threads, all, out_keys, out_cnt, cap, n_out)
                 : count_sorted<Wide>(reads, off, n, k, threads, all, out_keys, out_cnt, cap, n_out);
}

// The same histogram restricted to keys whose top `bits` bits (of the 2k-bit
// key; 1 <= bits <= min(2k, 32)) lie in [lo, hi). The slices of a partition
// of [0, 2^bits) concatenate, in order, to the full histogram.
int oracle_count_range(const uint8_t* reads, const uint64_t* off, uint64_t n, int k, int threads,
                       int bits, uint64_t lo, uint64_t hi, uint64_t* out_keys, uint32_t* out_cnt,
                       uint64_t cap, uint64_t* n_out) {
  if (bad_args(reads, off, n, k)) return -1;
  if (bits < 1 || bits > 32 || bits > 2 * k || lo > hi) return -1;
  if (threads < 1) threads = 1;
  Range range;
  range.bits = bits;
  range.lo = lo;
  range.hi = hi;
  if (k <= 32)
    return count_sorted<uint64_t>(reads, off, n, k, threads, range, out_keys, out_cnt, cap, n_out);
  return k <= 64
             ? count_sorted<u128>(reads, off, n, k, threads, range, out_keys, out_cnt, cap, n_out)
             : count_sorted<Wide>(reads, off, n, k, threads, range, out_keys, out_cnt, cap, n_out);
}

// Cross-check counter: an ordered std::map tally instead of sorting.
int oracle_count_map(const uint8_t* reads, const uint64_t* off, uint64_t n, int k,
                     uint64_t* out_keys, uint32_t* out_cnt, uint64_t cap, uint64_t* n_out) {
  if (bad_args(reads, off, n, k)) return -1;
  if (k <= 32) return count_in_map<uint64_t>(reads, off, n, k, out_keys, out_cnt, cap, n_out);
  return k <= 64 ? count_in_map<u128>(reads, off, n, k, out_keys, out_cnt, cap, n_out)
                 : count_in_map<Wide>(reads, off, n, k, out_keys, out_cnt, cap, n_out);
}

// Counts of chosen keys only (for inputs too large to tally in full): every
// valid window's key is looked up among the nkeys requested keys (w words
// each, as written above). out_cnt[i] receives the count of key i (0 if it
// does not occur).
int oracle_count_selected(const uint8_t* reads, const uint64_t* off, uint64_t n, int k, int threads,
                          const uint64_t* keys, uint64_t nkeys, uint64_t* out_cnt) {
  if (bad_args(reads, off, n, k)) return -1;
  if (threads < 1) threads = 1;
  if (k <= 32) return count_chosen<uint64_t>(reads, off, n, k, threads, keys, nkeys, out_cnt);
  return k <= 64 ? count_chosen<u128>(reads, off, n, k, threads, keys, nkeys, out_cnt)
                 : count_chosen<Wide>(reads, off, n, k, threads, keys, nkeys, out_cnt);
}

}  // extern "C"
