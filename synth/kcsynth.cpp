// Seeded synthetic DNA input generator: genomes (uniform ACGT backbone plus
// diverged repeat-family copies) and sequencing reads (random start, random
// strand, substitution errors, N bases). It serves both the CPU oracle and the
// GPU path as an input source only; it contains no k-mer arithmetic.
//
// Randomness: SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
// number generators", OOPSLA 2014) used as a counter-based generator: every
// read r of a call draws from its own stream seeded by mixing (seed, r), so the
// output does not depend on the thread count.
#include <cstdint>
#include <cstring>
#include <cmath>
#include <vector>
#include <thread>
#include <algorithm>

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ULL;

inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

struct Stream {
  uint64_t s;
  Stream(uint64_t seed, uint64_t id) : s(sm_mix(seed ^ sm_mix(id * kGamma + 0x632BE59BD9B4E019ULL))) {}
  inline uint64_t next() { s += kGamma; return sm_mix(s); }
  // uniform integer in [0, n) by multiply-high range reduction (Lemire 2019)
  inline uint64_t below(uint64_t n) { return (uint64_t)(((unsigned __int128)next() * n) >> 64); }
};

inline uint64_t prob_threshold(double p) {
  if (p <= 0.0) return 0;
  if (p >= 1.0) return ~0ULL;
  return (uint64_t)std::ldexp(p, 64);
}

const char kBase[4] = {'A', 'C', 'G', 'T'};

inline char complement_ascii(char c) {
  switch (c) {
    case 'A': return 'T'; case 'C': return 'G'; case 'G': return 'C'; case 'T': return 'A';
    case 'a': return 't'; case 'c': return 'g'; case 'g': return 'c'; case 't': return 'a';
    default: return c;
  }
}

inline int base_index(char c) {
  switch (c) { case 'A': return 0; case 'C': return 1; case 'G': return 2; case 'T': return 3; default: return -1; }
}

void fill_uniform(char* dst, uint64_t n, Stream& st) {
  uint64_t i = 0;
  while (i < n) {
    uint64_t r = st.next();
    for (int j = 0; j < 32 && i < n; ++j, ++i) { dst[i] = kBase[r & 3]; r >>= 2; }
  }
}

// Substitute each base with probability thr/2^64 by one of the other three bases.
inline void mutate(char* s, uint64_t n, uint64_t thr, Stream& st) {
  if (thr == 0) return;
  for (uint64_t i = 0; i < n; ++i) {
    if (st.next() < thr) {
      int b = base_index(s[i]);
      if (b < 0) continue;
      s[i] = kBase[(b + 1 + (int)st.below(3)) & 3];
    }
  }
}

template <class F>
void parallel_for(uint64_t n, int threads, F f) {
  if (threads <= 1 || n < 1024) { for (uint64_t i = 0; i < n; ++i) f(i); return; }
  std::vector<std::thread> ts;
  uint64_t chunk = (n + threads - 1) / threads;
  for (int t = 0; t < threads; ++t) {
    uint64_t a = t * chunk, b = std::min(n, a + chunk);
    if (a >= b) break;
    ts.emplace_back([a, b, &f] { for (uint64_t i = a; i < b; ++i) f(i); });
  }
  for (auto& t : ts) t.join();
}

}  // namespace

extern "C" {

// Length of the genome kcsynth_genome() will produce for this repeat layout.
uint64_t kcsynth_genome_length(uint64_t backbone_len, uint32_t n_families,
                               const uint64_t* family_len, const uint64_t* copies) {
  uint64_t g = backbone_len;
  for (uint32_t f = 0; f < n_families; ++f) g += family_len[f] * copies[f];
  return g;
}

// Genome = uniform ACGT backbone of backbone_len bases with copies[f] diverged
// copies of family f (consensus of family_len[f] uniform bases) inserted at
// uniform backbone positions. Copy c of family f has each base substituted
// with probability divergence[f]. out must hold kcsynth_genome_length() bytes.
void kcsynth_genome(uint64_t seed, uint64_t backbone_len, uint32_t n_families,
                    const uint64_t* family_len, const uint64_t* copies,
                    const double* divergence, char* out) {
  Stream sb(seed, 0xB0B0ULL);
  std::vector<char> backbone(backbone_len);
  fill_uniform(backbone.data(), backbone_len, sb);
  std::vector<std::vector<char>> cons(n_families);
  for (uint32_t f = 0; f < n_families; ++f) {
    Stream sf(seed, 0xFA000000ULL + f);
    cons[f].resize(family_len[f]);
    fill_uniform(cons[f].data(), family_len[f], sf);
  }
  struct Ins { uint64_t pos; uint32_t fam; uint64_t copy; };
  std::vector<Ins> ins;
  Stream sp(seed, 0x9051ULL);
  for (uint32_t f = 0; f < n_families; ++f)
    for (uint64_t c = 0; c < copies[f]; ++c) ins.push_back({sp.below(backbone_len + 1), f, c});
  std::stable_sort(ins.begin(), ins.end(), [](const Ins& a, const Ins& b) { return a.pos < b.pos; });
  uint64_t o = 0, prev = 0;
  for (const Ins& e : ins) {
    std::memcpy(out + o, backbone.data() + prev, e.pos - prev);
    o += e.pos - prev; prev = e.pos;
    uint64_t L = family_len[e.fam];
    std::memcpy(out + o, cons[e.fam].data(), L);
    Stream sc(seed, 0xC0000000000ULL + ((uint64_t)e.fam << 32) + e.copy);
    mutate(out + o, L, prob_threshold(divergence[e.fam]), sc);
    o += L;
  }
  std::memcpy(out + o, backbone.data() + prev, backbone_len - prev);
}

// Reads: read r has length lens[r] (or read_len when lens is NULL) and is
// written at out + offsets[r] - offsets[0]. Each read starts at a uniform
// position of the genome, is reverse-complemented with probability 1/2, then
// each base is substituted with probability err_rate and finally set to 'N'
// with probability n_rate. Reads longer than the genome are clipped to it
// (their remaining bytes are 'N'). Stream ids are stream_base + r.
void kcsynth_reads(uint64_t seed, uint64_t stream_base, const char* genome, uint64_t G,
                   uint64_t n_reads, uint64_t read_len, const uint64_t* lens,
                   const uint64_t* offsets, double err_rate, double n_rate,
                   int threads, char* out) {
  const uint64_t terr = prob_threshold(err_rate), tn = prob_threshold(n_rate);
  const uint64_t base = offsets[0];
  parallel_for(n_reads, threads, [&](uint64_t r) {
    Stream st(seed, stream_base + r);
    uint64_t L = lens ? lens[r] : read_len;
    char* dst = out + (offsets[r] - base);
    uint64_t Lc = std::min(L, G);
    uint64_t start = st.below(G - Lc + 1);
    bool rev = (st.next() >> 63) != 0;
    if (!rev) {
      std::memcpy(dst, genome + start, Lc);
    } else {
      for (uint64_t j = 0; j < Lc; ++j) dst[j] = complement_ascii(genome[start + Lc - 1 - j]);
    }
    for (uint64_t j = Lc; j < L; ++j) dst[j] = 'N';
    mutate(dst, Lc, terr, st);
    if (tn) for (uint64_t j = 0; j < L; ++j) if (st.next() < tn) dst[j] = 'N';
  });
}

// Uniform i.i.d. bytes drawn from an alphabet (used for tiny adversarial inputs).
void kcsynth_random_text(uint64_t seed, uint64_t stream, const char* alphabet, int alpha_len,
                         uint64_t n, char* out) {
  Stream st(seed, stream);
  for (uint64_t i = 0; i < n; ++i) out[i] = alphabet[st.below((uint64_t)alpha_len)];
}

}  // extern "C"
