// Parsing of FASTQ and FASTA text held in device memory into the reads +
// offsets form the counter takes (entry point kc_parse_fastx of include/kc.h).
// The paper leaves input parsing out of its measurements (Section VI); this
// lets a file's bytes be copied to the device as they are and counted there.
//
// Three passes over the text, each HBM-bound (tiles of 16 KiB, 16 bytes per
// thread and round, loads of whole aligned 16-byte chunks):
//   1. per tile: newlines, FASTA header starts, start of the last line;
//      one-block scan over the tiles (sums and a running maximum);
//   2. per tile: bytes kept (sequence-line bytes other than CR/LF) and the
//      FASTQ layout check; scan;
//   3. kept bytes written in order, staged in LDS so that each tile's output
//      (one contiguous run) is written with consecutive stores, and one
//      offset per record.
// Every position a kernel reads is inside [lo, hi) of the trimmed text.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/kc.h"
#include "kc_host.h"

namespace {

typedef unsigned long long ull;

constexpr int kTB = 256;
constexpr int kRounds = 4;
constexpr int kChunk = 16;
constexpr uint64_t kTile = (uint64_t)kTB * kRounds * kChunk;  // 16 KiB

struct Plus {
  __device__ ull operator()(ull a, ull b) const { return a + b; }
};
struct Max {
  __device__ ull operator()(ull a, ull b) const { return a > b ? a : b; }
};
// four 16-bit fields, each its own maximum
struct Max4 {
  __device__ ull operator()(ull a, ull b) const {
    ull r = 0;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const ull x = (a >> (16 * f)) & 0xFFFFu, y = (b >> (16 * f)) & 0xFFFFu;
      r |= (x > y ? x : y) << (16 * f);
    }
    return r;
  }
};

__device__ __forceinline__ uint32_t field(ull v, int f) { return (uint32_t)(v >> (16 * f)) & 0xFFFFu; }

// Exclusive scan over the block (NT threads) in thread order; *total
// receives the reduction of all threads. sh holds NT / 64 values; reusable on
// return.
template <class Op, int NT = kTB>
__device__ ull block_exscan(ull v, Op op, ull* sh, ull* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  ull x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const ull y = __shfl_up(x, (unsigned)d, 64);
    if (lane >= d) x = op(y, x);
  }
  ull ex = __shfl_up(x, 1u, 64);
  if (lane == 0) ex = 0;
  if (lane == 63) sh[w] = x;
  __syncthreads();
  ull before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    if (i < w) before = op(before, sh[i]);
    all = op(all, sh[i]);
  }
  __syncthreads();
  *total = all;
  return op(before, ex);
}

__device__ __forceinline__ uint32_t byte_of(const uint4& v, int j) {
  const uint32_t w = j < 4 ? v.x : j < 8 ? v.y : j < 12 ? v.z : v.w;
  return (w >> (8 * (j & 3))) & 0xFFu;
}

struct Ld {
  uint4 v;
  uint32_t m;
};

// Bytes [pos, pos + 16) of B; bit j of m is set when pos + j lies in
// [lo, hi) (other bytes read as 0). Only whole in-range chunks use the
// 16-byte load.
__device__ __forceinline__ Ld load16(const uint8_t* __restrict__ B, uint64_t pos, uint64_t lo,
                                     uint64_t hi) {
  if (pos >= lo && pos + kChunk <= hi) return Ld{*reinterpret_cast<const uint4*>(B + pos), 0xFFFFu};
  // partial chunk (first or last of the text): byte loads
  ull w0 = 0, w1 = 0;
  uint32_t m = 0;
  for (int j = 0; j < kChunk; ++j) {
    const uint64_t p = pos + j;
    if (p >= lo && p < hi) {
      const ull b = B[p];
      if (j < 8) w0 |= b << (8 * j);
      else w1 |= b << (8 * (j - 8));
      m |= 1u << j;
    }
  }
  return Ld{make_uint4((uint32_t)w0, (uint32_t)(w0 >> 32), (uint32_t)w1, (uint32_t)(w1 >> 32)), m};
}

// 4-bit mask of the zero bytes of x (bit i: byte i). (x & 0x7F..) + 0x7F..
// sets a byte's top bit when its low seven bits are not all zero, without
// carries between bytes; OR-ing x adds its own top bit; the complement keeps
// 0x80 exactly in the zero bytes. The multiply by 2^0 + 2^7 + 2^14 + 2^21
// moves the four flags (bits 0, 8, 16, 24 after the shift) to bits 21..24;
// no two partial products share a bit position.
__device__ __forceinline__ uint32_t zero_bytes4(uint32_t x) {
  const uint32_t t = ~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x | 0x7F7F7F7Fu);
  return (((t >> 7) * 0x00204081u) >> 21) & 0xFu;
}

// Bit j set where byte j equals ch.
__device__ __forceinline__ uint32_t eq_mask(const uint4& v, uint32_t ch) {
  const uint32_t c4 = ch * 0x01010101u;
  return zero_bytes4(v.x ^ c4) | zero_bytes4(v.y ^ c4) << 4 | zero_bytes4(v.z ^ c4) << 8 |
         zero_bytes4(v.w ^ c4) << 12;
}

// The tile's four chunks of this thread (round r: tile bytes
// [(r * kTB + t) * 16, +16)), their validity masks and newline masks.
struct Chunks {
  uint4 v[kRounds];
  uint32_t m[kRounds], nl[kRounds];
};

__device__ __forceinline__ Chunks load_tile(const uint8_t* __restrict__ B, uint64_t tile0,
                                            uint64_t lo, uint64_t hi) {
  Chunks c;
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const uint64_t pos = tile0 + ((uint64_t)r * kTB + threadIdx.x) * kChunk;
    const Ld x = pos < hi ? load16(B, pos, lo, hi) : Ld{make_uint4(0, 0, 0, 0), 0u};
    c.v[r] = x.v;
    c.m[r] = x.m;
  }
#pragma unroll
  for (int r = 0; r < kRounds; ++r) c.nl[r] = eq_mask(c.v[r], '\n') & c.m[r];
  return c;
}

// Local line-start value of a chunk: tile offset of the byte after its last
// newline (1..16384), 0 when it has none.
__device__ __forceinline__ uint32_t last_start(uint32_t nlm, int r) {
  return nlm ? (uint32_t)((r * kTB + threadIdx.x) * kChunk) + (32u - __clz(nlm)) : 0u;
}

__global__ void __launch_bounds__(kTB) k_fx_lines(const uint8_t* __restrict__ B, uint64_t lo,
                                                  uint64_t hi, int fasta, ull* __restrict__ t_nl,
                                                  ull* __restrict__ t_hd, ull* __restrict__ t_ls) {
  __shared__ ull sh[kTB / 64];
  const uint64_t tile0 = (uint64_t)blockIdx.x * kTile;
  const Chunks c = load_tile(B, tile0, lo, hi);
  uint32_t nl = 0, hd = 0, ls = 0;
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    nl += __popc(c.nl[r]);
    const uint32_t s = last_start(c.nl[r], r);
    ls = s > ls ? s : ls;
    if (fasta && c.m[r]) {
      // header starts: '>' at a line start (after a newline, or at lo)
      const uint64_t pos = tile0 + ((uint64_t)r * kTB + threadIdx.x) * kChunk;
      uint32_t starts = (c.nl[r] << 1) & 0xFFFFu;
      if (pos > lo) starts |= B[pos - 1] == '\n' ? 1u : 0u;
      else starts |= 1u << (uint32_t)(lo - pos);
      hd += __popc(starts & eq_mask(c.v[r], '>') & c.m[r]);
    }
  }
  ull tot;
  block_exscan(nl, Plus(), sh, &tot);
  if (threadIdx.x == 0) t_nl[blockIdx.x] = tot;
  if (fasta) {
    block_exscan(hd, Plus(), sh, &tot);
    if (threadIdx.x == 0) t_hd[blockIdx.x] = tot;
  } else if (threadIdx.x == 0) {
    t_hd[blockIdx.x] = 0;
  }
  block_exscan(ls, Max(), sh, &tot);
  if (threadIdx.x == 0) t_ls[blockIdx.x] = tot ? tile0 + tot : 0;
}

// Tile scans in two levels. Level 1 (many blocks): each group of 1024
// consecutive tiles is scanned in place (exclusive, from 0) and its total
// written to g[group]. Level 2 (one block): the group totals are scanned
// (exclusive, from init); g[n_groups] = the reduction of everything. A tile's
// exclusive prefix is then op(g[tile >> 10], t[tile]). Up to three arrays
// per launch; is_max selects the running maximum instead of the sum.
constexpr int kScanGroup = 1024;

struct ScanArrays {
  ull* t[3];
  ull* g[3];
  ull init[3];
  int is_max[3];
  int n;
};

__global__ void __launch_bounds__(kScanGroup) k_fx_scan_groups(ScanArrays s, uint64_t nt) {
  __shared__ ull sh[kScanGroup / 64];
  const uint64_t i = (uint64_t)blockIdx.x * kScanGroup + threadIdx.x;
  for (int a = 0; a < s.n; ++a) {
    const ull v = i < nt ? s.t[a][i] : 0;
    ull total;
    const ull ex = s.is_max[a] ? block_exscan<Max, kScanGroup>(v, Max(), sh, &total)
                               : block_exscan<Plus, kScanGroup>(v, Plus(), sh, &total);
    if (i < nt) s.t[a][i] = ex;
    if (threadIdx.x == 0) s.g[a][blockIdx.x] = total;
  }
}

__global__ void __launch_bounds__(kScanGroup) k_fx_scan_top(ScanArrays s, uint64_t ng) {
  __shared__ ull sh[kScanGroup / 64];
  for (int a = 0; a < s.n; ++a) {
    ull carry = s.init[a];
    for (uint64_t base = 0; base < ng; base += kScanGroup) {
      const uint64_t j = base + threadIdx.x;
      const ull v = j < ng ? s.g[a][j] : 0;
      ull total;
      ull ex;
      if (s.is_max[a]) {
        ex = block_exscan<Max, kScanGroup>(v, Max(), sh, &total);
        ex = ex > carry ? ex : carry;
        carry = total > carry ? total : carry;
      } else {
        ex = carry + block_exscan<Plus, kScanGroup>(v, Plus(), sh, &total);
        carry += total;
      }
      if (j < ng) s.g[a][j] = ex;
    }
    if (threadIdx.x == 0) s.g[a][ng] = carry;
  }
}

// Passes 2 (kWrite = false: kept bytes per tile into t_keep, FASTQ layout
// check into err_line) and 3 (kWrite: t_keep holds each tile's output offset;
// kept bytes and record offsets written). The per-round prefixes of the
// tile's chunks come from one block scan each, the four rounds packed in
// 16-bit fields (a round holds at most 4096 bytes).
template <bool kWrite>
__global__ void __launch_bounds__(kTB) k_fx_seq(const uint8_t* __restrict__ B, uint64_t lo,
                                                uint64_t hi, int fasta,
                                                const ull* __restrict__ t_nl,
                                                const ull* __restrict__ t_hd,
                                                const ull* __restrict__ t_ls,
                                                const ull* __restrict__ g_nl,
                                                const ull* __restrict__ g_hd,
                                                const ull* __restrict__ g_ls,
                                                ull* __restrict__ t_keep,
                                                const ull* __restrict__ g_keep,
                                                ull* __restrict__ err_line,
                                                uint8_t* __restrict__ out_reads,
                                                uint64_t* __restrict__ out_offsets) {
  __shared__ ull sh[kTB / 64];
  __shared__ uint8_t stage[kWrite ? kTile : 1];
  const uint64_t tile0 = (uint64_t)blockIdx.x * kTile;
  const Chunks c = load_tile(B, tile0, lo, hi);
  const uint64_t grp = blockIdx.x / kScanGroup;
  const ull c_nl = g_nl[grp] + t_nl[blockIdx.x];
  const ull c_ls = g_ls[grp] > t_ls[blockIdx.x] ? g_ls[grp] : t_ls[blockIdx.x];

  ull nl4 = 0, ls4 = 0;
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    nl4 |= (ull)__popc(c.nl[r]) << (16 * r);
    ls4 |= (ull)last_start(c.nl[r], r) << (16 * r);
  }
  ull tot_nl4, tot_ls4;
  const ull ex_nl4 = block_exscan(nl4, Plus(), sh, &tot_nl4);
  const ull ex_ls4 = block_exscan(ls4, Max4(), sh, &tot_ls4);

  // per chunk: line index and line start at its first byte, line-start and
  // kept masks
  uint32_t keep[kRounds], starts[kRounds];
  ull line0[kRounds];
  uint32_t nl_before = 0, ls_before = 0;  // earlier rounds of this tile
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const uint64_t pos = tile0 + ((uint64_t)r * kTB + threadIdx.x) * kChunk;
    const ull L = c_nl + nl_before + field(ex_nl4, r);
    const uint32_t lsl = ls_before > field(ex_ls4, r) ? ls_before : field(ex_ls4, r);
    const ull ls0 = lsl ? tile0 + lsl : c_ls;  // <= pos, except lo inside the first chunk
    nl_before += field(tot_nl4, r);
    ls_before = ls_before > field(tot_ls4, r) ? ls_before : field(tot_ls4, r);
    const uint32_t m = c.m[r], nlm = c.nl[r];
    uint32_t st = (nlm << 1) & 0xFFFFu;
    if (ls0 >= pos && ls0 < pos + kChunk) st |= 1u << (uint32_t)(ls0 - pos);
    st &= m;
    const uint32_t crm = eq_mask(c.v[r], '\r');
    uint32_t k = 0;
    if (fasta) {
      // segments between line starts; a segment is kept unless its line is
      // a header
      const uint32_t hdm = st & eq_mask(c.v[r], '>');
      bool hh = m && ls0 < pos && B[ls0] == '>';
      uint32_t from = 0;
      for (uint32_t rest = st;;) {
        const uint32_t to = rest ? (uint32_t)__ffs(rest) - 1 : kChunk;  // next line start
        if (!hh) k |= ((1u << to) - 1) & ~((1u << from) - 1);
        if (!rest) break;
        hh = hdm >> to & 1;
        from = to;
        rest &= rest - 1;
      }
      starts[r] = hdm;
    } else {
      // segments ending at newlines; lines 4i + 1 are kept
      uint32_t l = (uint32_t)L, from = 0;
      for (uint32_t rest = nlm;;) {
        const uint32_t to = rest ? (uint32_t)__ffs(rest) : kChunk;  // one past the newline
        if ((l & 3) == 1) k |= ((1u << to) - 1) & ~((1u << from) - 1);
        if (!rest) break;
        ++l;
        from = to;
        rest &= rest - 1;
      }
      if (!kWrite) {
        // layout check at line starts: '@' on header lines, '+' on separators
        for (uint32_t s = st; s;) {
          const int j = __ffs(s) - 1;
          s &= s - 1;
          const ull lj = L + __popc(nlm & ((1u << j) - 1));
          const uint32_t b = byte_of(c.v[r], j);
          if (((lj & 3) == 0 && b != '@') || ((lj & 3) == 2 && b != '+')) atomicMin(err_line, lj);
        }
      }
      starts[r] = st;
    }
    keep[r] = k & m & ~nlm & ~crm;
    line0[r] = L;
  }

  ull kp4 = 0;
#pragma unroll
  for (int r = 0; r < kRounds; ++r) kp4 |= (ull)__popc(keep[r]) << (16 * r);
  ull tot_kp4;
  const ull ex_kp4 = block_exscan(kp4, Plus(), sh, &tot_kp4);
  uint32_t tile_keep = 0;
#pragma unroll
  for (int r = 0; r < kRounds; ++r) tile_keep += field(tot_kp4, r);
  if (!kWrite) {
    if (threadIdx.x == 0) t_keep[blockIdx.x] = tile_keep;
    return;
  }

  const ull out0 = g_keep[grp] + t_keep[blockIdx.x];
  ull hd_ex4 = 0, tot_hd4 = 0;
  if (fasta) {
    ull hd4 = 0;
#pragma unroll
    for (int r = 0; r < kRounds; ++r) hd4 |= (ull)__popc(starts[r]) << (16 * r);
    hd_ex4 = block_exscan(hd4, Plus(), sh, &tot_hd4);
  }
  uint32_t kp_before = 0, hd_before = 0;
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    uint32_t at = kp_before + field(ex_kp4, r);  // tile-local output position
    kp_before += field(tot_kp4, r);
    const uint32_t km = keep[r];
    // record offsets: FASTA header starts; FASTQ starts of sequence lines
    if (fasta) {
      ull h = g_hd[grp] + t_hd[blockIdx.x] + hd_before + field(hd_ex4, r);
      for (uint32_t s = starts[r]; s;) {
        const int j = __ffs(s) - 1;
        s &= s - 1;
        out_offsets[h++] = out0 + at + __popc(km & ((1u << j) - 1));
      }
      hd_before += field(tot_hd4, r);
    } else {
      for (uint32_t s = starts[r]; s;) {
        const int j = __ffs(s) - 1;
        s &= s - 1;
        const ull lj = line0[r] + __popc(c.nl[r] & ((1u << j) - 1));
        if ((lj & 3) == 1) out_offsets[lj >> 2] = out0 + at + __popc(km & ((1u << j) - 1));
      }
    }
#pragma unroll
    for (int j = 0; j < kChunk; ++j)
      if (km >> j & 1) stage[at++] = (uint8_t)byte_of(c.v[r], j);
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < tile_keep; i += kTB) out_reads[out0 + i] = stage[i];
}

__global__ void k_fx_fill(ull* p, ull v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void k_fx_last(uint64_t* out_offsets, uint64_t n_records, const ull* total) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out_offsets[n_records] = *total;
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

int bad(const std::string& msg) {
  kc::set_last_error(msg);
  return KC_E_INVAL;
}

bool is_eol(uint8_t b) { return b == '\n' || b == '\r'; }

constexpr uint64_t kPeek = 4096;

// First position in [lo, hi) whose byte is not CR/LF, scanning forward
// (dir > 0), or last such position + 1 scanning backward; hi / lo if none.
uint64_t trim(const uint8_t* text, uint64_t lo, uint64_t hi, int dir, hipStream_t st) {
  uint8_t buf[kPeek];
  if (dir > 0) {
    for (uint64_t p = lo; p < hi;) {
      const uint64_t n = hi - p < kPeek ? hi - p : kPeek;
      chk(hipMemcpyAsync(buf, text + p, n, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
      chk(hipStreamSynchronize(st), "hipStreamSynchronize");
      for (uint64_t i = 0; i < n; ++i)
        if (!is_eol(buf[i])) return p + i;
      p += n;
    }
    return hi;
  }
  for (uint64_t e = hi; e > lo;) {
    const uint64_t n = e - lo < kPeek ? e - lo : kPeek;
    chk(hipMemcpyAsync(buf, text + e - n, n, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    chk(hipStreamSynchronize(st), "hipStreamSynchronize");
    for (uint64_t i = n; i > 0; --i)
      if (!is_eol(buf[i - 1])) return e - n + i;
    e -= n;
  }
  return lo;
}

// Trimmed range [*s0, *e0) and its first byte, with one round trip when the
// text's first and last kPeek bytes each hold a byte that is not CR/LF.
void trim_both(const uint8_t* text, uint64_t n, hipStream_t st, uint64_t* s0, uint64_t* e0,
               uint8_t* first) {
  uint8_t head[kPeek], tail[kPeek];
  const uint64_t nh = n < kPeek ? n : kPeek;
  chk(hipMemcpyAsync(head, text, nh, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
  chk(hipMemcpyAsync(tail, text + n - nh, nh, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
  chk(hipStreamSynchronize(st), "hipStreamSynchronize");
  uint64_t s = nh;
  for (uint64_t i = 0; i < nh; ++i)
    if (!is_eol(head[i])) {
      s = i;
      break;
    }
  if (s == nh) s = trim(text, nh, n, 1, st);
  if (s >= n) {
    *s0 = *e0 = n;
    return;
  }
  uint64_t e = 0;
  for (uint64_t i = nh; i > 0; --i)
    if (!is_eol(tail[i - 1])) {
      e = n - nh + i;
      break;
    }
  // a tail of line ends only lies after s (s holds a byte that is not CR/LF)
  if (e == 0) e = trim(text, s, n - nh, -1, st);
  *s0 = s;
  *e0 = e > s ? e : s + 1;  // s holds a byte that is not CR/LF
  if (s < nh) {
    *first = head[s];
  } else {
    chk(hipMemcpyAsync(first, text + s, 1, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    chk(hipStreamSynchronize(st), "hipStreamSynchronize");
  }
}

}  // namespace

extern "C" int kc_parse_fastx(const uint8_t* text, uint64_t n_bytes, int format,
                              uint8_t* out_reads, uint64_t reads_capacity, uint64_t* out_offsets,
                              uint64_t max_records, uint64_t* n_records, uint64_t* n_bases,
                              int* format_out, void* stream) {
  kc::set_last_error("");
  if (!n_records || !n_bases) return bad("n_records or n_bases is NULL");
  *n_records = 0;
  *n_bases = 0;
  if (format_out) *format_out = format;
  if (format < KC_FASTX_AUTO || format > KC_FASTA) return bad("unknown format");
  if (n_bytes && !text) return bad("text is NULL");
  if (!out_offsets) return bad("out_offsets is NULL");
  const hipStream_t st = (hipStream_t)stream;
  void* d = nullptr;
  try {
    uint64_t s0 = 0, e0 = 0;
    uint8_t first = 0;
    if (n_bytes) trim_both(text, n_bytes, st, &s0, &e0, &first);
    if (s0 >= e0) {  // nothing but line ends: no records
      const uint64_t zero = 0;
      chk(hipMemcpyAsync(out_offsets, &zero, 8, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
      chk(hipStreamSynchronize(st), "hipStreamSynchronize");
      return KC_OK;
    }
    if (format == KC_FASTX_AUTO) {
      if (first == '@') format = KC_FASTQ;
      else if (first == '>') format = KC_FASTA;
      else return bad("the text starts with neither '@' (FASTQ) nor '>' (FASTA)");
    }
    if (format_out) *format_out = format;
    if (format == KC_FASTA && first != '>') return bad("FASTA text does not start with '>'");
    const int fasta = format == KC_FASTA;

    // positions relative to the 16-byte aligned base B; the text is [lo, hi)
    const uint64_t a = (uint64_t)(uintptr_t)(text + s0) & 15u;
    const uint8_t* B = text + s0 - a;
    const uint64_t lo = a, hi = a + (e0 - s0);
    const uint64_t nt = (hi + kTile - 1) / kTile;
    if (nt > 0x7fffffffull) return bad("text too large");
    const uint64_t ng = (nt + kScanGroup - 1) / kScanGroup;
    chk(hipMallocAsync(&d, (4 * nt + 4 * (ng + 1) + 1) * sizeof(ull), st), "hipMallocAsync");
    ull* t_nl = (ull*)d;
    ull* t_hd = t_nl + nt;
    ull* t_ls = t_hd + nt;
    ull* t_keep = t_ls + nt;
    ull* g_nl = t_keep + nt;
    ull* g_hd = g_nl + (ng + 1);
    ull* g_ls = g_hd + (ng + 1);
    ull* g_keep = g_ls + (ng + 1);
    ull* err = g_keep + (ng + 1);
    ScanArrays sa3 = {{t_nl, t_hd, t_ls}, {g_nl, g_hd, g_ls}, {0, 0, (ull)lo}, {0, 0, 1}, 3};
    ScanArrays sa1 = {{t_keep, nullptr, nullptr}, {g_keep, nullptr, nullptr}, {0, 0, 0},
                      {0, 0, 0}, 1};
    hipLaunchKernelGGL(k_fx_fill, dim3(1), dim3(64), 0, st, err, ~0ull);
    hipLaunchKernelGGL(k_fx_lines, dim3((unsigned)nt), dim3(kTB), 0, st, B, lo, hi, fasta, t_nl,
                       t_hd, t_ls);
    hipLaunchKernelGGL(k_fx_scan_groups, dim3((unsigned)ng), dim3(kScanGroup), 0, st, sa3, nt);
    hipLaunchKernelGGL(k_fx_scan_top, dim3(1), dim3(kScanGroup), 0, st, sa3, ng);
    chk(hipGetLastError(), "parse launch");
    ull tot[2] = {0, 0};
    chk(hipMemcpyAsync(&tot[0], g_nl + ng, 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    chk(hipMemcpyAsync(&tot[1], g_hd + ng, 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    chk(hipStreamSynchronize(st), "hipStreamSynchronize");
    const uint64_t lines = tot[0] + 1;  // the trimmed text does not end with a newline
    if (!fasta && lines % 4) {
      chk(hipFreeAsync(d, st), "hipFreeAsync");
      d = nullptr;
      return bad("FASTQ text has " + std::to_string(lines) +
                 " lines, not a whole number of 4-line records");
    }
    const uint64_t R = fasta ? tot[1] : lines / 4;
    *n_records = R;
    if (R > max_records) {
      chk(hipFreeAsync(d, st), "hipFreeAsync");
      d = nullptr;
      chk(hipStreamSynchronize(st), "hipStreamSynchronize");
      kc::set_last_error("out_offsets has room for " + std::to_string(max_records) +
                         " records, the text holds " + std::to_string(R));
      return KC_E_CAPACITY;
    }
    hipLaunchKernelGGL(k_fx_seq<false>, dim3((unsigned)nt), dim3(kTB), 0, st, B, lo, hi, fasta,
                       t_nl, t_hd, t_ls, g_nl, g_hd, g_ls, t_keep, g_keep, err, nullptr, nullptr);
    hipLaunchKernelGGL(k_fx_scan_groups, dim3((unsigned)ng), dim3(kScanGroup), 0, st, sa1, nt);
    hipLaunchKernelGGL(k_fx_scan_top, dim3(1), dim3(kScanGroup), 0, st, sa1, ng);
    chk(hipGetLastError(), "parse launch");
    // the kept bytes are at most hi - lo: with that much room the write pass
    // follows at once and the checks are read after it
    const bool room = out_reads && reads_capacity >= hi - lo;
    ull res[2] = {0, ~0ull};  // kept bytes, first malformed FASTQ line (none: all ones)
    if (!room) {
      chk(hipMemcpyAsync(&res[0], g_keep + ng, 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
      chk(hipMemcpyAsync(&res[1], err, 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
      chk(hipStreamSynchronize(st), "hipStreamSynchronize");
      if (res[1] == ~0ull && res[0] > reads_capacity) {
        *n_bases = res[0];
        chk(hipFreeAsync(d, st), "hipFreeAsync");
        d = nullptr;
        chk(hipStreamSynchronize(st), "hipStreamSynchronize");
        kc::set_last_error("out_reads has room for " + std::to_string(reads_capacity) +
                           " bytes, the sequences hold " + std::to_string(res[0]));
        return KC_E_CAPACITY;
      }
      if (res[1] == ~0ull && res[0] && !out_reads) {
        chk(hipFreeAsync(d, st), "hipFreeAsync");
        d = nullptr;
        return bad("out_reads is NULL");
      }
    }
    if (res[1] == ~0ull) {
      hipLaunchKernelGGL(k_fx_seq<true>, dim3((unsigned)nt), dim3(kTB), 0, st, B, lo, hi, fasta,
                         t_nl, t_hd, t_ls, g_nl, g_hd, g_ls, t_keep, g_keep, err, out_reads,
                         out_offsets);
      hipLaunchKernelGGL(k_fx_last, dim3(1), dim3(64), 0, st, out_offsets, R, g_keep + ng);
      chk(hipGetLastError(), "parse launch");
    }
    if (room) {
      chk(hipMemcpyAsync(&res[0], g_keep + ng, 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
      chk(hipMemcpyAsync(&res[1], err, 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    }
    chk(hipFreeAsync(d, st), "hipFreeAsync");
    d = nullptr;
    chk(hipStreamSynchronize(st), "hipStreamSynchronize");
    if (res[1] != ~0ull) {
      *n_records = 0;
      const uint64_t l = res[1];
      return bad("FASTQ line " + std::to_string(l) + " (counting from 0) should start with '" +
                 ((l & 3) == 0 ? "@" : "+") + "'");
    }
    *n_bases = res[0];
  } catch (const Fail& f) {
    if (d) (void)hipFreeAsync(d, st);
    return f.code;
  }
  return KC_OK;
}
