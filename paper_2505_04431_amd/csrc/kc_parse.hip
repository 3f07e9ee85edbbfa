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

// Exclusive scan over the block in thread order; *total receives the
// reduction of all threads. sh holds kTB / 64 values; reusable on return.
template <class Op>
__device__ ull block_exscan(ull v, Op op, ull* sh, ull* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  ull x = v;
  for (int d = 1; d < 64; d <<= 1) {
    const ull y = __shfl_up(x, (unsigned)d, 64);
    if (lane >= d) x = op(y, x);
  }
  ull ex = __shfl_up(x, 1u, 64);
  if (lane == 0) ex = 0;
  if (lane == 63) sh[w] = x;
  __syncthreads();
  ull before = 0, all = 0;
  for (int i = 0; i < kTB / 64; ++i) {
    if (i < w) before = op(before, sh[i]);
    all = op(all, sh[i]);
  }
  __syncthreads();
  *total = all;
  return op(before, ex);
}

// Bytes [pos, pos + 16) of B; bit j of the result is set when pos + j lies in
// [lo, hi). Only whole in-range chunks use the 16-byte load.
__device__ __forceinline__ uint32_t load_chunk(const uint8_t* __restrict__ B, uint64_t pos,
                                               uint64_t lo, uint64_t hi, uint8_t (&c)[kChunk]) {
  if (pos >= lo && pos + kChunk <= hi) {
    const uint4 v = *reinterpret_cast<const uint4*>(B + pos);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int j = 0; j < kChunk; ++j) c[j] = (uint8_t)(w[j >> 2] >> (8 * (j & 3)));
    return 0xFFFFu;
  }
  uint32_t m = 0;
#pragma unroll
  for (int j = 0; j < kChunk; ++j) {
    const uint64_t p = pos + j;
    const bool ok = p >= lo && p < hi;
    c[j] = ok ? B[p] : 0;
    m |= (uint32_t)ok << j;
  }
  return m;
}

// Per-chunk summary: newlines, header starts ('>' at a line start), and the
// start of the last line begun in the chunk (position after its last
// newline; 0 = none). prev is the byte before the chunk ('\n' at lo).
__device__ __forceinline__ void chunk_lines(const uint8_t (&c)[kChunk], uint32_t m, uint64_t pos,
                                            uint8_t prev, uint32_t* nl, uint32_t* hd, ull* ls) {
  uint32_t a = 0, h = 0;
  ull s = 0;
#pragma unroll
  for (int j = 0; j < kChunk; ++j) {
    if (m >> j & 1) {
      h += (c[j] == '>' && prev == '\n') ? 1u : 0u;
      if (c[j] == '\n') {
        ++a;
        s = pos + j + 1;
      }
      prev = c[j];
    } else {
      prev = '\n';
    }
  }
  *nl = a;
  *hd = h;
  *ls = s;
}

__device__ __forceinline__ uint8_t byte_before(const uint8_t* __restrict__ B, uint64_t pos,
                                               uint64_t lo) {
  return pos > lo ? B[pos - 1] : (uint8_t)'\n';
}

__global__ void __launch_bounds__(kTB) k_fx_lines(const uint8_t* __restrict__ B, uint64_t lo,
                                                  uint64_t hi, ull* __restrict__ t_nl,
                                                  ull* __restrict__ t_hd, ull* __restrict__ t_ls) {
  __shared__ ull sh[kTB / 64];
  const uint64_t tile0 = (uint64_t)blockIdx.x * kTile;
  ull nl = 0, hd = 0, ls = 0;
  for (int r = 0; r < kRounds; ++r) {
    const uint64_t pos = tile0 + ((uint64_t)r * kTB + threadIdx.x) * kChunk;
    if (pos >= hi) break;
    uint8_t c[kChunk];
    const uint32_t m = load_chunk(B, pos, lo, hi, c);
    uint32_t a, h;
    ull s;
    chunk_lines(c, m, pos, byte_before(B, pos, lo), &a, &h, &s);
    nl += a;
    hd += h;
    ls = s > ls ? s : ls;
  }
  ull tot;
  block_exscan(nl, Plus(), sh, &tot);
  if (threadIdx.x == 0) t_nl[blockIdx.x] = tot;
  block_exscan(hd, Plus(), sh, &tot);
  if (threadIdx.x == 0) t_hd[blockIdx.x] = tot;
  block_exscan(ls, Max(), sh, &tot);
  if (threadIdx.x == 0) t_ls[blockIdx.x] = tot;
}

// Exclusive scan of nt tile values in place (one block); t[nt] = reduction.
// init is the value before the first tile (0 for sums, lo for line starts).
template <class Op>
__global__ void __launch_bounds__(1024) k_fx_scan(ull* __restrict__ t, uint64_t nt, ull init,
                                                  Op op) {
  __shared__ ull part[1024];
  const uint64_t per = (nt + 1023) / 1024;
  const uint64_t b = threadIdx.x * per, e = b + per < nt ? b + per : nt;
  ull s = 0;
  for (uint64_t i = b; i < e; ++i) s = op(s, t[i]);
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    ull run = init;
    for (int i = 0; i < 1024; ++i) {
      const ull x = part[i];
      part[i] = run;
      run = op(run, x);
    }
    t[nt] = run;
  }
  __syncthreads();
  ull run = part[threadIdx.x];
  for (uint64_t i = b; i < e; ++i) {
    const ull x = t[i];
    t[i] = run;
    run = op(run, x);
  }
}

// Passes 2 (kWrite = false: kept bytes per tile into t_keep, FASTQ layout
// check into err_line) and 3 (kWrite: t_keep holds each tile's output offset;
// kept bytes and record offsets written).
template <bool kWrite>
__global__ void __launch_bounds__(kTB) k_fx_seq(const uint8_t* __restrict__ B, uint64_t lo,
                                                uint64_t hi, int fasta,
                                                const ull* __restrict__ t_nl,
                                                const ull* __restrict__ t_hd,
                                                const ull* __restrict__ t_ls,
                                                ull* __restrict__ t_keep, ull* __restrict__ err_line,
                                                uint8_t* __restrict__ out_reads,
                                                uint64_t* __restrict__ out_offsets) {
  __shared__ ull sh[kTB / 64];
  __shared__ uint8_t stage[kWrite ? kTile : 1];
  const uint64_t tile0 = (uint64_t)blockIdx.x * kTile;
  ull c_nl = t_nl[blockIdx.x], c_hd = t_hd[blockIdx.x], c_ls = t_ls[blockIdx.x];
  const ull out0 = kWrite ? t_keep[blockIdx.x] : 0;
  ull c_keep = 0;  // kept bytes of this tile before the current round
  for (int r = 0; r < kRounds; ++r) {
    const uint64_t pos = tile0 + ((uint64_t)r * kTB + threadIdx.x) * kChunk;
    uint8_t c[kChunk];
    uint32_t m = 0;
    if (pos < hi) m = load_chunk(B, pos, lo, hi, c);
    else
      for (int j = 0; j < kChunk; ++j) c[j] = 0;
    uint32_t a = 0, h = 0;
    ull s = 0;
    if (m) chunk_lines(c, m, pos, byte_before(B, pos, lo), &a, &h, &s);
    ull tot_nl, tot_hd, tot_ls, tot_keep;
    ull L = c_nl + block_exscan(a, Plus(), sh, &tot_nl);
    const ull hd0 = c_hd + block_exscan(h, Plus(), sh, &tot_hd);
    const ull ls_ex = block_exscan(s, Max(), sh, &tot_ls);
    const ull ls0 = ls_ex > c_ls ? ls_ex : c_ls;
    // state at the chunk's first byte: line index L, line start ls0 (<= pos)
    bool hdr = false;
    if (fasta && m && ls0 < pos) hdr = B[ls0] == '>';
    uint32_t keep = 0;
    {
      ull ls = ls0, l = L;
      bool hh = hdr;
      for (int j = 0; j < kChunk; ++j) {
        if (!(m >> j & 1)) continue;
        const uint64_t p = pos + j;
        if (p == ls) {
          if (fasta) {
            hh = c[j] == '>';
          } else if (!kWrite) {
            const int type = (int)(l & 3);
            if ((type == 0 && c[j] != '@') || (type == 2 && c[j] != '+')) atomicMin(err_line, l);
          }
        }
        const bool kept = c[j] != '\n' && c[j] != '\r' && (fasta ? !hh : (l & 3) == 1);
        keep |= (uint32_t)kept << j;
        if (c[j] == '\n') {
          ++l;
          ls = p + 1;
        }
      }
    }
    const ull before = block_exscan((ull)__popc(keep), Plus(), sh, &tot_keep);
    if (kWrite) {
      // kept bytes into the tile's staging area; record offsets
      uint32_t at = (uint32_t)(c_keep + before);
      ull ls = ls0, l = L, hd = hd0;
      for (int j = 0; j < kChunk; ++j) {
        if (!(m >> j & 1)) continue;
        const uint64_t p = pos + j;
        if (p == ls) {
          if (fasta) {
            if (c[j] == '>') out_offsets[hd++] = out0 + at;
          } else if ((l & 3) == 1) {
            out_offsets[l >> 2] = out0 + at;
          }
        }
        if (keep >> j & 1) stage[at++] = c[j];
        if (c[j] == '\n') {
          ++l;
          ls = p + 1;
        }
      }
    }
    c_nl += tot_nl;
    c_hd += tot_hd;
    c_ls = tot_ls > c_ls ? tot_ls : c_ls;
    c_keep += tot_keep;
  }
  if (!kWrite) {
    if (threadIdx.x == 0) t_keep[blockIdx.x] = c_keep;
  } else {
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < (uint32_t)c_keep; i += kTB) out_reads[out0 + i] = stage[i];
  }
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

// First position in [lo, hi) whose byte is not CR/LF, scanning forward
// (dir > 0) or last such position + 1 scanning backward; lo / hi if none.
uint64_t trim(const uint8_t* text, uint64_t lo, uint64_t hi, int dir, hipStream_t st) {
  uint8_t buf[4096];
  if (dir > 0) {
    for (uint64_t p = lo; p < hi;) {
      const uint64_t n = hi - p < sizeof buf ? hi - p : sizeof buf;
      chk(hipMemcpyAsync(buf, text + p, n, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
      chk(hipStreamSynchronize(st), "hipStreamSynchronize");
      for (uint64_t i = 0; i < n; ++i)
        if (!is_eol(buf[i])) return p + i;
      p += n;
    }
    return hi;
  }
  for (uint64_t e = hi; e > lo;) {
    const uint64_t n = e - lo < sizeof buf ? e - lo : sizeof buf;
    chk(hipMemcpyAsync(buf, text + e - n, n, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    chk(hipStreamSynchronize(st), "hipStreamSynchronize");
    for (uint64_t i = n; i > 0; --i)
      if (!is_eol(buf[i - 1])) return e - n + i;
    e -= n;
  }
  return lo;
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
    const uint64_t s0 = n_bytes ? trim(text, 0, n_bytes, 1, st) : 0;
    const uint64_t e0 = s0 < n_bytes ? trim(text, s0, n_bytes, -1, st) : s0;
    if (s0 >= e0) {  // nothing but line ends: no records
      const uint64_t zero = 0;
      chk(hipMemcpyAsync(out_offsets, &zero, 8, hipMemcpyHostToDevice, st), "hipMemcpyAsync");
      chk(hipStreamSynchronize(st), "hipStreamSynchronize");
      return KC_OK;
    }
    uint8_t first = 0;
    chk(hipMemcpyAsync(&first, text + s0, 1, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    chk(hipStreamSynchronize(st), "hipStreamSynchronize");
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
    chk(hipMallocAsync(&d, (4 * (nt + 1) + 2) * sizeof(ull), st), "hipMallocAsync");
    ull* t_nl = (ull*)d;
    ull* t_hd = t_nl + (nt + 1);
    ull* t_ls = t_hd + (nt + 1);
    ull* t_keep = t_ls + (nt + 1);
    ull* err = t_keep + (nt + 1);
    hipLaunchKernelGGL(k_fx_fill, dim3(1), dim3(64), 0, st, err, ~0ull);
    hipLaunchKernelGGL(k_fx_lines, dim3((unsigned)nt), dim3(kTB), 0, st, B, lo, hi, t_nl, t_hd,
                       t_ls);
    hipLaunchKernelGGL(k_fx_scan<Plus>, dim3(1), dim3(1024), 0, st, t_nl, nt, 0ull, Plus());
    hipLaunchKernelGGL(k_fx_scan<Plus>, dim3(1), dim3(1024), 0, st, t_hd, nt, 0ull, Plus());
    hipLaunchKernelGGL(k_fx_scan<Max>, dim3(1), dim3(1024), 0, st, t_ls, nt, (ull)lo, Max());
    chk(hipGetLastError(), "parse launch");
    ull tot[2] = {0, 0};
    chk(hipMemcpyAsync(&tot[0], t_nl + nt, 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    chk(hipMemcpyAsync(&tot[1], t_hd + nt, 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
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
                       t_nl, t_hd, t_ls, t_keep, err, nullptr, nullptr);
    hipLaunchKernelGGL(k_fx_scan<Plus>, dim3(1), dim3(1024), 0, st, t_keep, nt, 0ull, Plus());
    chk(hipGetLastError(), "parse launch");
    ull chk2[2] = {0, 0};
    chk(hipMemcpyAsync(&chk2[0], t_keep + nt, 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    chk(hipMemcpyAsync(&chk2[1], err, 8, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    chk(hipStreamSynchronize(st), "hipStreamSynchronize");
    if (chk2[1] != ~0ull) {
      chk(hipFreeAsync(d, st), "hipFreeAsync");
      d = nullptr;
      const uint64_t l = chk2[1];
      return bad("FASTQ line " + std::to_string(l) + " (counting from 0) should start with '" +
                 ((l & 3) == 0 ? "@" : "+") + "'");
    }
    *n_bases = chk2[0];
    if (chk2[0] > reads_capacity) {
      chk(hipFreeAsync(d, st), "hipFreeAsync");
      d = nullptr;
      chk(hipStreamSynchronize(st), "hipStreamSynchronize");
      kc::set_last_error("out_reads has room for " + std::to_string(reads_capacity) +
                         " bytes, the sequences hold " + std::to_string(chk2[0]));
      return KC_E_CAPACITY;
    }
    if (chk2[0] && !out_reads) {
      chk(hipFreeAsync(d, st), "hipFreeAsync");
      d = nullptr;
      return bad("out_reads is NULL");
    }
    hipLaunchKernelGGL(k_fx_seq<true>, dim3((unsigned)nt), dim3(kTB), 0, st, B, lo, hi, fasta,
                       t_nl, t_hd, t_ls, t_keep, err, out_reads, out_offsets);
    hipLaunchKernelGGL(k_fx_last, dim3(1), dim3(64), 0, st, out_offsets, R, t_keep + nt);
    chk(hipGetLastError(), "parse launch");
    chk(hipFreeAsync(d, st), "hipFreeAsync");
    d = nullptr;
    chk(hipStreamSynchronize(st), "hipStreamSynchronize");
  } catch (const Fail& f) {
    if (d) (void)hipFreeAsync(d, st);
    return f.code;
  }
  return KC_OK;
}
