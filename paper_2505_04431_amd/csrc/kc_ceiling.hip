// Measured ceilings for the counting path (entry point kc_measure_ceilings of
// include/kc_bench.h): the rates its kernels are judged against, taken on the
// device at hand instead of quoted from a data sheet.
//   copy        streaming read + write (GB/s moved)
//   hbm insert  random open-addressing inserts (64-bit CAS of the key, 32-bit
//               add of the count) into a table far larger than the caches
//   mall insert the same into a table that fits the on-package cache
//   lds insert  the same into per-workgroup LDS tables
// All indices are masked into their arrays; every probe loop is bounded.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/kc.h"
#include "../../include/kc_bench.h"
#include "kc_host.h"

namespace {

__device__ __forceinline__ uint64_t mix(uint64_t z) {  // SplitMix64 output function
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_copy(const uint4* __restrict__ a, uint4* __restrict__ b, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) b[i] = a[i];
}

__global__ void k_clear(unsigned long long* keys, uint32_t* cnt, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    keys[i] = ~0ull;
    cnt[i] = 0;
  }
}

// n_ops inserts of keys drawn from n_keys distinct values (each repeated
// n_ops / n_keys times) into a table of mask+1 slots (load 1/2).
__global__ void k_insert(unsigned long long* __restrict__ keys, uint32_t* __restrict__ cnt,
                         uint64_t mask, uint64_t n_ops, uint64_t n_keys, uint32_t* lost) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_ops; i += stride) {
    const unsigned long long key = mix(i % n_keys) >> 2;
    uint64_t pos = mix(key ^ 0x5bd1e995ull) & mask;
    bool done = false;
    for (int probe = 0; probe < 256 && !done; ++probe) {
      const unsigned long long prev = atomicCAS(&keys[pos], ~0ull, key);
      if (prev == ~0ull || prev == key) {
        atomicAdd(&cnt[pos], 1u);
        done = true;
      }
      pos = (pos + 1) & mask;
    }
    if (!done) atomicAdd(lost, 1u);
  }
}

constexpr int kLdsSlots = 4096;

__global__ void __launch_bounds__(512) k_lds_insert(uint64_t ops_per_block, uint32_t* lost) {
  __shared__ unsigned long long tk[kLdsSlots];
  __shared__ uint32_t tc[kLdsSlots];
  for (int j = threadIdx.x; j < kLdsSlots; j += blockDim.x) {
    tk[j] = ~0ull;
    tc[j] = 0;
  }
  __syncthreads();
  uint32_t miss = 0;
  for (uint64_t i = threadIdx.x; i < ops_per_block; i += blockDim.x) {
    // 2048 distinct keys per block: the load of the paper path's large tables
    const unsigned long long key = mix(blockIdx.x * 2048ull + (i & 2047)) >> 2;
    uint32_t pos = (uint32_t)mix(key) & (kLdsSlots - 1);
    bool done = false;
    for (int probe = 0; probe < kLdsSlots && !done; ++probe) {
      const unsigned long long prev = atomicCAS(&tk[pos], ~0ull, key);
      if (prev == ~0ull || prev == key) {
        atomicAdd(&tc[pos], 1u);
        done = true;
      }
      pos = (pos + 1) & (kLdsSlots - 1);
    }
    miss += !done;
  }
  __syncthreads();
  uint32_t s = 0;
  for (int j = threadIdx.x; j < kLdsSlots; j += blockDim.x) s += tc[j];
  // the table must hold every insert: a shortfall is reported as lost
  __shared__ uint32_t total;
  if (threadIdx.x == 0) total = 0;
  __syncthreads();
  atomicAdd(&total, s);
  __syncthreads();
  if (threadIdx.x == 0 && (total != ops_per_block || miss)) atomicAdd(lost, 1u);
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

struct Mem {
  void* p = nullptr;
  ~Mem() {
    if (p) (void)hipFree(p);
  }
};

template <class Launch>
double time_ms(hipStream_t st, hipEvent_t a, hipEvent_t b, int reps, Launch&& launch) {
  launch();  // warm-up
  chk(hipEventRecord(a, st), "hipEventRecord");
  for (int r = 0; r < reps; ++r) launch();
  chk(hipEventRecord(b, st), "hipEventRecord");
  chk(hipEventSynchronize(b), "hipEventSynchronize");
  float ms = 0;
  chk(hipEventElapsedTime(&ms, a, b), "hipEventElapsedTime");
  return ms / reps;
}

}  // namespace

extern "C" int kc_measure_ceilings(uint64_t table_bytes, kc_ceilings* out, void* stream) {
  kc::set_last_error("");
  if (!out) return KC_E_INVAL;
  if (table_bytes < (64ull << 20)) return KC_E_INVAL;
  const hipStream_t st = (hipStream_t)stream;
  hipEvent_t a = nullptr, b = nullptr;
  try {
    chk(hipEventCreate(&a), "hipEventCreate");
    chk(hipEventCreate(&b), "hipEventCreate");
    // one allocation: the copy uses it as two halves, the tables as keys + counts
    Mem m;
    chk(hipMalloc(&m.p, table_bytes), "hipMalloc");
    Mem lost;
    chk(hipMalloc(&lost.p, 4), "hipMalloc");
    uint32_t* d_lost = (uint32_t*)lost.p;
    chk(hipMemsetAsync(d_lost, 0, 4, st), "hipMemsetAsync");

    const uint64_t half = (table_bytes / 2) & ~(uint64_t)15;
    const uint64_t n16 = half / 16;
    const double copy_ms = time_ms(st, a, b, 5, [&] {
      hipLaunchKernelGGL(k_copy, dim3(8192), dim3(256), 0, st, (const uint4*)m.p,
                         (uint4*)((char*)m.p + half), n16);
    });
    out->copy_gbs = 2.0 * (double)half / (copy_ms * 1e6);

    // tables: slots of 8 + 4 bytes; largest power of two that fits
    uint64_t slots = 1;
    while (slots * 2 * 12 <= table_bytes) slots *= 2;
    auto insert_rate = [&](uint64_t S) {
      unsigned long long* keys = (unsigned long long*)m.p;
      uint32_t* cnt = (uint32_t*)((char*)m.p + S * 8);
      const uint64_t ops = 1ull << 26;
      return time_ms(st, a, b, 3, [&] {
        hipLaunchKernelGGL(k_clear, dim3(4096), dim3(256), 0, st, keys, cnt, S);
        hipLaunchKernelGGL(k_insert, dim3(8192), dim3(256), 0, st, keys, cnt, S - 1, ops, S / 2,
                           d_lost);
      });
    };
    // subtract the clear (timed alone) from clear + insert
    auto clear_ms = [&](uint64_t S) {
      unsigned long long* keys = (unsigned long long*)m.p;
      uint32_t* cnt = (uint32_t*)((char*)m.p + S * 8);
      return time_ms(st, a, b, 3, [&] {
        hipLaunchKernelGGL(k_clear, dim3(4096), dim3(256), 0, st, keys, cnt, S);
      });
    };
    const double ops = (double)(1ull << 26);
    const uint64_t s_big = slots, s_small = 1ull << 20;  // 12 MiB: inside the 256 MB cache
    out->hbm_table_bytes = s_big * 12;
    out->hbm_insert_gops = ops / ((insert_rate(s_big) - clear_ms(s_big)) * 1e6);
    out->mall_table_bytes = s_small * 12;
    out->mall_insert_gops = ops / ((insert_rate(s_small) - clear_ms(s_small)) * 1e6);

    const int blocks = 4096;
    const uint64_t per_block = 1ull << 16;
    const double lds_ms = time_ms(st, a, b, 3, [&] {
      hipLaunchKernelGGL(k_lds_insert, dim3(blocks), dim3(512), 0, st, per_block, d_lost);
    });
    out->lds_insert_gops = (double)blocks * (double)per_block / (lds_ms * 1e6);
    uint32_t h_lost = 0;
    chk(hipMemcpyAsync(&h_lost, d_lost, 4, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
    chk(hipStreamSynchronize(st), "hipStreamSynchronize");
    out->lost = h_lost;
  } catch (const Fail& f) {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    return f.code;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return out->lost ? KC_E_INTERNAL : KC_OK;
}
