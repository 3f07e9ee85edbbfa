/*
 * kc_bench.h — measured ceilings for the k-mer counting path on one MI355X.
 *
 * The counting path (kc.h) is bound by HBM traffic and by hash-table atomics
 * (Section V of the paper models the same two costs for a CPU node:
 * intranode memory traffic and integer work). This call measures, on the
 * current device, the rates those kernels are judged against:
 *   copy_gbs          streaming copy, bytes read + written per second (GB/s)
 *   hbm_insert_gops   random open-addressing inserts (64-bit CAS claim of the
 *                     key, 32-bit atomic add of the count) into a table of
 *                     hbm_table_bytes, far larger than the caches (G inserts/s)
 *   mall_insert_gops  the same into a table of mall_table_bytes (12 MiB)
 *   lds_insert_gops   the same into 4096-slot tables in LDS, one per workgroup
 *   lost              inserts that found no slot (0 unless something is wrong)
 *
 * table_bytes: device memory to use (>= 64 MiB; the copy moves half of it
 * each way, the large table takes all of it). Allocates and frees it, so it
 * must not run inside graph capture. stream: hipStream_t as void* (NULL =
 * default). Returns KC_OK, KC_E_INVAL, KC_E_NOMEM, KC_E_DEVICE, or
 * KC_E_INTERNAL if lost != 0.
 */
#ifndef KC_BENCH_H
#define KC_BENCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kc_ceilings {
  double copy_gbs;
  double hbm_insert_gops;
  double mall_insert_gops;
  double lds_insert_gops;
  uint64_t hbm_table_bytes;
  uint64_t mall_table_bytes;
  uint64_t lost;
} kc_ceilings;

int kc_measure_ceilings(uint64_t table_bytes, kc_ceilings* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* KC_BENCH_H */
