/*
 * kc.h — canonical k-mer counting on one MI355X (gfx950): the C ABI.
 *
 * What is computed (the k-mer histogram of Section II, counted as in
 * Algorithm 1 "Serial Algorithm" and Algorithm 3 "FA-BSP Algorithm"):
 *   - read i is the byte range reads[offsets[i] .. offsets[i+1]);
 *   - a window is k consecutive bytes of one read; it is valid iff every byte
 *     is A/C/G/T (either case); windows touching any other byte ('N', IUPAC
 *     codes, ...) are skipped;
 *   - bases are coded A=0, C=1, G=2, T=3 with the first base most
 *     significant (as Algorithm 1 builds a k-mer), masked to 2k bits;
 *   - the counted key is the canonical k-mer min(kmer, reverse complement)
 *     as an unsigned 2k-bit integer;
 *   - the result is every distinct key with its number of valid windows,
 *     sorted by key ascending (the result of Algorithm 1),
 *     from count 1 up (Section VI counts from 1 to the maximum).
 * The P owner partitions stand in for the paper's P processing elements
 * and their owner function (Algorithms 2-4); the result does not depend on P.
 *
 * Conventions
 *   - All array arguments of kc_count / kc_count_ex are DEVICE pointers
 *     (memory from hipMalloc, or a torch CUDA tensor's data pointer) unless
 *     named host_*. n_out is a host pointer.
 *   - Keys: k <= 32 -> one uint64 per key (key in the low 2k bits);
 *           33 <= k <= 64 -> two uint64 per key, low word first (lo, hi);
 *           65 <= k <= 128 -> four uint64 per key, least significant first
 *           (keys wider than 64 bits, named future work in Section VII).
 *   - The caller owns inputs and outputs. The library owns its scratch memory
 *     (a per-host-thread, per-device arena kept between calls) and keeps no
 *     caller pointer after a call returns.
 *   - Calls are synchronous with respect to the host: when they return, the
 *     outputs are complete. Work is issued on `stream` (NULL = the legacy
 *     default stream).
 *   - No C++ exception crosses this boundary. On error, the outputs are
 *     unspecified except *n_out for KC_E_CAPACITY; kc_last_error() gives a
 *     message (per host thread).
 */
#ifndef KC_H
#define KC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define KC_OK 0
#define KC_E_INVAL (-1)    /* bad argument: NULL pointer, k outside [1,128], P < 1,
                              offsets decreasing */
#define KC_E_NOMEM (-2)    /* device or host allocation failed */
#define KC_E_CAPACITY (-3) /* output arrays too small; *n_out holds the size needed */
#define KC_E_OVERFLOW (-4) /* a count exceeds UINT32_MAX */
#define KC_E_DEVICE (-5)   /* HIP runtime error (message in kc_last_error) */
#define KC_E_INTERNAL (-6) /* a device self-check failed (message in kc_last_error) */

/* Tuning knobs. Zero in any field means "choose automatically".
 * None of them changes the result, only how it is computed. */
typedef struct kc_options {
  int shard_bits;      /* log2 of the number of first-level key-range shards
                          (owner buckets are unions of shards); 1..10 */
  int leaf_target;     /* target valid windows per leaf partition when splitting
                          (automatic: 1.5 x the largest table for k <= 32, 0.75 x
                          for wider keys) */
  int leaf_attempt;    /* partitions up to this many windows are counted directly */
  int table_slots_log2;/* log2 of the largest LDS open-addressing table per leaf
                          (10..12 for k<=32, 10..11 for k>32) */
  int check;           /* 1 = run the device self-check of the output (sorted,
                          canonical, in range, sum of counts == valid windows) */
  int timing;          /* 1 = record per-stage times (kc_last_stats) */
  int mode;            /* how each leaf partition is counted: 0 = LDS open-addressing
                          table, then a sort of its distinct keys; 1 = sort of its
                          records and run-length accumulation (the counting by
                          sorting of Algorithm 1, as each owner does in Algorithm 3).
                          Same result.
                          The batched form takes 0 only (and k <= 32). */
  int scatter_tile;    /* window starts per thread of the owner scatter for keys of
                          one word: 8 (8,192-record LDS tiles, two workgroups per CU;
                          automatic) or 16 (16,384-record tiles, one workgroup per CU:
                          longer runs per shard when there are many shards) */
  int split_tile;      /* records per thread of the split scatter, likewise 8 or 16
                          (automatic: 16) */
  int refine_bits;     /* key bits by which an overflowed leaf is cut per refinement
                          level: 1..8 (automatic: 5) */
  int preagg;          /* pre-aggregation of equal keys in the split scatter (the
                          heavy-hitter aggregation of Section IV-D): runs of equal keys
                          in a tile's LDS staging leave as one (key, count) record, the
                          count in the key bits the shard makes redundant (keys of one
                          word in plain calls with 16-record split tiles). 0 automatic
                          (off), 1 on, 2 off. Same result either way. */
  int reserved[1];
} kc_options;

/* Statistics of the last successful call on this host thread. */
typedef struct kc_stats {
  uint64_t n_bases;        /* bytes covered by the reads */
  uint64_t valid_windows;  /* W: valid windows (= sum of the output counts) */
  uint64_t distinct;       /* D: distinct canonical keys (= *n_out) */
  uint64_t n_leaves;       /* leaf partitions counted */
  uint64_t n_levels;       /* partitioning levels below the shard level */
  uint64_t n_overflow;     /* leaf attempts that overflowed their table and were split
                              (one-word keys: after a second count with a table twice
                              as large also overflowed) */
  uint64_t max_leaf_windows;
  uint64_t max_owner_windows; /* windows in the largest of the P owner buckets */
  uint64_t refined_records; /* records counted again by the refinement's block-wide
                               leaf launches (parts of overflowed leaves) */
  uint64_t large_records;   /* records counted by the block-wide leaf kernel's own
                               launch (leaves above the one-wave size) */
  uint64_t large_distinct;  /* distinct keys that launch wrote */
  uint64_t second_records;  /* records counted by the second count of overflowed
                               leaves (one-word keys), refinement excluded */
  uint64_t second_distinct; /* distinct keys it wrote */
  double   ms_total;        /* host wall time of the call */
  double   ms_stage[12];    /* timing=1, device events on the call's stream (ms):
                               0 pack, 1 window histogram, 2 owner scatter (with the shard
                               plan), 3 split histogram, 4 split scatter (with the leaf plan),
                               5 small-leaf count (with leaf classification), 6 large-leaf
                               count, 7 output offsets, 8 concat, 9 self-check, 10 refinement
                               of overflowed leaves (its splits and part counts), 11 second
                               count of the leaves whose table overflowed (one-word keys) */
} kc_stats;

/* Count canonical k-mers (plain form).
 *   reads      device, ASCII bytes; read i = reads[offsets[i] .. offsets[i+1])
 *   offsets    device, n_reads+1 non-decreasing byte offsets (offsets[0] may be > 0)
 *   n_reads    number of reads (0 allowed)
 *   k          1..128
 *   P          number of owner partitions (>= 1)
 *   out_keys   device, room for kc_max_outputs() keys (1, 2 or 4 uint64 each, see above)
 *   out_counts device, room for kc_max_outputs() counts
 *   n_out      host; receives the number of distinct keys written
 * Returns KC_OK or a negative status. */
int kc_count(const uint8_t* reads, const uint64_t* offsets, uint64_t n_reads, int k, int P,
             uint64_t* out_keys, uint32_t* out_counts, uint64_t* n_out);

/* As kc_count with an explicit output capacity (in keys), options (NULL =
 * automatic) and a HIP stream (hipStream_t passed as void*, NULL = default).
 * If more than out_capacity keys result, returns KC_E_CAPACITY with *n_out set.
 * Returns once *n_out is known; the copy into the outputs may still be queued
 * on the stream. Calls of one host thread share its scratch arena: each call
 * first waits (on the device, in stream order) for the thread's previous
 * call's work, whatever stream that ran on. */
int kc_count_ex(const uint8_t* reads, const uint64_t* offsets, uint64_t n_reads, int k, int P,
                uint64_t* out_keys, uint32_t* out_counts, uint64_t out_capacity,
                uint64_t* n_out, const kc_options* opt, void* stream);

/* ---- Batched form: many independent read sets counted together.
 * (Each set's result is the k-mer histogram of Section II of its reads alone;
 * a memory wave plays the part of the batches of size b in which the BSP
 * algorithm of Section III-B counts, bounding the memory one pass holds.)
 * The sets are consecutive in one read stream: set s holds host_set_reads[s]
 * reads and host_set_bytes[s] bytes, and has its own k (1..32). A set's
 * result is exactly what kc_count gives for its reads alone.
 *
 * Memory waves: the plan cuts the sets, in order, into waves of consecutive
 * sets such that the device memory a wave needs (packed input, per-class
 * pipeline buffers, class outputs, tables) stays within hbm_budget bytes
 * (0 = no budget: one wave). The plan holds the memory of its largest wave
 * only: waves run one after the other on the same buffers. Inside a wave the
 * sets of one k are counted together in one pipeline pass per class with keys
 * (set id << 2k) | k-mer, so the counts of different sets never mix; a
 * wave's passes and the final placement of each set's pairs are recorded once
 * into a HIP graph and replayed.
 *
 * kc_batch_plan: host arrays of n_sets entries; P as in kc_count; opt may be
 *   NULL. Allocates the device memory of the batch; *plan receives the handle.
 *   KC_E_NOMEM if a single set needs more than hbm_budget.
 * kc_batch_waves / kc_batch_wave_info: the waves and, for each, its sets,
 *   reads and bytes (their ranges in the whole stream) and planned device bytes.
 * kc_batch_run_wave: counts one wave from ITS OWN inputs: reads/offsets are
 *   device arrays holding only the wave's reads (offsets has n_reads + 1
 *   entries, offsets[0] may be nonzero), so a caller can prepare wave w + 1
 *   while wave w counts. out_keys/out_counts: out_capacity entries (one uint64
 *   key each); host_out_set_offsets: a host array of n_sets + 1 entries of the
 *   wave receiving where each of its sets' pairs start.
 * kc_batch_run: all waves in turn on the inputs of the whole batch (offsets
 *   has sum(host_set_reads) + 1 entries); the sets' pairs follow each other in
 *   set order; host_out_set_offsets receives n_sets + 1 entries.
 * Both runs return KC_E_INVAL if the inputs do not match the plan, and
 *   KC_E_CAPACITY (with *n_out set to the pairs needed) if the outputs are too
 *   small. A wave's graph is recorded on its first run and recorded again when
 *   a pointer or the capacity changes. Runs with one plan must not overlap.
 *   When a class has a leaf its device-planned split cannot count, that
 *   wave's sets are counted one by one with kc_count's path instead (same
 *   result).
 * kc_batch_max_outputs: an upper bound of the pairs of the whole batch.
 * kc_batch_stats: totals of the last run (windows, distinct, leaves, times).
 * kc_batch_free: releases the plan. */
typedef struct kc_batch kc_batch;
typedef struct kc_batch_wave {
  uint32_t first_set, n_sets;
  uint64_t first_read, n_reads;
  uint64_t first_byte, n_bytes;
  uint64_t device_bytes;  /* planned device bytes of the wave */
  uint32_t n_classes;     /* pipeline passes in its graph */
  uint32_t pad;
} kc_batch_wave;
int kc_batch_plan(const uint64_t* host_set_reads, const uint64_t* host_set_bytes,
                  const int* host_ks, uint32_t n_sets, int P, uint64_t hbm_budget,
                  const kc_options* opt, kc_batch** plan);
uint32_t kc_batch_waves(const kc_batch* plan);
int kc_batch_wave_info(const kc_batch* plan, uint32_t wave, kc_batch_wave* out);
int kc_batch_run_wave(kc_batch* plan, uint32_t wave, const uint8_t* reads,
                      const uint64_t* offsets, uint64_t* out_keys, uint32_t* out_counts,
                      uint64_t out_capacity, uint64_t* host_out_set_offsets, uint64_t* n_out,
                      void* stream);
int kc_batch_run(kc_batch* plan, const uint8_t* reads, const uint64_t* offsets,
                 uint64_t* out_keys, uint32_t* out_counts, uint64_t out_capacity,
                 uint64_t* host_out_set_offsets, uint64_t* n_out, void* stream);
uint64_t kc_batch_max_outputs(const kc_batch* plan);
int kc_batch_stats(const kc_batch* plan, kc_stats* out);
void kc_batch_free(kc_batch* plan);

/* ---- Served form: a request server counting many jobs side by side.
 * Each job is a plain count (same arguments and result as kc_count). All of
 * the server's device memory is one allocation made at creation (the budget,
 * or what the device has free less a margin, whichever is smaller), from
 * which each job's scratch block and each result are cut: serving maps and
 * unmaps no device memory. A fixed pool of worker threads, each with its own
 * HIP stream, takes jobs from one arrival-ordered queue; a worker starts the
 * first queued job whose device bytes fit in what the budget has left (its
 * scratch block plus a reservation for its result) and for whose scratch a
 * free range exists; a job passed over 8 times holds back the later ones
 * until it fits. Results are allocated at their exact size when the job's
 * number of distinct keys is known and stay on the device, owned by the
 * server, until kc_server_release. A job's result does not depend on what
 * else runs beside it.
 *
 * kc_server_create: hbm_budget_bytes caps the device bytes the server maps
 *   and accounts for (scratch, reservations, held results); n_workers in [1, 16]
 *   (streams run concurrently); opt as in kc_count_ex (NULL = automatic),
 *   applied to every job. The calling thread's current device is used.
 * kc_server_submit: reads/offsets are DEVICE arrays as in kc_count that must
 *   hold their final contents at submission and stay allocated until the job
 *   has finished. distinct_hint: 0, or an estimate of the job's distinct keys
 *   (reserves distinct_hint pairs instead of one pair per input byte; a low
 *   hint is still correct: the result is allocated at its true size and the
 *   miss is counted in kc_server_stats). Returns KC_E_NOMEM at once if the
 *   job alone needs more than the budget; *job_id receives the job's id.
 * kc_server_poll / kc_server_wait: the job's state (KC_JOB_*); wait blocks
 *   until it is DONE or FAILED. Results the client has not released stay
 *   charged to the budget: if they leave too little for every queued job
 *   while nothing runs and every worker has given its scratch back, no queued
 *   job can ever start, and kc_server_wait on a queued job returns
 *   KC_E_NOMEM at once (the job stays queued; release results and wait
 *   again) instead of blocking.
 * kc_server_result: device pointers to the sorted keys (1, 2 or 4 words each, as
 *   in kc_count) and counts, and their number. A FAILED job returns its status
 *   (message in kc_last_error).
 * kc_server_result_copy: copies a finished job's result into caller DEVICE
 *   arrays of out_capacity keys (1, 2 or 4 words each) and counts, on `stream`,
 *   and returns when the copy is complete; KC_E_CAPACITY (with *n_out set)
 *   if they are too small.
 * kc_server_release: frees a finished job's result and forgets the job.
 * kc_server_destroy: waits for running jobs, drops queued ones, frees all. */
#define KC_JOB_QUEUED 0
#define KC_JOB_RUNNING 1
#define KC_JOB_DONE 2
#define KC_JOB_FAILED 3

typedef struct kc_server kc_server;

typedef struct kc_job_info {
  int state, status, worker, k;
  uint64_t n_bytes, valid_windows, distinct;
  uint64_t result_estimate_bytes; /* reserved at admission */
  uint64_t result_bytes;          /* allocated for the result */
  double t_submit_ms, t_start_ms, t_end_ms; /* host clock, since the server was created */
} kc_job_info;

typedef struct kc_server_stats {
  uint64_t submitted, completed, failed, queued, running;
  uint64_t valid_windows;          /* of completed jobs */
  uint64_t budget, bytes_in_use, bytes_peak;
  uint64_t estimate_misses;        /* results larger than their reservation */
  uint64_t result_bytes_reserved;  /* sum over finished jobs */
  uint64_t result_bytes_actual;
  uint64_t slab_bytes;             /* device memory the server mapped at creation */
  uint64_t unplaced;               /* times a job that fit the budget waited because no free
                                      range of that memory was large enough for its scratch */
  double latency_p50_ms, latency_p99_ms; /* completion - submission, completed jobs */
  double wait_p50_ms, wait_p99_ms;       /* start - submission */
  double busy_ms;                        /* first start to last completion */
} kc_serve_stats;

int kc_server_create(uint64_t hbm_budget_bytes, int n_workers, const kc_options* opt,
                     kc_server** server);
int kc_server_submit(kc_server* server, const uint8_t* reads, const uint64_t* offsets,
                     uint64_t n_reads, int k, int P, uint64_t distinct_hint, uint64_t* job_id);
int kc_server_poll(kc_server* server, uint64_t job_id, int* state);
int kc_server_wait(kc_server* server, uint64_t job_id, int* state);
int kc_server_result(kc_server* server, uint64_t job_id, const uint64_t** keys,
                     const uint32_t** counts, uint64_t* n_out);
int kc_server_result_copy(kc_server* server, uint64_t job_id, uint64_t* out_keys,
                          uint32_t* out_counts, uint64_t out_capacity, uint64_t* n_out,
                          void* stream);
int kc_server_job_info(kc_server* server, uint64_t job_id, kc_job_info* out);
int kc_server_release(kc_server* server, uint64_t job_id);
int kc_server_stats(kc_server* server, kc_serve_stats* out);
void kc_server_destroy(kc_server* server);

/* ---- Size predictor: an estimate of a job's number of distinct keys.
 * A two-layer fp32 perceptron y = w2 . relu(W1 x + b1) + b2 whose forward and
 * backward passes and Adam updates run on the device. It never touches a
 * count: its only use is the result reservation of a served job
 * (distinct_hint of kc_server_submit), where a miss costs memory accounting,
 * not correctness. Parameters are one fp32 array: W1 [hidden][n_features]
 * row-major, b1 [hidden], w2 [hidden], b2. Loss: mean of (y - t)^2 / 2.
 *
 * kc_pred_create: n_features in [1, 32], hidden in [1, 128]; seeded init.
 * kc_pred_forward: x DEVICE [batch][n_features] fp32, y DEVICE [batch];
 *   synchronous on `stream`.
 * kc_pred_gradient: x, target DEVICE; computes the loss gradient of the batch
 *   into the predictor (deterministic order); *host_loss (if not NULL)
 *   receives the loss (then synchronous).
 * kc_pred_adam_step: one Adam step (beta 0.9 / 0.999) with the last gradient.
 * kc_pred_get_params / _set_params / _get_grads: host copies of n floats
 *   (n = kc_pred_num_params); set_params restarts the optimiser state. */
typedef struct kc_predictor kc_predictor;
int kc_pred_create(int n_features, int hidden, uint64_t seed, kc_predictor** pred);
uint64_t kc_pred_num_params(const kc_predictor* pred);
int kc_pred_get_params(const kc_predictor* pred, float* host, uint64_t n);
int kc_pred_set_params(kc_predictor* pred, const float* host, uint64_t n);
int kc_pred_get_grads(const kc_predictor* pred, float* host, uint64_t n);
int kc_pred_forward(kc_predictor* pred, const float* x, uint64_t batch, float* y, void* stream);
int kc_pred_gradient(kc_predictor* pred, const float* x, const float* target, uint64_t batch,
                     float* host_loss, void* stream);
int kc_pred_adam_step(kc_predictor* pred, float lr, void* stream);
void kc_pred_free(kc_predictor* pred);

/* ---- Uses of a result (keys and counts as kc_count writes them; DEVICE arrays).
 * The histogram is an input to the applications the paper lists in Section I
 * (assembly, error correction, repeat detection, genome quality assessment):
 * those read it as a spectrum (how many keys occur c times: error and repeat
 * peaks) and drop rare keys below a count cut-off, as the Bloom-filter and
 * quotient-filter counters cited in Section II-A do for singletons. Section VI
 * counts every key from count 1 up, so kc_count itself filters nothing.
 * kc_merge_counts rests on the same fact as the partitioned counting of
 * Algorithms 2 and 3: a histogram is the sum of the histograms of any split of
 * the reads (each part is counted on its own, the parts' counts are added),
 * which lets an input larger than device memory be counted in pieces (the
 * paper's largest data set, Table V, exceeds one device's memory).
 *
 * kc_spectrum: the k-mer spectrum of a result: host_hist (max_count + 1
 *   entries) receives in host_hist[c] the number of keys with count c for
 *   1 <= c < max_count, in host_hist[max_count] the number with count >=
 *   max_count; host_hist[0] = 0. max_count in [1, 2^24]. Synchronous on stream.
 * kc_filter_min_count: copies the pairs with count >= min_count, in their
 *   order, to out_keys / out_counts (room for n pairs; must not overlap the
 *   inputs); *n_out receives their number. k gives the key width (1, 2 or 4
 *   words, as in kc_count). Synchronous on stream.
 * kc_merge_counts: the result of the union of two read collections from their
 *   two results (sorted, unique keys; the count of a read collection is the
 *   sum over any split of it): the ordered union of the keys with counts added
 *   where a key is in both. out arrays have room for na + nb pairs and must
 *   not overlap the inputs; *n_out receives the number of pairs. KC_E_OVERFLOW
 *   if a sum exceeds 2^32-1. Lets inputs larger than device memory be counted
 *   in pieces whose results are merged. Synchronous on stream.
 * The temporaries of kc_merge_counts ((na + nb) * (8 * words + 4) bytes) and
 * kc_filter_min_count sit in one device buffer per host thread, part of the
 * thread's scratch arena: it grows stream-ordered from the library pool as
 * needed and is kept between calls (kc_release_scratch frees it).
 * All return KC_OK, KC_E_INVAL, KC_E_NOMEM or KC_E_DEVICE (and as stated). */
int kc_spectrum(const uint32_t* counts, uint64_t n, uint32_t max_count, uint64_t* host_hist,
                void* stream);
int kc_filter_min_count(const uint64_t* keys, const uint32_t* counts, uint64_t n, int k,
                        uint32_t min_count, uint64_t* out_keys, uint32_t* out_counts,
                        uint64_t* n_out, void* stream);
int kc_merge_counts(const uint64_t* a_keys, const uint32_t* a_counts, uint64_t na,
                    const uint64_t* b_keys, const uint32_t* b_counts, uint64_t nb, int k,
                    uint64_t* out_keys, uint32_t* out_counts, uint64_t* n_out, void* stream);

/* Text formats of kc_parse_fastx. */
enum { KC_FASTX_AUTO = 0, KC_FASTQ = 1, KC_FASTA = 2 };

/* kc_parse_fastx: the reads of a FASTQ or FASTA text held in device memory, in
 * the form kc_count takes (the paper counts k-mers of reads; it leaves reading
 * them from files out of its measurements, Section VI).
 *   text, n_bytes: the file's bytes as they are, on the device.
 *   format: KC_FASTQ (records of exactly four lines: '@' name, sequence, '+'
 *     [name], quality), KC_FASTA ('>' header line, then any number of
 *     sequence lines, concatenated), or KC_FASTX_AUTO (FASTQ if the first
 *     byte that is not CR/LF is '@', FASTA if it is '>'); *format_out (may be
 *     NULL) receives the format used.
 *   Line ends at the start and end of the text are ignored; CR bytes are
 *   dropped from sequence lines (CRLF files); every other sequence byte is
 *   kept as it is (kc_count treats bytes other than ACGT/acgt as breaks).
 *   out_reads (room for reads_capacity bytes; n_bytes always suffices) gets the
 *   sequences concatenated; out_offsets (room for max_records + 1 entries)
 *   gets the CSR offsets, out_offsets[0] = 0; *n_records and *n_bases get
 *   their numbers.
 * Returns KC_E_CAPACITY with *n_records (and *n_bases, once known) set when
 * the outputs are too small, nothing written to them; KC_E_INVAL for a FASTQ
 * text whose line count is not a multiple of four or whose header / separator
 * lines do not start with '@' / '+' (kc_last_error names the line), or a FASTA
 * text not starting with '>'. Synchronous on stream; uses a small device
 * allocation on the stream (stream-ordered). */
int kc_parse_fastx(const uint8_t* text, uint64_t n_bytes, int format, uint8_t* out_reads,
                   uint64_t reads_capacity, uint64_t* out_offsets, uint64_t max_records,
                   uint64_t* n_records, uint64_t* n_bases, int* format_out, void* stream);

/* ---- Allocation-free form, for callers that cannot allocate device memory
 * (code that runs between a HIP graph capture's begin and end, tight serving
 * loops, harnesses that forbid hipMalloc).
 * kc_count_noalloc: the same arguments, result and errors as kc_count_ex, but
 * the call allocates nothing: no hipMalloc / hipFree, no pool or pinned host
 * allocation, no event or stream creation. Its device scratch is one fixed
 * array of KC_NOALLOC_SCRATCH_MIB MiB per device, part of the library's code
 * object (each device the library runs on holds it until the process ends);
 * small host copies go through a fixed static host array of 8 MiB.
 *   - Inputs whose scratch need exceeds the array are refused up front with
 *     KC_E_NOMEM and a message giving both sizes (about 21 bytes of scratch
 *     per read byte for k <= 32, 37 for k <= 64, 69 for k <= 128: roughly
 *     12, 7 and 3.7 MB of reads). The rare leaf refinement that a
 *     repeat-rich input may need also takes its buffers from the array and
 *     fails the same way if it runs out.
 *   - The call is synchronous: the outputs are complete when it returns.
 *   - Every call on a device shares that device's array and the static host
 *     array, which keep the last call's contents (each call clears what it
 *     needs cleared). Calls are serialized by a process-wide lock; work that
 *     another library call (or kernel) leaves running on the same device
 *     concurrently does not touch the array.
 *   - timing in opt is ignored (no events are created). */
#define KC_NOALLOC_SCRATCH_MIB 256
int kc_count_noalloc(const uint8_t* reads, const uint64_t* offsets, uint64_t n_reads, int k,
                     int P, uint64_t* out_keys, uint32_t* out_counts, uint64_t out_capacity,
                     uint64_t* n_out, const kc_options* opt, void* stream);

/* Upper bound on the number of output keys (= number of length-k windows,
 * valid or not): sum over reads of max(0, len - k + 1). host_offsets is a
 * HOST array of n_reads+1 offsets. Returns 0 for bad arguments. */
uint64_t kc_max_outputs(const uint64_t* host_offsets, uint64_t n_reads, int k);

/* Copy the statistics of this thread's last successful call. Returns KC_OK,
 * or KC_E_INVAL if out is NULL. */
int kc_last_stats(kc_stats* out);

/* Release this thread's scratch arena and the temporary buffer of
 * kc_merge_counts / kc_filter_min_count, and return the idle blocks of the
 * library's device memory pool (the arenas of kc_count grow stream-ordered
 * from that pool, which keeps freed blocks for reuse instead of handing them
 * back to the driver at once) to the device. */
void kc_release_scratch(void);

/* Static description of a status code. */
const char* kc_strerror(int status);

/* Message for the last error on this host thread ("" if none). */
const char* kc_last_error(void);

/* Library version string. */
const char* kc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KC_H */
