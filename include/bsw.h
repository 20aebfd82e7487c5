/*
 * bsw.h -- C ABI of libbsw.so: banded Smith-Waterman seed extension (BSW)
 * on AMD Instinct MI355X (gfx950).
 *
 * The operation (paper Sec. 5.1, Eq. (2) and (3); rules (a)-(c) of
 * Sec. 5.1; outputs of Sec. 5.4 (a),(b)): for each pair (query q, target t,
 * seed score h0) extend the seed by affine-gap dynamic programming over a
 * band around the diagonal, one target position per row and one query
 * position per column, stopping when a row is all zero or has dropped
 * further than z-drop below the best score, and narrowing the band after
 * each row by its empty cells at both ends.  Readings of the points the
 * paper leaves open (gap cost o + k*e with gaps opening from the diagonal
 * term, positive-diagonal gating, boundary rows, tie rules, band cap by the
 * end bonus) are documented with the implementation; every result is
 * bit-identical to the reference implementation of those rules.
 *
 * Conventions for every entry point:
 *  - Sequences are byte codes 0..3 = A,C,G,T and 4 = N, concatenated; pair
 *    k's query is q[q_off[k] .. q_off[k+1]) and its target
 *    t[t_off[k] .. t_off[k+1]).  Offsets are non-decreasing uint64.
 *  - Lengths are at most BSW_MAX_LEN; 1 <= h0 <= BSW_MAX_H0.
 *  - param_id[k] selects params[param_id[k]] (n_params <= 256); a NULL
 *    param_id means set 0 for every pair.
 *  - The caller owns every input and output buffer.  The library keeps no
 *    pointer to them once a call has returned (blocking calls) or once the
 *    stream has passed the enqueued work (asynchronous calls).  It owns only
 *    its context (device arena, streams, events).
 *  - Errors are negative status codes; bsw_last_error() describes the most
 *    recent one of the calling thread.  On an error no output is written.
 *  - n = 0 is a no-op that returns BSW_OK.
 *  - One context per host thread (a context is not thread-safe).
 *  - A context holds at most one asynchronous call: until bsw_ctx_wait has
 *    returned for it, every call that enqueues work on the context returns
 *    BSW_EBUSY and enqueues nothing (the pending call's queued work still
 *    reads the context's scoring table, status block and captured graph).
 */
#ifndef BSW_H
#define BSW_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BSW_ABI_VERSION 1

#define BSW_MAX_LEN   65535
#define BSW_MAX_H0    (1 << 24)
#define BSW_MAX_GAP   1000      /* max o_* and e_*                      */
#define BSW_MAX_BONUS (1 << 24)

/* One scoring set (56 bytes).  mat[a*5+b] scores target code a against
 * query code b.  A gap of length k >= 1 costs o + k*e; deletions consume
 * target only, insertions query only.  Requirements: 0 <= o <= 1000,
 * 1 <= e <= 1000, w >= 0, 0 <= end_bonus <= 2^24; zdrop <= 0 disables the
 * drop-from-best abort.  The end bonus only narrows the band:
 * w' = min(w, cap_ins, cap_del), cap = (qlen*A + end_bonus - o)/e + 1 with
 * A = max(0, max mat). */
typedef struct bsw_params {
  int8_t  mat[25];
  int8_t  pad_[3];
  int32_t o_del, e_del, o_ins, e_ins;
  int32_t w;
  int32_t zdrop;
  int32_t end_bonus;
} bsw_params;

/* Per-pair result (24 bytes). */
typedef struct bsw_result {
  int32_t score;   /* best score; h0 when nothing beat the seed            */
  int32_t qle;     /* 1-based query end of the best cell; 0 = none         */
  int32_t tle;     /* 1-based target end of the best cell; 0 = none        */
  int32_t gtle;    /* 1-based target end where gscore was reached; 0 = never */
  int32_t gscore;  /* best score reaching the query end; -1 = never        */
  int32_t max_off; /* largest |column - row| over improving cells          */
} bsw_result;

/* Optional per-pair diagnostics (16 bytes). */
typedef struct bsw_diag {
  int32_t rows;    /* rows entered, the stopping row included              */
  int32_t stop;    /* 0 = target exhausted, 1 = all-zero row, 2 = z-drop   */
  int64_t cells;   /* band cells computed over those rows                  */
} bsw_diag;

enum {
  BSW_OK = 0,
  BSW_EINVAL = -1,  /* bad argument or pair (see bsw_last_error)           */
  BSW_ENOMEM = -2,  /* device or host allocation failed                    */
  BSW_EDEVICE = -3, /* no usable gfx950 device, or a HIP call failed       */
  BSW_ETOOBIG = -4, /* request larger than the context's HBM budget        */
  BSW_EBUSY = -5,   /* serving: queue full; context: an asynchronous call
                     * is still pending (call bsw_ctx_wait)                 */
  BSW_ETIMEOUT = -6 /* serving: ticket not complete within the timeout     */
};

/* Execution path used by a call. */
enum {
  BSW_PATH_BATCHED = 0, /* length binning + persistent longest-first tile
                         * queues; the default                              */
  BSW_PATH_PLAIN = 1    /* length binning + one ordinary launch per bin     */
};

typedef struct bsw_ctx bsw_ctx;

/* Options for bsw_ctx_create (zero-initialise, then set what you need). */
typedef struct bsw_ctx_opts {
  int32_t device;          /* HIP device ordinal                           */
  int32_t min_lane_bits;   /* 0 = pick 8/16/32 from each pair's score bound;
                            * 16 or 32 forces at least that width           */
  int32_t max_groups;      /* batched path: cap on the persistent workgroups
                            * of each kernel class (0 = as many as are
                            * resident on the device); a cap below a class's
                            * tile count makes every workgroup take several
                            * tiles from the class queue                    */
  int32_t path;            /* BSW_PATH_BATCHED or BSW_PATH_PLAIN            */
  size_t  hbm_budget;      /* cap on the context's device arena in bytes
                            * (0 = none); a call that would need more fails
                            * with BSW_ETOOBIG before any work is enqueued   */
  const char* tune_cache;  /* JSON file of tuned launch shapes (the path is
                            * copied at creation), or NULL: an
                            * entry for the device, band limit, gap symmetry
                            * and min_lane_bits of a call is used when
                            * present; bsw_ctx_tune adds or replaces it      */
  int32_t no_graph;        /* batched path: 0 = capture the pipeline into a
                            * HIP graph on the first call with a given set of
                            * pointers and shapes and replay it on later
                            * calls; 1 = enqueue every step eagerly          */
} bsw_ctx_opts;

/* Create a context on a device.  Returns BSW_EDEVICE when the device is
 * missing or is not gfx950.  *out is set only on success. */
int bsw_ctx_create(bsw_ctx** out, const bsw_ctx_opts* opts);
void bsw_ctx_destroy(bsw_ctx* ctx);

/* Host-memory batch: validates every argument first, stages the inputs
 * into the context's device arena, runs the extension and copies the
 * results (and diagnostics when diag != NULL) back.  Blocking. */
int bsw_extend_batch(bsw_ctx* ctx, int64_t n,
                     const uint8_t* q, const uint64_t* q_off,
                     const uint8_t* t, const uint64_t* t_off,
                     const int32_t* h0, const uint8_t* param_id,
                     const bsw_params* params, int32_t n_params,
                     bsw_result* out, bsw_diag* diag);

/* Device-memory batch.  q, q_off, t, t_off, h0, param_id (nullable), out
 * and diag (nullable) are device pointers; params is a host array.  The
 * work is enqueued on `stream` (a hipStream_t; NULL = the context's own
 * stream).  q_off[n] and t_off[n] are read on the device, so the sequence
 * sizes need not be known on the host.  Per-pair checks (codes, lengths,
 * h0, param_id) run on the device before any result is written; a bad
 * pair makes the whole call write nothing.  With async = 0 the call waits
 * for the stream and returns the final status; with async != 0 it returns
 * after enqueueing and bsw_ctx_wait() returns the status later.  Between
 * an asynchronous call and its wait the inputs must stay valid. */
int bsw_extend_batch_device(bsw_ctx* ctx, int64_t n,
                            const uint8_t* q, const uint64_t* q_off,
                            const uint8_t* t, const uint64_t* t_off,
                            const int32_t* h0, const uint8_t* param_id,
                            const bsw_params* params, int32_t n_params,
                            bsw_result* out, bsw_diag* diag,
                            void* stream, int32_t async);

/* Allocation-free form of bsw_extend_batch_device, for callers that cannot
 * allocate device memory: code being captured into a HIP graph, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, checks,
 * results and status as bsw_extend_batch_device on the batched path, but
 * the call allocates nothing (no hipMalloc/hipFree, no library routine that
 * allocates) and captures no graph of its own: its workspace lives in one
 * fixed 16 MiB device array per GPU, reserved with the library and held
 * until the process ends, whose address each context takes when it is
 * created.  Limits: at most BSW_NOALLOC_MAX_PAIRS pairs per call (more
 * gives BSW_ETOOBIG before anything is enqueued); pairs whose values need
 * 16-bit records run on at most 64 workgroups per class and queries longer
 * than 256 on 4 waves, so such batches are slower than on the ordinary
 * entry point; the context's path must be BSW_PATH_BATCHED (else
 * BSW_EINVAL).  Every context on a GPU shares that GPU's array, and it
 * keeps the last call's contents (each call clears what must start at
 * zero), so calls that overlap on one GPU, from any context or stream,
 * race and must be serialised by the caller.  async as in
 * bsw_extend_batch_device (under graph capture pass async != 0). */
#define BSW_NOALLOC_MAX_PAIRS 131072
int bsw_extend_batch_device_noalloc(bsw_ctx* ctx, int64_t n,
                                    const uint8_t* q, const uint64_t* q_off,
                                    const uint8_t* t, const uint64_t* t_off,
                                    const int32_t* h0, const uint8_t* param_id,
                                    const bsw_params* params, int32_t n_params,
                                    bsw_result* out, bsw_diag* diag,
                                    void* stream, int32_t async);

/* Autotuner of the batched path.  Runs the batched path over a device batch
 * (arguments as bsw_extend_batch_device; results are written to out as by
 * a normal call) under candidate launch shapes, by coordinate descent from
 * the default shape: each knob in turn takes every value while the others
 * stay at the best so far.  The knobs are the side streams the kernel
 * classes are spread over (4, 2, 1; at most GPU_MAX_HW_QUEUES - 2, so that
 * with the caller's and the runtime's default stream no two streams share a
 * hardware queue; default 2), the share of resident groups per CU
 * for the 8-bit classes (100%, 75%, 50%), whether pairs whose score bound
 * needs 16 bits are tried at 8 bits first (yes, no), and the query cap from
 * which the 32-bit classes run one pair per wave instead of one pair per
 * lane (64, 128, 256, never, 32; Sec. 5.2.1 intra-task vs Sec. 5.3
 * inter-task).  Each candidate runs eagerly: one warm-up call, then reps
 * (1..100) timed calls, scored by their median device time; a shape must
 * beat the best so far by more than 1%.  The winner is used
 * by every later batched call of the context with the same band limit and
 * gap symmetry, and is stored in tune_cache when one is set.  *best_ms
 * (nullable) receives its time.  Blocking. */
int bsw_ctx_tune(bsw_ctx* ctx, int64_t n, const uint8_t* q, const uint64_t* q_off,
                 const uint8_t* t, const uint64_t* t_off, const int32_t* h0,
                 const uint8_t* param_id, const bsw_params* params, int32_t n_params,
                 bsw_result* out, int32_t reps, double* best_ms);

/* The context's current launch shape: out3 = {side streams, 8-bit share of
 * resident groups in percent, 16-bit pairs tried at 8 bits (0/1)}. */
int bsw_ctx_tune_info(bsw_ctx* ctx, int32_t out3[3]);

/* The context's current launch shape for pair batches: out[0..n) receives
 * up to four values {side streams, 8-bit share of resident groups in
 * percent, 16-bit pairs tried at 8 bits (0/1), query cap from which 32-bit
 * classes run in wave mode (512 = never)}.  Returns the number of values
 * the shape has (4). */
int bsw_ctx_shape(bsw_ctx* ctx, int32_t* out, int32_t n);

/* Wait for the last asynchronous call on ctx and return its status
 * (BSW_EINVAL with the first bad pair in bsw_last_error if a pair was
 * rejected on the device). */
int bsw_ctx_wait(bsw_ctx* ctx);

/* Timing of the last completed call's device work, in milliseconds:
 * [0] = whole pipeline (first to last kernel), [1] = prepare and bin,
 * [2] = DP kernels, [3] = number of DP kernel launches.  A call that ran as
 * a graph replay has [0] only ([1] = [2] = 0).  Returns BSW_OK. */
int bsw_ctx_last_timing(bsw_ctx* ctx, double out4[4]);

/* Band cells settled by the last completed call (all of its BSW passes;
 * the rerun of pairs that overflowed a narrow record width counts again);
 * after bsw_fm_smem_device the extension steps it ran, after the other
 * index calls 0.  Returns BSW_OK. */
int bsw_ctx_last_cells(bsw_ctx* ctx, int64_t* cells);

/* Per-launch record of the last completed call's DP kernels: for launch k,
 * cls[k] = kernel class (see bsw_class_name), cells[k] = band cells the
 * launch settled, ms[k] = its device time from HIP events on the launch
 * stream (0 for a call that ran as a graph replay: events inside a graph
 * carry no timestamps; use a context with no_graph = 1 to time launches).
 * Any output pointer may be NULL; at most max entries are written.
 * Returns the number of launches (may exceed max). */
int bsw_ctx_last_kernels(bsw_ctx* ctx, int32_t* cls, int64_t* cells, double* ms,
                         int32_t max);

/* Work behind the cells of the last completed call's DP launches, in the
 * order of bsw_ctx_last_kernels: work[k] = lane-cells launch k stepped
 * through (each wave's column span of every row it ran, times its 64
 * lanes, lanes that were padding or had already stopped included), so
 * that cells[k] / work[k] is the share of the launch's work that the
 * method needed (Sec. 6, the useful-cell share of the inter-task kernel).
 * 0 for kernels that do not count it (one pair per wave or per lane with
 * a private buffer).  At most max entries are written.  Returns the number
 * of launches. */
int bsw_ctx_last_work(bsw_ctx* ctx, int64_t* work, int32_t max);

/* Name of a kernel class ("lane8_q256" = one pair per lane, 8-bit row
 * buffer, queries up to 256; "rerun" = one pair per wave with 32-bit values,
 * for the pairs a class could not settle in its record width). */
const char* bsw_class_name(int32_t cls);

/* ------------------------------------------------------------------------
 * Serving (the paper's reorganisation of the work into large batches with
 * buffers reused across them, Sec. 3.2 and 5.3.1, applied to requests that
 * arrive over time).  A server owns one device arena of hbm_budget bytes
 * that holds the data of every admitted request (sequences, offsets, h0 and
 * param_id) from admission until its batch has run, and max_inflight
 * execution slots (each a context with its own stream and workspace).
 * Requests are admitted strictly in arrival order while the head request
 * fits in the free arena space.  Whenever a slot is free, the admitted
 * requests join one batch (up to max_batch_pairs pairs): on the slot's own
 * stream their data is copied to their regions, their codes are checked,
 * and the batched path runs; results are copied back into each request's
 * own output buffer.  A request's results equal those of the same pairs
 * run alone (pairs are independent).
 * ---------------------------------------------------------------------- */
typedef struct bsw_server bsw_server;

typedef struct bsw_server_opts {
  int32_t device;
  int32_t max_inflight;     /* slots (concurrent batches), 1..8; 0 = 3      */
  int64_t max_batch_pairs;  /* pairs per batch cap; 0 = 4,194,304; a larger
                             * request runs as a batch of its own            */
  size_t  hbm_budget;       /* arena for resident request data; 0 = 16 GiB  */
  int32_t max_queued;       /* submitted, not yet admitted requests before
                             * bsw_server_submit returns BSW_EBUSY; 0 = 65536 */
  int32_t min_lane_bits;    /* as in bsw_ctx_opts                          */
} bsw_server_opts;

/* Latency and throughput since creation or the last reset.  Latency runs
 * from bsw_server_submit to the results being in the caller's buffers. */
typedef struct bsw_server_report {
  int64_t submitted;        /* accepted by bsw_server_submit               */
  int64_t completed;        /* finished with BSW_OK                        */
  int64_t failed;           /* finished with an error (invalid pair)       */
  int64_t batches;          /* batches run                                 */
  int64_t pairs;            /* pairs of the completed requests             */
  int64_t cells;            /* band cells settled by the batches           */
  double  mean_batch_pairs;
  double  lat_p50_ms, lat_p99_ms, lat_p999_ms, lat_max_ms;
  double  admit_wait_mean_ms, admit_wait_p99_ms; /* submit -> admission    */
  double  window_s;         /* first submit -> last completion             */
  double  gcups;            /* cells / window_s / 1e9                      */
} bsw_server_report;

/* Create a server on a device with one scoring table for all requests
 * (n_params <= 256, validated as for bsw_extend_batch).  The arena and the
 * slots are allocated here; BSW_ENOMEM if they do not fit. */
int bsw_server_create(bsw_server** out, const bsw_server_opts* opts,
                      const bsw_params* params, int32_t n_params);
/* Finish every submitted request, then release the server. */
void bsw_server_destroy(bsw_server* srv);

/* Submit a request of n >= 1 pairs in host memory (same layout and rules
 * as bsw_extend_batch; param_id indexes the server's table).  Offsets,
 * lengths, h0 and param_id are checked here (BSW_EINVAL); the codes are
 * checked on the device when the request's batch runs, and a bad code
 * fails the request (alone) at bsw_server_wait.  Returns BSW_ETOOBIG if the
 * request needs more than the whole arena, BSW_EBUSY if max_queued
 * requests are waiting for admission.  On success *ticket identifies the
 * request.  Arrays in pinned host memory (hipHostMalloc) are read by the
 * device directly, the others are copied by the runtime.  Every buffer of
 * the request, out and diag (nullable) included, must stay valid and
 * unchanged until bsw_server_wait has returned for the ticket. */
int bsw_server_submit(bsw_server* srv, int64_t n,
                      const uint8_t* q, const uint64_t* q_off,
                      const uint8_t* t, const uint64_t* t_off,
                      const int32_t* h0, const uint8_t* param_id,
                      bsw_result* out, bsw_diag* diag, uint64_t* ticket);

/* Wait up to timeout_ms (< 0 = no limit) for a request; returns its status
 * (BSW_OK, or BSW_EINVAL for a request with a bad code) and forgets the
 * ticket, or BSW_ETIMEOUT (the ticket stays valid), or BSW_EINVAL for an
 * unknown ticket.  Any thread may wait; each ticket is waited for once. */
int bsw_server_wait(bsw_server* srv, uint64_t ticket, int32_t timeout_ms);

/* Fill *out; reset != 0 starts a new measurement window. */
int bsw_server_stats(bsw_server* srv, bsw_server_report* out, int32_t reset);

/* ------------------------------------------------------------------------
 * Read-level seed extension: the step around BSW in the read mapper
 * (Sec. 2: a seed, an exact match of read bases to the reference, is
 * extended on both sides; Sec. 5.3.2: every seed is extended, and the
 * removal of seeds the mapper would not have extended comes afterwards and
 * is not part of this step).  For each seed, with w and end_bonus of the
 * scoring set:
 *  1. left: BSW on the reversed read prefix read[0, qb) against the
 *     reversed reference window ref[max(0, rb - qb - w), rb), from the seed
 *     score h0;
 *  2. the end kept is the read start when gscore > 0 and
 *     gscore > score - end_bonus (reaching the end of the read costs less
 *     than the bonus), else the best cell; the kept score is h1;
 *  3. right: BSW on read[qe, len) against ref[re, min(ref_len,
 *     re + len - qe + w)) with re = rb + qe - qb, from h1; the end is kept
 *     by the same rule.
 * A side with nothing to extend (qb = 0, or qe = len) keeps the seed
 * boundary and carries the score over; its BSW call sees an empty query and
 * its result is not used.  The two BSW calls run the batched path of the
 * context (never as a graph replay).
 * ---------------------------------------------------------------------- */

/* One seed (24 bytes): read[qb, qe) equals ref[rb, rb + qe - qb). */
typedef struct bsw_seed {
  int32_t read;   /* read index, 0 <= read < n_reads                      */
  int32_t qb, qe; /* 0 <= qb <= qe <= read length                         */
  int32_t h0;     /* seed score, 1..BSW_MAX_H0                            */
  int64_t rb;     /* 0 <= rb, rb + qe - qb <= ref_len                     */
} bsw_seed;

/* Which end a side kept. */
enum { BSW_END_LOCAL = 0, BSW_END_READ = 1, BSW_END_NONE = 2 };

/* Result of one seed (32 bytes). */
typedef struct bsw_seed_result {
  int32_t score;      /* score after both sides                           */
  int32_t qbeg, qend; /* extended read interval [qbeg, qend)              */
  int32_t how;        /* left | right << 2, each a BSW_END_* value        */
  int64_t rbeg, rend; /* extended reference interval [rbeg, rend)         */
} bsw_seed_result;

/* Host-memory form.  Reads are byte codes 0..4 concatenated, read i being
 * reads[read_off[i] .. read_off[i+1]) (n_reads + 1 non-decreasing offsets,
 * lengths <= BSW_MAX_LEN); ref holds ref_len codes 0..4.  params is one
 * scoring set (as for bsw_extend_batch).  Every seed is checked on the host
 * first (BSW_EINVAL names the first bad one, as does a reference window
 * longer than BSW_MAX_LEN); a code > 4 in a read or in the reference fails
 * the call on the device.  The reads, the reference and the seeds are
 * copied to the device on every call.  Blocking; n = 0 is a no-op. */
int bsw_extend_seeds(bsw_ctx* ctx, const uint8_t* reads, const uint64_t* read_off,
                     int64_t n_reads, const uint8_t* ref, uint64_t ref_len,
                     const bsw_seed* seeds, int64_t n, const bsw_params* params,
                     bsw_seed_result* out);

/* Device-memory form: reads (reads_len bytes), read_off, ref, ref_rev,
 * seeds and out are device pointers; params is host memory.  ref_rev is
 * the reference reversed (ref_rev[i] = ref[ref_len - 1 - i]), which a
 * caller that extends many batches against one reference makes once; NULL
 * makes the library reverse ref into its arena on every call.  The reads
 * are reversed into the arena on every call.  Seeds, offsets and codes are
 * checked on the device before any result is written; a bad one makes the
 * call write nothing and return BSW_EINVAL naming the first bad seed (or
 * read).  stream and async as for bsw_extend_batch_device; between an
 * asynchronous call and bsw_ctx_wait the inputs must stay valid and
 * bsw_ctx_wait returns the status.  Every byte of reads and ref must be a
 * code 0..4.  Arena use per call: reads_len (+ ref_len without ref_rev)
 * bytes, 160 bytes per seed and the BSW pipeline's own workspace.  After
 * the call, bsw_ctx_last_timing gives [0] = the whole call, [1] = checks,
 * reversal and the left side, [2] = the right side, [3] = DP launches of
 * both sides; bsw_ctx_last_cells counts the cells of both sides;
 * bsw_ctx_last_kernels lists the right side's launches. */
int bsw_extend_seeds_device(bsw_ctx* ctx, const uint8_t* reads, uint64_t reads_len,
                            const uint64_t* read_off, int64_t n_reads,
                            const uint8_t* ref, const uint8_t* ref_rev, uint64_t ref_len,
                            const bsw_seed* seeds, int64_t n, const bsw_params* params,
                            bsw_seed_result* out, void* stream, int32_t async);

/* The filter after extending every seed (Sec. 5.3.2 extends all seeds of a
 * read first, removing the dependence between them, then drops the ones
 * the sequential mapper would not have extended).  A chain is a run of
 * consecutive seeds with the same read, in the order given (the mapper's
 * order, best seed first).  Walking a chain, a seed is dropped when the
 * extension of an earlier kept seed of the chain contains it both in the
 * read ([qbeg, qend) holds [qb, qe)) and in the reference ([rbeg, rend)
 * holds [rb, rb + qe - qb)); the first seed of a chain is kept.  seeds and
 * res (the results of bsw_extend_seeds*_device for those seeds) are device
 * arrays of n entries; keep (device, n bytes) receives 1 for a kept seed,
 * 0 for a dropped one.  stream and async as for bsw_extend_batch_device. */
int bsw_filter_seeds_device(bsw_ctx* ctx, const bsw_seed* seeds, int64_t n,
                            const bsw_seed_result* res, uint8_t* keep, void* stream,
                            int32_t async);

/* Autotuner of the seed driver: as bsw_ctx_tune, with whole seed calls
 * (arguments as bsw_extend_seeds_device, blocking, on the context's
 * stream) as the unit that is timed.  The winner is the launch shape of
 * both BSW passes of every later seed call of the context (pair batches
 * keep their own), stored in tune_cache under its own entry.  out3
 * (nullable) receives it as bsw_ctx_tune_info describes. */
int bsw_ctx_tune_seeds(bsw_ctx* ctx, const uint8_t* reads, uint64_t reads_len,
                       const uint64_t* read_off, int64_t n_reads,
                       const uint8_t* ref, const uint8_t* ref_rev, uint64_t ref_len,
                       const bsw_seed* seeds, int64_t n, const bsw_params* params,
                       bsw_seed_result* out, int32_t reps, double* best_ms,
                       int32_t out3[3]);

/* ------------------------------------------------------------------------
 * Suffix-array lookup (SAL, Sec. 4.5, Eq. (1)).  The seeding step finds,
 * for each seed, its SA interval: the rows of the index's sorted-suffix
 * order (Sec. 2.2) whose suffixes start with the seed.  SAL turns every row
 * i of an interval into the seed's coordinate in the indexed text,
 * j = S[i], read from the uncompressed suffix array kept in device memory
 * (8 bytes per text position: a human reference and its reverse complement,
 * 6.2 G positions, take about 50 GB, which one MI355X holds).
 * ---------------------------------------------------------------------- */

/* Rows [k, k + s) of the suffix array (16 bytes). */
typedef struct bsw_sa_interval {
  uint64_t k;
  uint64_t s;
} bsw_sa_interval;

/* Device form only (the suffix array stays resident): sa (sa_len entries),
 * iv (n intervals), out_off (n + 1 entries) and out_pos (out_cap entries)
 * are device pointers.  Interval m's coordinates S[k], ..., S[k + s - 1]
 * are written to out_pos[out_off[m] .. out_off[m + 1]), out_off[0] = 0, in
 * interval order.  Checks on the device: every interval lies inside the
 * suffix array (k + s <= sa_len) and holds at most 2^32 rows, and the total
 * fits out_cap (at most 2^40); a failed check
 * writes nothing and returns BSW_EINVAL naming the first bad interval, or
 * BSW_ETOOBIG with the total needed.  *total (host, nullable) receives the
 * number of coordinates (blocking calls; after an asynchronous call it is
 * out_off[n]).  stream and async as for bsw_extend_batch_device.
 * bsw_ctx_last_timing then gives [0] = the whole call, [1] = checks and the
 * offset scan, [2] = the gather, [3] = 0.  Arena use: 8 (n + 1) bytes, 8
 * bytes per 2,048 intervals and 8 bytes per 256 entries of out_cap.  n = 0
 * is a no-op (*total = 0). */
int bsw_sa_lookup_device(bsw_ctx* ctx, const int64_t* sa, uint64_t sa_len,
                         const bsw_sa_interval* iv, int64_t n, uint64_t* out_off,
                         int64_t* out_pos, uint64_t out_cap, uint64_t* total,
                         void* stream, int32_t async);

/* ------------------------------------------------------------------------
 * FM-index backward search (Sec. 4.1, Algorithms 1 and 2; the index layout
 * of Sec. 4.4).  The index covers a text T holding both strands (a
 * reference followed by its reverse complement), with the end marker $
 * after it.  Its occurrence table is cut into buckets of BSW_FM_ETA = 32
 * rows; each bucket is one 64-byte entry: the counts of A, C, G, T in the
 * BWT before the bucket, the bucket's 32 BWT symbols as bytes (0..3, 4 for
 * $, 5 past the last row) and 16 bytes of padding, so one entry is one
 * cache line.  O(c, t) = count[c] of entry t / 32 plus the occurrences of c
 * among the first t % 32 + 1 symbols of that entry (Algorithm 1).
 * ---------------------------------------------------------------------- */
#define BSW_FM_ETA 32

typedef struct bsw_fm_entry {
  uint32_t count[4];  /* occurrences of A, C, G, T in BWT rows before the bucket */
  uint8_t  bwt[32];   /* the bucket's BWT symbols                               */
  uint8_t  pad_[16];
} bsw_fm_entry;

typedef struct bsw_fm_meta {
  uint64_t rows;     /* |T| + 1 (rows of the BW matrix)                      */
  uint64_t C[4];     /* first row of the suffixes that start with A, C, G, T */
  uint64_t primary;  /* row whose suffix is all of T (its BWT symbol is $)   */
  uint64_t entries;  /* ceil(rows / 32)                                      */
} bsw_fm_meta;

/* Bi-interval of a pattern X (32 bytes): X occupies rows [k, k + s), its
 * reverse complement rows [l, l + s); matched = length of the longest
 * suffix of X that occurs in T.  k = l = s = 0 unless all of X occurs. */
typedef struct bsw_bi_interval {
  uint64_t k, l, s;
  int32_t matched;
  int32_t pad_;
} bsw_bi_interval;

/* Build the index on the host from T (n codes 0..3) and the suffix array of
 * T$ (n + 1 entries, a permutation of 0..n with sa[0] = n).  entries has
 * room for ceil((n + 1) / 32) entries; meta receives the rest.  Returns
 * BSW_EINVAL for a code > 3 or an entry of sa outside 0..n. */
int bsw_fm_build(const uint8_t* text, uint64_t n, const int64_t* sa, bsw_fm_entry* entries,
                 bsw_fm_meta* meta);

/* Backward search of n patterns (device memory): pattern m is
 * pat[pat_off[m] .. pat_off[m + 1]), codes 0..4 (an N ends the search);
 * entries is the index in device memory (meta->entries entries), meta host
 * memory.  Every pattern is extended from its last base to its first by the
 * bi-interval update of Algorithm 2, stopping when the interval empties;
 * out[m] receives its bi-interval.  stream and async as for
 * bsw_extend_batch_device.  bsw_ctx_last_timing [0] = the search kernel. */
int bsw_fm_backward_search_device(bsw_ctx* ctx, const bsw_fm_entry* entries,
                                  const bsw_fm_meta* meta, const uint8_t* pat,
                                  const uint64_t* pat_off, int64_t n, bsw_bi_interval* out,
                                  void* stream, int32_t async);

/* One SMEM of a read (32 bytes): read[start, end) occurs in T at the rows
 * of its bi-interval (k, l, s). */
typedef struct bsw_smem {
  uint32_t start, end;
  uint64_t k, l, s;
} bsw_smem;

/* Super-maximal exact matches (Sec. 2.3 SMEM step; Algorithms 3 and 4) of
 * n_reads reads against the index (device memory; meta host memory): read
 * r is reads[read_off[r] .. read_off[r + 1]), codes 0..4, at most max_len
 * bases.  For pivot x = 0, the matches through x are found by extending
 * X[x] forward while it occurs (keeping the bi-interval each time the
 * number of occurrences changes), then extending those backward, longest
 * first; a match that stops growing to the left and is contained in no
 * longer one is an SMEM.  The next pivot is the end of the longest forward
 * match (a pivot on an N moves on by one).  Every SMEM of a read is found
 * once.  The SMEMs of read r, in order of start, go to
 * out[read_off[r] - read_off[0] ...] (out has room for as many entries as
 * the reads have bases) and their number to counts[r].  A read longer than
 * max_len, offsets out of order or a code > 4 fail the call with nothing
 * written.  One read per lane, with as many lanes as the device holds at
 * once (at most one per read); arena use: 48 * max_len bytes per lane
 * (about 2.4 GB for 151-base reads on a full MI355X).  bsw_ctx_last_timing [0]
 * = the search kernel; bsw_ctx_last_cells = the extension steps run (two
 * index entries read each).  stream and async as for
 * bsw_extend_batch_device. */
int bsw_fm_smem_device(bsw_ctx* ctx, const bsw_fm_entry* entries, const bsw_fm_meta* meta,
                       const uint8_t* reads, const uint64_t* read_off, int64_t n_reads,
                       uint32_t max_len, bsw_smem* out, int32_t* counts, void* stream,
                       int32_t async);

/* Measured integer-VALU peak of a device: the rate that the extension
 * kernels' operation counts are compared with (they are integer max-plus
 * dynamic programming, so the vector ALU bounds them; Sec. 5.4.1 picks 8-
 * or 16-bit lanes to put more cells through it).  Every lane of a grid of
 * 8 waves per SIMD over every CU runs eight independent chains of one
 * instruction kind; *instr_per_s receives lane-instructions per second
 * (best of three timed runs after a warm-up), *ops_per_s (nullable) the
 * operations per second, two per lane-instruction for the packed 16-bit
 * kinds.  Blocking; allocates a small scratch buffer on the device.
 * Returns BSW_EINVAL for an unknown kind, BSW_EDEVICE if the device is
 * missing or a HIP call fails. */
enum {
  BSW_PEAK_ADD_U32 = 0,    /* v_add_u32                                    */
  BSW_PEAK_MAX3_I32 = 1,   /* v_max3_i32                                   */
  BSW_PEAK_PK_ADD_U16 = 2, /* v_pk_add_u16 (two 16-bit additions)          */
  BSW_PEAK_PK_MAX_I16 = 3  /* v_pk_max_i16 (two 16-bit maxima)             */
};
int bsw_valu_peak(int32_t device, int32_t kind, double* instr_per_s, double* ops_per_s);

/* Text of the calling thread's most recent error ("" if none). */
const char* bsw_last_error(void);

/* ABI version of the loaded library (BSW_ABI_VERSION). */
int bsw_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif
