// bsw_runtime.h -- host-side internals shared by the runtime (bsw_host.cpp)
// and the serving loop (bsw_server.cpp).  Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "../../include/bsw.h"
#include "bsw_hostutil.h"
#include "bsw_internal.h"

namespace bsw {

// Device pointers of one call.
struct Args {
  int64_t n;
  const uint8_t* q;
  const uint64_t* q_off;
  const uint8_t* t;
  const uint64_t* t_off;
  const int32_t* h0;
  const uint8_t* pid;
  int32_t n_params;
  bsw_result* out;
  bsw_diag* diag;
  // end offsets (pair k ends at q_end[k]); null = q_off + 1
  const uint64_t* q_end;
  const uint64_t* t_end;
  bool codes_checked;  // the sequence bytes were validated beforehand
};

// Workload kinds with a shape of their own: pair batches, and the BSW
// passes of the read-level seed driver (many short, similar pairs).
enum { KIND_PAIRS = 0, KIND_SEEDS = 1, NKIND = 2 };

// Set the calling thread's error text; returns code.
int set_error(int code, const char* fmt, ...);

// Device bytes a context may hold (0 = no cap) and holds.
struct Budget {
  size_t limit = 0;
  size_t used = 0;
};

// A growable device buffer, counted against its context's budget.
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  Budget* b = nullptr;
  int ensure(size_t bytes) {
    if (bytes <= cap) return BSW_OK;
    // grow by at least half, so that slowly rising sizes reallocate (and
    // synchronise the device in hipFree) only a few times
    const size_t want = std::max(std::max(bytes, cap + cap / 2), (size_t)1 << 20);
    if (b && b->limit && b->used - cap + want > b->limit)
      return set_error(BSW_ETOOBIG, "the call needs %zu more device bytes than the "
                       "context's budget of %zu", b->used - cap + want - b->limit, b->limit);
    release();
    if (hipMalloc(&p, want) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      return set_error(BSW_ENOMEM, "device allocation of %zu bytes failed", want);
    }
    cap = want;
    if (b) b->used += cap;
    return BSW_OK;
  }
  void release() {
    if (p) (void)hipFree(p);
    if (b) b->used -= cap;
    p = nullptr;
    cap = 0;
  }
};

// Load a context's scoring table (validated).
int ctx_set_params(bsw_ctx* c, const bsw_params* params, int32_t n_params);
// Side streams the batched path spreads the classes over (0: all classes
// on the call's stream; the context then keeps to one hardware queue).
void ctx_set_side_streams(bsw_ctx* c, int nside);
// Allocate a context's device buffers for calls of up to n pairs with its
// current scoring table, so that such calls allocate nothing.
int ctx_reserve(bsw_ctx* c, int64_t n, int32_t n_params);
// Enqueue one call on stream s (the context's path), ending with the copy
// of its status to the host.
int ctx_enqueue(bsw_ctx* c, const Args& a, hipStream_t s);
// After the stream has passed the call: its status, then its timing.
int ctx_finish(bsw_ctx* c);
// Band cells settled by the last finished call.
unsigned long long ctx_last_cells(const bsw_ctx* c);
hipStream_t ctx_stream(const bsw_ctx* c);
// As ctx_enqueue, but never captured into or replayed from a graph (for
// drivers that run the pipeline several times per call on other buffers).
int ctx_enqueue_eager(bsw_ctx* c, const Args& a, hipStream_t s);
// Device status block of the last enqueued call (valid until the next).
Status* ctx_status_dev(const bsw_ctx* c);
Budget* ctx_budget(bsw_ctx* c);
// DP launches the last enqueued call made.
int ctx_launches(const bsw_ctx* c);
// bsw_ctx_last_timing's four values, and the band cells bsw_ctx_last_cells
// reports, of the last finished call (a driver adjusts them after
// ctx_finish).
double* ctx_timing(bsw_ctx* c);
void ctx_add_cells(bsw_ctx* c, unsigned long long cells);
void ctx_set_cells(bsw_ctx* c, unsigned long long cells);
int ctx_set_device(bsw_ctx* c);
int ctx_num_cu(const bsw_ctx* c);
// Mark the context as having an asynchronous call in flight on s whose
// completion is checked by done (bsw_ctx_wait calls it).
void ctx_set_pending(bsw_ctx* c, hipStream_t s, int (*done)(bsw_ctx*));
// BSW_EBUSY (with the message set) while an asynchronous call is pending:
// every entry point that enqueues work on a context checks this first, so
// that a new call never rewrites the pinned tables, status or graph that the
// pending call's queued work still reads.
int ctx_check_idle(const bsw_ctx* c);

// Kind of the calls enqueued from now on (the shape they use and the tune
// cache entry it comes from).
void ctx_set_kind(bsw_ctx* c, int kind);
// Autotune the shape of one kind: for every candidate, run(c, arg) makes
// one whole blocking call (reps + 1 times, the first untimed); the score is
// the median of the calls' device time (bsw_ctx_last_timing [0]); another
// shape must beat the default by more than 1%.  The winner becomes the
// kind's shape and is stored in the tune cache.  n_params: size of the
// loaded scoring table.
int ctx_tune_shapes(bsw_ctx* c, int kind, int n_params, int reps,
                    int (*run)(bsw_ctx*, void*), void* arg, double* best_ms);
Tune ctx_shape(const bsw_ctx* c, int kind);

// State of the read-level seed driver, owned by the context (created on
// first use, released with the context).
struct SeedState;
SeedState*& ctx_seed_state(bsw_ctx* c);
void seed_state_free(SeedState* s);
// State of the suffix-array lookup, likewise.
struct SalState;
SalState*& ctx_sal_state(bsw_ctx* c);
void sal_state_free(SalState* s);
// State of the FM-index search, likewise.
struct FmState;
FmState*& ctx_fm_state(bsw_ctx* c);
void fm_state_free(FmState* s);

void launch_fill(uint32_t* p, int64_t nwords, hipStream_t s);
void launch_codes(const uint8_t* seq, const uint64_t* off, int64_t n, Status* st,
                  uint64_t bytes, hipStream_t s);
// One byte range a serving batch copies from host memory the device can
// read (pinned, mapped) into its arena (see k_gather); chunk0 is the first
// 4 KiB chunk of the range in the batch's list of chunks.
struct CopySeg {
  const uint8_t* src;
  uint8_t* dst;
  unsigned long long bytes;
  unsigned long long chunk0;
};

// Copy the byte ranges segs[0 .. ns) (nchunks 4 KiB chunks in all) from
// mapped host memory to the device.
void launch_gather(const CopySeg* segs, int ns, unsigned long long nchunks, hipStream_t s);
// Serving batches: flag (bad[a] = ~(first bad pair), else 0) every request
// of the table with a sequence byte > 4, then gather the pairs of the
// unflagged requests (a flagged request's pairs get no bytes).
void launch_req_codes(const ReqSlice* tab, int m, int64_t n, const uint8_t* base,
                      unsigned long long* bad, hipStream_t s);
void launch_assemble(const ReqSlice* tab, int m, int64_t n, uint64_t* qb, uint64_t* qe,
                     uint64_t* tb, uint64_t* te, int32_t* h0, uint8_t* pid,
                     const unsigned long long* bad, hipStream_t s);

}  // namespace bsw
