// bsw_seeds.cpp -- read-level seed driver (bsw_extend_seeds*): each seed is
// extended to the left on the reversed read prefix, the end kept by the
// end-bonus rule, then to the right from the kept score (Sec. 2; Sec.
// 5.3.2: every seed is extended).  Both sides run the BSW pipeline as it
// is, with pair tables that index the caller's reads and reference (right)
// or their reversed copies (left); the kernels of bsw_seed_kernels.hip
// build the tables and read the results.  Everything after the argument
// checks runs on the device, on one stream, with no host round trip other
// than the plain path's own.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "bsw_runtime.h"
#include "bsw_seed_internal.h"

namespace bsw {

struct SeedState {
  DevBuf ws;     // pair tables, results of both sides, status blocks
  DevBuf rev;    // reversed reads, then (without a caller's copy) reference
  DevBuf stage;  // host form: reads, reference, offsets, seeds, results
  Status* h_sts = nullptr;  // pinned copy of the call's status blocks
  hipEvent_t ev[3] = {};    // start, left side done, end
  int left_launches = 0;    // DP launches of the left call
};

void seed_state_free(SeedState* s) {
  if (!s) return;
  s->ws.release();
  s->rev.release();
  s->stage.release();
  if (s->h_sts) (void)hipHostFree(s->h_sts);
  for (auto& e : s->ev)
    if (e) (void)hipEventDestroy(e);
  delete s;
}

}  // namespace bsw

using namespace bsw;

namespace {

#define HIPCHK(expr)                                                          \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess)                                                     \
      return set_error(e_ == hipErrorOutOfMemory ? BSW_ENOMEM : BSW_EDEVICE,  \
                       "%s failed: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int seed_state(bsw_ctx* c, SeedState** out) {
  SeedState*& s = ctx_seed_state(c);
  if (!s) {
    SeedState* x = new (std::nothrow) SeedState;
    if (!x) return set_error(BSW_ENOMEM, "out of host memory");
    for (DevBuf* d : {&x->ws, &x->rev, &x->stage}) d->b = ctx_budget(c);
    bool ok = hipHostMalloc((void**)&x->h_sts, sizeof(Status) * ST_COUNT, 0) == hipSuccess;
    for (auto& e : x->ev) ok = ok && hipEventCreate(&e) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      seed_state_free(x);
      return set_error(BSW_EDEVICE, "seed driver set-up failed");
    }
    s = x;
  }
  *out = s;
  return BSW_OK;
}

// Workspace of a call with n seeds (byte offsets from the base).
struct SeedLayout {
  size_t sts, offs, tab[8], lh0, rh0, lres, rres, part, total;
};

SeedLayout seed_layout(int64_t n) {
  SeedLayout L;
  size_t o = 0;
  auto take = [&o](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L.sts = take(sizeof(Status) * ST_COUNT);
  L.offs = take(4 * sizeof(uint64_t));
  for (size_t& t : L.tab) t = take(8 * (size_t)n);
  L.lh0 = take(4 * (size_t)n);
  L.rh0 = take(4 * (size_t)n);
  L.lres = take(sizeof(bsw_result) * (size_t)n);
  L.rres = take(sizeof(bsw_result) * (size_t)n);
  L.part = take(sizeof(SeedPart) * (size_t)n);
  L.total = o;
  return L;
}

struct SeedArgs {
  const uint8_t* reads;
  uint64_t reads_len;
  const uint64_t* read_off;
  int64_t n_reads;
  const uint8_t* ref;
  const uint8_t* ref_rev;
  uint64_t ref_len;
  const bsw_seed* seeds;
  int64_t n;
  bsw_seed_result* out;
};

// Both BSW passes of a seed call use the context's seed-driver shape.
struct SeedKind {
  bsw_ctx* c;
  explicit SeedKind(bsw_ctx* cc) : c(cc) { ctx_set_kind(c, KIND_SEEDS); }
  ~SeedKind() { ctx_set_kind(c, KIND_PAIRS); }
};

// Enqueue one seed call on stream s (n >= 1; params already loaded).
int seeds_enqueue(bsw_ctx* c, SeedState* S, const SeedArgs& a, const bsw_params& P,
                  hipStream_t s) {
  const SeedKind kind(c);
  const SeedLayout L = seed_layout(a.n);
  const size_t rr = align_up(a.reads_len + 1, 256);
  int rc;
  if ((rc = S->ws.ensure(L.total))) return rc;
  if ((rc = S->rev.ensure(rr + (a.ref_rev ? 0 : a.ref_len + 1)))) return rc;
  char* b = (char*)S->ws.p;
  Status* sts = (Status*)(b + L.sts);
  uint64_t* offs = (uint64_t*)(b + L.offs);
  SeedTables T;
  uint64_t** tabs[8] = {&T.lq0, &T.lq1, &T.lt0, &T.lt1, &T.rq0, &T.rq1, &T.rt0, &T.rt1};
  for (int i = 0; i < 8; ++i) *tabs[i] = (uint64_t*)(b + L.tab[i]);
  T.lh0 = (int32_t*)(b + L.lh0);
  T.rh0 = (int32_t*)(b + L.rh0);
  bsw_result* lres = (bsw_result*)(b + L.lres);
  bsw_result* rres = (bsw_result*)(b + L.rres);
  SeedPart* part = (SeedPart*)(b + L.part);
  uint8_t* rreads = (uint8_t*)S->rev.p;
  const uint8_t* rref = a.ref_rev ? a.ref_rev : rreads + rr;

  HIPCHK(hipEventRecord(S->ev[0], s));
  launch_fill((uint32_t*)sts, (int64_t)(sizeof(Status) * ST_COUNT / 4), s);
  launch_seed_offsets(offs, a.reads_len, a.ref_len, s);
  launch_codes(a.reads, offs, 1, &sts[ST_READS], a.reads_len, s);
  launch_codes(a.ref, offs + 2, 1, &sts[ST_REF], a.ref_len, s);
  launch_seed_setup(a.seeds, a.n, a.read_off, a.n_reads, a.reads_len, a.ref_len, P.w, T, sts,
                    s);
  launch_reverse(a.reads, rreads, a.reads_len, s);
  if (!a.ref_rev) launch_reverse(a.ref, (uint8_t*)rref, a.ref_len, s);
  HIPCHK(hipGetLastError());
  const Args left = {a.n, rreads, T.lq0, rref, T.lt0, T.lh0, nullptr, 1, lres, nullptr,
                     T.lq1, T.lt1, true};
  if ((rc = ctx_enqueue_eager(c, left, s))) return rc;
  S->left_launches = ctx_launches(c);
  launch_seed_mid(a.seeds, a.n, lres, ctx_status_dev(c), &sts[ST_LEFT], P.end_bonus, T, part,
                  sts, s);
  HIPCHK(hipEventRecord(S->ev[1], s));
  const Args right = {a.n, a.reads, T.rq0, a.ref, T.rt0, T.rh0, nullptr, 1, rres, nullptr,
                      T.rq1, T.rt1, true};
  if ((rc = ctx_enqueue_eager(c, right, s))) return rc;
  launch_seed_finish(a.n, part, rres, sts, ctx_status_dev(c), P.end_bonus, a.out, s);
  HIPCHK(hipMemcpyAsync(S->h_sts, sts, sizeof(Status) * ST_COUNT, hipMemcpyDeviceToHost, s));
  HIPCHK(hipEventRecord(S->ev[2], s));
  HIPCHK(hipGetLastError());
  return BSW_OK;
}

float elapsed(hipEvent_t x, hipEvent_t y) {
  float ms = 0;
  if (hipEventElapsedTime(&ms, x, y) != hipSuccess) {
    (void)hipGetLastError();
    ms = 0;
  }
  return ms;
}

// After the stream has passed a seed call: its checks in the order they
// ran, then the right call's own status, timing and cells.
int seed_done(bsw_ctx* c) {
  SeedState* S = ctx_seed_state(c);
  const Status* st = S->h_sts;
  auto idx = [&](int i) { return ~(unsigned long long)st[i].first_bad_inv; };
  if (st[ST_READS].bad) return set_error(BSW_EINVAL, "a read byte is not a code 0..4");
  if (st[ST_REF].bad) return set_error(BSW_EINVAL, "a reference byte is not a code 0..4");
  if (st[ST_SEED].bad)
    return set_error(BSW_EINVAL, "seed %llu is invalid (read index, interval, h0, "
                     "reference range, or a window longer than %d)", idx(ST_SEED), BSW_MAX_LEN);
  if (st[ST_LEFT].bad)
    return set_error(BSW_EINVAL, "seed %llu: its left pair was rejected", idx(ST_LEFT));
  if (st[ST_H1].bad)
    return set_error(BSW_EINVAL, "seed %llu: the score after the left side exceeds %d",
                     idx(ST_H1), BSW_MAX_H0);
  const int rc = ctx_finish(c);
  if (rc) {
    const std::string why = bsw_last_error();
    return set_error(rc, "right side: %s", why.c_str());
  }
  double* t = ctx_timing(c);
  t[0] = elapsed(S->ev[0], S->ev[2]);
  t[1] = elapsed(S->ev[0], S->ev[1]);
  t[2] = elapsed(S->ev[1], S->ev[2]);
  t[3] += S->left_launches;
  unsigned long long left_cells = 0;
  for (int k = 0; k <= NCLS; ++k) left_cells += st[ST_LEFT].cls_cells[k];
  ctx_add_cells(c, left_cells);
  return BSW_OK;
}

// Checks of the device form's host-side arguments.
int check_device_args(bsw_ctx* c, const uint8_t* reads, uint64_t reads_len,
                      const uint64_t* read_off, int64_t n_reads, const uint8_t* ref,
                      uint64_t ref_len, const bsw_seed* seeds, int64_t n,
                      const bsw_seed_result* out) {
  if (!c) return set_error(BSW_EINVAL, "ctx is NULL");
  if (int rc0 = ctx_check_idle(c)) return rc0;
  if (n < 0 || n > 0x7fffffffLL)
    return set_error(BSW_EINVAL, "n = %lld out of range", (long long)n);
  if (n == 0) return BSW_OK;
  if (n_reads < 1 || n_reads > 0x7fffffffLL)
    return set_error(BSW_EINVAL, "n_reads = %lld out of range", (long long)n_reads);
  if ((reads_len && !reads) || !read_off || (ref_len && !ref) || !seeds || !out)
    return set_error(BSW_EINVAL, "a required device pointer is NULL");
  if (reads_len > (1ull << 48) || ref_len > (1ull << 48))
    return set_error(BSW_EINVAL, "reads_len or ref_len above 2^48");
  return BSW_OK;
}

struct TuneRun {
  SeedState* S;
  SeedArgs a;
  bsw_params P;
};

// One whole blocking seed call (the tuner's unit of work).
int tune_run(bsw_ctx* c, void* arg) {
  const TuneRun& r = *(const TuneRun*)arg;
  const hipStream_t s = ctx_stream(c);
  int rc = seeds_enqueue(c, r.S, r.a, r.P, s);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(s));
  return seed_done(c);
}

}  // namespace

extern "C" {

int bsw_ctx_tune_seeds(bsw_ctx* c, const uint8_t* reads, uint64_t reads_len,
                       const uint64_t* read_off, int64_t n_reads, const uint8_t* ref,
                       const uint8_t* ref_rev, uint64_t ref_len, const bsw_seed* seeds,
                       int64_t n, const bsw_params* params, bsw_seed_result* out,
                       int32_t reps, double* best_ms, int32_t out3[3]) {
  int rc = check_device_args(c, reads, reads_len, read_off, n_reads, ref, ref_len, seeds, n,
                             out);
  if (rc) return rc;
  if (n < 1) return set_error(BSW_EINVAL, "tuning needs at least one seed");
  if (reps < 1 || reps > 100) return set_error(BSW_EINVAL, "reps must be 1..100");
  if ((rc = ctx_set_params(c, params, 1))) return rc;
  if ((rc = ctx_set_device(c))) return rc;
  TuneRun r;
  if ((rc = seed_state(c, &r.S))) return rc;
  r.a = {reads, reads_len, read_off, n_reads, ref, ref_rev, ref_len, seeds, n, out};
  r.P = *params;
  if ((rc = ctx_tune_shapes(c, KIND_SEEDS, 1, reps, tune_run, &r, best_ms))) return rc;
  if (out3) {
    const Tune t = ctx_shape(c, KIND_SEEDS);
    out3[0] = t.nside;
    out3[1] = t.occ8;
    out3[2] = t.spec16;
  }
  return BSW_OK;
}

int bsw_extend_seeds_device(bsw_ctx* c, const uint8_t* reads, uint64_t reads_len,
                            const uint64_t* read_off, int64_t n_reads, const uint8_t* ref,
                            const uint8_t* ref_rev, uint64_t ref_len, const bsw_seed* seeds,
                            int64_t n, const bsw_params* params, bsw_seed_result* out,
                            void* stream, int32_t async) {
  int rc = check_device_args(c, reads, reads_len, read_off, n_reads, ref, ref_len, seeds, n,
                             out);
  if (rc || n == 0) return rc;
  rc = ctx_set_params(c, params, 1);
  if (rc) return rc;
  if ((rc = ctx_set_device(c))) return rc;
  SeedState* S;
  if ((rc = seed_state(c, &S))) return rc;
  hipStream_t s = stream ? (hipStream_t)stream : ctx_stream(c);
  const SeedArgs a = {reads, reads_len, read_off, n_reads, ref, ref_rev, ref_len, seeds, n, out};
  if ((rc = seeds_enqueue(c, S, a, *params, s))) return rc;
  if (async) {
    ctx_set_pending(c, s, seed_done);
    return BSW_OK;
  }
  HIPCHK(hipStreamSynchronize(s));
  return seed_done(c);
}

// The filter has no status to read back: nothing is left to do once its
// stream has drained.
static int filter_done(bsw_ctx*) { return BSW_OK; }

int bsw_filter_seeds_device(bsw_ctx* c, const bsw_seed* seeds, int64_t n,
                            const bsw_seed_result* res, uint8_t* keep, void* stream,
                            int32_t async) {
  if (!c) return set_error(BSW_EINVAL, "ctx is NULL");
  if (int rc0 = ctx_check_idle(c)) return rc0;
  if (n < 0) return set_error(BSW_EINVAL, "n = %lld out of range", (long long)n);
  if (n == 0) return BSW_OK;
  if (!seeds || !res || !keep) return set_error(BSW_EINVAL, "a required device pointer is NULL");
  int rc = ctx_set_device(c);
  if (rc) return rc;
  hipStream_t s = stream ? (hipStream_t)stream : ctx_stream(c);
  launch_seed_filter(seeds, n, res, keep, s);
  HIPCHK(hipGetLastError());
  if (async) {
    ctx_set_pending(c, s, filter_done);
    return BSW_OK;
  }
  HIPCHK(hipStreamSynchronize(s));
  return BSW_OK;
}

int bsw_extend_seeds(bsw_ctx* c, const uint8_t* reads, const uint64_t* read_off,
                     int64_t n_reads, const uint8_t* ref, uint64_t ref_len,
                     const bsw_seed* seeds, int64_t n, const bsw_params* params,
                     bsw_seed_result* out) {
  if (!c) return set_error(BSW_EINVAL, "ctx is NULL");
  if (int rc0 = ctx_check_idle(c)) return rc0;
  if (int rc0 = ctx_check_idle(c)) return rc0;
  if (n < 0 || n > 0x7fffffffLL)
    return set_error(BSW_EINVAL, "n = %lld out of range", (long long)n);
  if (n == 0) return BSW_OK;
  if (n_reads < 1 || n_reads > 0x7fffffffLL)
    return set_error(BSW_EINVAL, "n_reads = %lld out of range", (long long)n_reads);
  if (!read_off || !seeds || !out || (ref_len && !ref))
    return set_error(BSW_EINVAL, "a required pointer is NULL");
  if (ref_len > (1ull << 48)) return set_error(BSW_EINVAL, "ref_len above 2^48");
  int rc = ctx_set_params(c, params, 1);
  if (rc) return rc;
  if (const int64_t i = first_bad_read(read_off, n_reads); i >= 0)
    return set_error(BSW_EINVAL, "read %lld: bad offsets or length > %d", (long long)i,
                     BSW_MAX_LEN);
  const uint64_t r0 = read_off[0], reads_len = read_off[n_reads] - r0;
  if (reads_len && !reads) return set_error(BSW_EINVAL, "reads is NULL");
  if (const int64_t k = first_bad_seed(seeds, n, read_off, n_reads, ref_len, params->w); k >= 0)
    return set_error(BSW_EINVAL, "seed %lld is invalid (read index, interval, h0, "
                     "reference range, or a window longer than %d)", (long long)k,
                     BSW_MAX_LEN);
  if ((rc = ctx_set_device(c))) return rc;
  SeedState* S;
  if ((rc = seed_state(c, &S))) return rc;
  // stage: reads, reference, rebased read offsets, seeds, results
  size_t o = 0;
  const size_t o_reads = o; o = align_up(o + reads_len + 1, 256);
  const size_t o_ref = o; o = align_up(o + ref_len + 1, 256);
  const size_t o_off = o; o = align_up(o + 8 * (size_t)(n_reads + 1), 256);
  const size_t o_seed = o; o = align_up(o + sizeof(bsw_seed) * (size_t)n, 256);
  const size_t o_out = o; o = align_up(o + sizeof(bsw_seed_result) * (size_t)n, 256);
  if ((rc = S->stage.ensure(o))) return rc;
  char* d = (char*)S->stage.p;
  std::vector<uint64_t> off((size_t)n_reads + 1);
  for (int64_t i = 0; i <= n_reads; ++i) off[i] = read_off[i] - r0;
  hipStream_t s = ctx_stream(c);
  if (reads_len) HIPCHK(hipMemcpyAsync(d + o_reads, reads + r0, reads_len, hipMemcpyHostToDevice, s));
  if (ref_len) HIPCHK(hipMemcpyAsync(d + o_ref, ref, ref_len, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(d + o_off, off.data(), 8 * off.size(), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(d + o_seed, seeds, sizeof(bsw_seed) * (size_t)n, hipMemcpyHostToDevice,
                        s));
  const SeedArgs a = {(const uint8_t*)(d + o_reads), reads_len, (const uint64_t*)(d + o_off),
                      n_reads, (const uint8_t*)(d + o_ref), nullptr, ref_len,
                      (const bsw_seed*)(d + o_seed), n, (bsw_seed_result*)(d + o_out)};
  if ((rc = seeds_enqueue(c, S, a, *params, s))) return rc;
  HIPCHK(hipStreamSynchronize(s));
  if ((rc = seed_done(c))) return rc;
  HIPCHK(hipMemcpyAsync(out, d + o_out, sizeof(bsw_seed_result) * (size_t)n,
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return BSW_OK;
}

}  // extern "C"
