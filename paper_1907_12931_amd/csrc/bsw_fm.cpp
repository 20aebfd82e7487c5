// bsw_fm.cpp -- FM-index build (host) and backward search (device) of the
// C ABI: bsw_fm_build, bsw_fm_backward_search_device (Sec. 4.1-4.2, 4.4).
#include <hip/hip_runtime.h>

#include <new>
#include <vector>

#include "bsw_runtime.h"

namespace bsw {

void launch_fm_check(const uint64_t* off, int64_t n, Status* st, hipStream_t s);
void launch_fm_search(const bsw_fm_entry* E, const bsw_fm_meta& meta, const uint8_t* pat,
                      const uint64_t* off, int64_t n, const Status* st, bsw_bi_interval* out,
                      hipStream_t s);

void launch_smem_check(const uint64_t* off, int64_t n, uint32_t cap, Status* st,
                       hipStream_t s);
size_t smem_list_entry_bytes();
int fm_smem_blocks_per_cu();
void launch_fm_smem(const bsw_fm_entry* E, const bsw_fm_meta& meta, const uint8_t* reads,
                    const uint64_t* off, int64_t n, uint32_t cap, void* scratch,
                    unsigned blocks, Status* st, bsw_smem* out, int32_t* counts,
                    hipStream_t s);


struct FmState {
  DevBuf ws;               // status block, list scratch
  Status* h_st = nullptr;  // pinned copy
  hipEvent_t ev[2] = {};   // search start, end
};

void fm_state_free(FmState* s) {
  if (!s) return;
  s->ws.release();
  if (s->h_st) (void)hipHostFree(s->h_st);
  for (auto& e : s->ev)
    if (e) (void)hipEventDestroy(e);
  delete s;
}

}  // namespace bsw

using namespace bsw;

static_assert(sizeof(bsw_fm_entry) == 64, "one entry per 64-byte line");
static_assert(sizeof(bsw_bi_interval) == 32, "bsw_bi_interval layout");

namespace {

#define HIPCHK(expr)                                                          \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess)                                                     \
      return set_error(e_ == hipErrorOutOfMemory ? BSW_ENOMEM : BSW_EDEVICE,  \
                       "%s failed: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

int fm_state(bsw_ctx* c, FmState** out) {
  FmState*& s = ctx_fm_state(c);
  if (!s) {
    FmState* x = new (std::nothrow) FmState;
    if (!x) return set_error(BSW_ENOMEM, "out of host memory");
    x->ws.b = ctx_budget(c);
    bool ok = hipHostMalloc((void**)&x->h_st, sizeof(Status), 0) == hipSuccess;
    for (auto& e : x->ev) ok = ok && hipEventCreate(&e) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      fm_state_free(x);
      return set_error(BSW_EDEVICE, "FM search set-up failed");
    }
    s = x;
  }
  *out = s;
  return BSW_OK;
}

int fm_finish(bsw_ctx* c, const char* what) {
  FmState* S = ctx_fm_state(c);
  if (S->h_st->bad)
    return set_error(BSW_EINVAL, "%s %llu: offsets out of order, too long or a code > 4", what,
                     ~(unsigned long long)S->h_st->first_bad_inv);
  float ms = 0;
  if (hipEventElapsedTime(&ms, S->ev[0], S->ev[1]) != hipSuccess) {
    (void)hipGetLastError();
    ms = 0;
  }
  double* t = ctx_timing(c);
  t[0] = ms;
  t[1] = t[2] = t[3] = 0;
  ctx_set_cells(c, S->h_st->cls_cells[0]);
  return BSW_OK;
}

int fm_done(bsw_ctx* c) { return fm_finish(c, "pattern"); }
int smem_done(bsw_ctx* c) { return fm_finish(c, "read"); }

int check_meta(const bsw_fm_meta* meta) {
  if (meta->rows < 1 || meta->entries != (meta->rows + BSW_FM_ETA - 1) / BSW_FM_ETA ||
      meta->primary >= meta->rows || meta->C[0] != 1 || meta->rows > 0xffffffffull)
    return set_error(BSW_EINVAL, "meta does not describe an index built by bsw_fm_build");
  for (int k = 1; k < 4; ++k)
    if (meta->C[k] < meta->C[k - 1] || meta->C[k] > meta->rows)
      return set_error(BSW_EINVAL, "meta does not describe an index built by bsw_fm_build");
  return BSW_OK;
}

}  // namespace

extern "C" {

int bsw_fm_build(const uint8_t* text, uint64_t n, const int64_t* sa, bsw_fm_entry* E,
                 bsw_fm_meta* meta) {
  if ((n && !text) || !sa || !E || !meta) return set_error(BSW_EINVAL, "NULL argument");
  if (n >= 0xffffffffull) return set_error(BSW_EINVAL, "the text must be shorter than 2^32 - 1");
  const uint64_t rows = n + 1;
  uint64_t cnt[4] = {0, 0, 0, 0};
  for (uint64_t i = 0; i < n; ++i) {
    if (text[i] > 3) return set_error(BSW_EINVAL, "text[%llu] = %d is not a base code 0..3",
                                      (unsigned long long)i, text[i]);
    ++cnt[text[i]];
  }
  std::vector<bool> seen(rows, false);
  for (uint64_t r = 0; r < rows; ++r) {
    if (sa[r] < 0 || (uint64_t)sa[r] > n || seen[(size_t)sa[r]])
      return set_error(BSW_EINVAL, "sa is not a permutation of 0..%llu (row %llu)",
                       (unsigned long long)n, (unsigned long long)r);
    seen[(size_t)sa[r]] = true;
  }
  meta->rows = rows;
  meta->entries = (rows + BSW_FM_ETA - 1) / BSW_FM_ETA;
  meta->C[0] = 1;  // row 0 is the suffix $ alone
  for (int c = 1; c < 4; ++c) meta->C[c] = meta->C[c - 1] + cnt[c - 1];
  meta->primary = 0;
  uint32_t run[4] = {0, 0, 0, 0};
  for (uint64_t e = 0; e < meta->entries; ++e) {
    bsw_fm_entry& x = E[e];
    for (int c = 0; c < 4; ++c) x.count[c] = run[c];
    for (int j = 0; j < BSW_FM_ETA; ++j) {
      const uint64_t r = e * BSW_FM_ETA + (uint64_t)j;
      uint8_t v = 5;  // past the last row
      if (r < rows) {
        if (sa[r] == 0) {
          v = 4;
          meta->primary = r;
        } else {
          v = text[sa[r] - 1];
          ++run[v];
        }
      }
      x.bwt[j] = v;
    }
    for (auto& b : x.pad_) b = 0;
  }
  return BSW_OK;
}

int bsw_fm_backward_search_device(bsw_ctx* c, const bsw_fm_entry* E, const bsw_fm_meta* meta,
                                  const uint8_t* pat, const uint64_t* pat_off, int64_t n,
                                  bsw_bi_interval* out, void* stream, int32_t async) {
  if (!c) return set_error(BSW_EINVAL, "ctx is NULL");
  if (int rc0 = ctx_check_idle(c)) return rc0;
  if (n < 0 || n > 0x7fffffffLL)
    return set_error(BSW_EINVAL, "n = %lld out of range", (long long)n);
  if (n == 0) return BSW_OK;
  if (!E || !meta || !pat_off || !out)
    return set_error(BSW_EINVAL, "a required pointer is NULL");
  int rc = check_meta(meta);
  if (rc) return rc;
  if ((rc = ctx_set_device(c))) return rc;
  if (rc) return rc;
  FmState* S;
  if ((rc = fm_state(c, &S))) return rc;
  if ((rc = S->ws.ensure(sizeof(Status)))) return rc;
  Status* st = (Status*)S->ws.p;
  hipStream_t s = stream ? (hipStream_t)stream : ctx_stream(c);
  launch_fill((uint32_t*)st, (int64_t)(sizeof(Status) / 4), s);
  launch_fm_check(pat_off, n, st, s);
  if (pat) launch_codes(pat, pat_off, n, st, 0, s);
  HIPCHK(hipEventRecord(S->ev[0], s));
  launch_fm_search(E, *meta, pat, pat_off, n, st, out, s);
  HIPCHK(hipEventRecord(S->ev[1], s));
  HIPCHK(hipMemcpyAsync(S->h_st, st, sizeof(Status), hipMemcpyDeviceToHost, s));
  HIPCHK(hipGetLastError());
  if (async) {
    ctx_set_pending(c, s, fm_done);
    return BSW_OK;
  }
  HIPCHK(hipStreamSynchronize(s));
  return fm_done(c);
}

int bsw_fm_smem_device(bsw_ctx* c, const bsw_fm_entry* E, const bsw_fm_meta* meta,
                       const uint8_t* reads, const uint64_t* read_off, int64_t n,
                       uint32_t max_len, bsw_smem* out, int32_t* counts, void* stream,
                       int32_t async) {
  if (!c) return set_error(BSW_EINVAL, "ctx is NULL");
  if (int rc0 = ctx_check_idle(c)) return rc0;
  if (n < 0 || n > 0x7fffffffLL)
    return set_error(BSW_EINVAL, "n_reads = %lld out of range", (long long)n);
  if (n == 0) return BSW_OK;
  if (!E || !meta || !read_off || !counts || (max_len && (!reads || !out)))
    return set_error(BSW_EINVAL, "a required pointer is NULL");
  if (max_len > BSW_MAX_LEN) return set_error(BSW_EINVAL, "max_len above %d", BSW_MAX_LEN);
  int rc = check_meta(meta);
  if (rc) return rc;
  if ((rc = ctx_set_device(c))) return rc;
  FmState* S;
  if ((rc = fm_state(c, &S))) return rc;
  // as many lanes as can be resident at once (the search hides its latency
  // with them), but no more than one per read; each has its own list slot
  const size_t resident = (size_t)fm_smem_blocks_per_cu() * ctx_num_cu(c);
  const size_t blocks = std::max<size_t>(1, std::min(resident, (size_t)(n + 255) / 256));
  const size_t lanes = blocks * 256;
  const size_t cap = max_len ? max_len : 1;
  const size_t o_scr = (sizeof(Status) + 255) / 256 * 256;  // lists after the status
  if ((rc = S->ws.ensure(o_scr + lanes * 2 * cap * smem_list_entry_bytes()))) return rc;
  Status* st = (Status*)S->ws.p;
  hipStream_t s = stream ? (hipStream_t)stream : ctx_stream(c);
  launch_fill((uint32_t*)st, (int64_t)(sizeof(Status) / 4), s);
  launch_smem_check(read_off, n, max_len, st, s);
  if (reads) launch_codes(reads, read_off, n, st, 0, s);
  HIPCHK(hipEventRecord(S->ev[0], s));
  launch_fm_smem(E, *meta, reads, read_off, n, (uint32_t)cap, (char*)S->ws.p + o_scr,
                 (unsigned)blocks, st, out, counts, s);
  HIPCHK(hipEventRecord(S->ev[1], s));
  HIPCHK(hipMemcpyAsync(S->h_st, st, sizeof(Status), hipMemcpyDeviceToHost, s));
  HIPCHK(hipGetLastError());
  if (async) {
    ctx_set_pending(c, s, smem_done);
    return BSW_OK;
  }
  HIPCHK(hipStreamSynchronize(s));
  return smem_done(c);
}

}  // extern "C"
