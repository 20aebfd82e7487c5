// bsw_sal.cpp -- suffix-array lookup (bsw_sa_lookup_device, Sec. 4.5,
// Eq. (1)): checks, offset scan, tile map and gather on one stream, all on
// the device; the host only reads the status at the end.
#include <hip/hip_runtime.h>

#include <new>

#include "bsw_runtime.h"
#include "bsw_sal_internal.h"

namespace bsw {

struct SalState {
  DevBuf ws;                  // status, offsets, tile sums, tile map
  SalStatus* h_st = nullptr;  // pinned copy of the status
  hipEvent_t ev[3] = {};      // start, gather start, end
  uint64_t* total_out = nullptr;  // where a blocking call reports the total
};

void sal_state_free(SalState* s) {
  if (!s) return;
  s->ws.release();
  if (s->h_st) (void)hipHostFree(s->h_st);
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

int sal_state(bsw_ctx* c, SalState** out) {
  SalState*& s = ctx_sal_state(c);
  if (!s) {
    SalState* x = new (std::nothrow) SalState;
    if (!x) return set_error(BSW_ENOMEM, "out of host memory");
    x->ws.b = ctx_budget(c);
    bool ok = hipHostMalloc((void**)&x->h_st, sizeof(SalStatus), 0) == hipSuccess;
    for (auto& e : x->ev) ok = ok && hipEventCreate(&e) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      sal_state_free(x);
      return set_error(BSW_EDEVICE, "lookup set-up failed");
    }
    s = x;
  }
  *out = s;
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

// After the stream has passed a lookup: its status, total and timing.
int sal_done(bsw_ctx* c) {
  SalState* S = ctx_sal_state(c);
  const SalStatus& st = *S->h_st;
  if (st.bad)
    return set_error(BSW_EINVAL, "interval %llu leaves the suffix array (k + s > sa_len) "
                     "or holds more than 2^32 rows",
                     ~(unsigned long long)st.first_bad_inv);
  if (st.too_big)
    return set_error(BSW_ETOOBIG, "the intervals hold %llu rows, more than out_cap",
                     (unsigned long long)st.total);
  if (S->total_out) *S->total_out = st.total;
  double* t = ctx_timing(c);
  t[0] = elapsed(S->ev[0], S->ev[2]);
  t[1] = elapsed(S->ev[0], S->ev[1]);
  t[2] = elapsed(S->ev[1], S->ev[2]);
  t[3] = 0;
  ctx_set_cells(c, 0);
  return BSW_OK;
}

}  // namespace

extern "C" {

int bsw_sa_lookup_device(bsw_ctx* c, const int64_t* sa, uint64_t sa_len,
                         const bsw_sa_interval* iv, int64_t n, uint64_t* out_off,
                         int64_t* out_pos, uint64_t out_cap, uint64_t* total, void* stream,
                         int32_t async) {
  if (!c) return set_error(BSW_EINVAL, "ctx is NULL");
  if (int rc0 = ctx_check_idle(c)) return rc0;
  if (n < 0 || n > 0x7fffffffLL)
    return set_error(BSW_EINVAL, "n = %lld out of range", (long long)n);
  if (n == 0) {
    if (total) *total = 0;
    return BSW_OK;
  }
  if ((sa_len && !sa) || !iv || !out_off || (out_cap && !out_pos))
    return set_error(BSW_EINVAL, "a required device pointer is NULL");
  if (out_cap > (1ull << 40)) return set_error(BSW_EINVAL, "out_cap above 2^40");
  int rc = ctx_set_device(c);
  if (rc) return rc;
  SalState* S;
  if ((rc = sal_state(c, &S))) return rc;
  // workspace: status, offsets (n + 1), tile sums, tile map
  const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  const uint64_t ntiles = (out_cap + SAL_TILE - 1) / SAL_TILE;
  size_t o = 0;
  const size_t o_st = o; o = align_up(o + sizeof(SalStatus), 256);
  const size_t o_off = o; o = align_up(o + 8 * (size_t)(n + 1), 256);
  const size_t o_part = o; o = align_up(o + 8 * (size_t)nb, 256);
  const size_t o_map = o; o = align_up(o + 8 * (size_t)(ntiles + 1), 256);
  if ((rc = S->ws.ensure(o))) return rc;
  char* b = (char*)S->ws.p;
  SalStatus* st = (SalStatus*)(b + o_st);
  uint64_t* off = (uint64_t*)(b + o_off);
  uint64_t* part = (uint64_t*)(b + o_part);
  int64_t* map = (int64_t*)(b + o_map);
  hipStream_t s = stream ? (hipStream_t)stream : ctx_stream(c);
  S->total_out = async ? nullptr : total;
  HIPCHK(hipEventRecord(S->ev[0], s));
  launch_fill((uint32_t*)st, (int64_t)(sizeof(SalStatus) / 4), s);
  launch_iv_check(iv, n, sa_len, off, st, s);  // row counts, scanned in place
  launch_offset_scan(off, n, part, off, s);
  launch_sal_total(off, n, out_cap, st, s);
  launch_tile_map(off, n, st, map, s);
  HIPCHK(hipEventRecord(S->ev[1], s));
  // a persistent grid over the tiles: their number is known on the device
  launch_sal_gather(sa, iv, off, n, map, st, out_off, out_pos, 8 * 256, s);
  HIPCHK(hipMemcpyAsync(S->h_st, st, sizeof(SalStatus), hipMemcpyDeviceToHost, s));
  HIPCHK(hipEventRecord(S->ev[2], s));
  HIPCHK(hipGetLastError());
  if (async) {
    ctx_set_pending(c, s, sal_done);
    return BSW_OK;
  }
  HIPCHK(hipStreamSynchronize(s));
  return sal_done(c);
}

}  // extern "C"
