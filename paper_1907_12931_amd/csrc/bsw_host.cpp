// bsw_host.cpp -- host runtime and C ABI of libbsw.so.
//
// A context owns one device arena (grown on demand and reused across
// batches, the paper's "few large buffers allocated once", Sec. 3.2), a
// stream, timing events and pinned staging for the small per-call tables.
// Every batch runs the same device pipeline: prepare + bin (counting sort
// by kernel class and length, Sec. 5.3.1), then one DP kernel per
// non-empty class.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/bsw.h"
#include "bsw_internal.h"

namespace bsw {
size_t lane_lds_per_wave(int cls);
int lane_waves_per_block(int cls);
hipError_t lane_setup(int cls, bool persist);
int lane_blocks_per_cu(int cls, bool persist, size_t lds);
int lane8_ring_chunks(int cls, int wmax);
size_t lane8_qtile_words(int cls);
size_t lane_chunk_row_bytes(int cls);
void launch_fill(uint32_t* p, int64_t nwords, hipStream_t s);
void launch_prep(int64_t n, const uint8_t* q, const uint8_t* t, const uint64_t* q_off,
                 const uint64_t* t_off, const int32_t* h0, const uint8_t* pid,
                 int n_params, const KParams* kp, int min_bits, int force_mode,
                 uint32_t* keys, uint32_t* hist, Status* st, hipStream_t s);
void launch_codes(const uint8_t* seq, const uint64_t* off, int64_t n, Status* st,
                  hipStream_t s);
void launch_scan(const uint32_t* hist, uint32_t* cursor, long long* cls_range,
                 hipStream_t s);
void launch_scatter(int64_t n, const uint64_t* q_off, const uint64_t* t_off,
                    const int32_t* h0, const uint8_t* pid, const uint32_t* keys,
                    uint32_t* cursor, PairDesc* desc, const Status* st,
                    hipStream_t s);
void launch_lane(int cls, bool persist, unsigned blocks, const PairDesc* desc,
                 const long long* range, const uint8_t* q, const uint8_t* t,
                 const KParams* kp, bsw_result* out, bsw_diag* diag,
                 uint32_t* tile_ctr, const Status* st, uint32_t* qtiles,
                 PairDesc* ovf, long long* ovf_count, int ring, bool sym,
                 unsigned long long* cls_cells, hipStream_t s);
void launch_long(const PairDesc* desc, const long long* range, const uint8_t* q,
                 const uint8_t* t, const KParams* kp, bsw_result* out,
                 bsw_diag* diag, uint32_t* ctr, int2* gbuf, uint8_t* gq,
                 const Status* st, unsigned long long* cls_cells, hipStream_t s);
}  // namespace bsw

using namespace bsw;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                          \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess)                                                     \
      return fail(e_ == hipErrorOutOfMemory ? BSW_ENOMEM : BSW_EDEVICE,       \
                  "%s failed: %s", #expr, hipGetErrorString(e_));             \
  } while (0)

// A growable device buffer.
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  int ensure(size_t bytes) {
    if (bytes <= cap) return BSW_OK;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    size_t want = std::max(bytes, (size_t)1 << 20);
    if (hipMalloc(&p, want) != hipSuccess) {
      p = nullptr;
      return fail(BSW_ENOMEM, "device allocation of %zu bytes failed", want);
    }
    cap = want;
    return BSW_OK;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Workspace carve-up for n pairs.
struct Layout {
  size_t keys, desc, ovf, ovf2, hist, cursor, cls_range, status, ctr, zero_beg, zero_end,
      total;
};

constexpr int NCTR = NCLS + 3;  // one tile counter per class, two reruns, spare

Layout layout_for(int64_t n) {
  Layout L;
  size_t o = 0;
  // zeroed block first: histogram, status, counters
  L.zero_beg = o;
  L.hist = o;
  o = align_up(o + (size_t)NBINS * 4, 256);
  L.status = o;
  o = align_up(o + sizeof(Status), 256);
  L.ctr = o;
  o = align_up(o + (size_t)NCTR * 4, 256);
  L.zero_end = o;
  L.cursor = o;
  o = align_up(o + (size_t)NBINS * 4, 256);
  L.cls_range = o;
  o = align_up(o + (size_t)NCLS * 16, 256);
  L.keys = o;
  o = align_up(o + (size_t)n * 4, 256);
  L.desc = o;
  o = align_up(o + (size_t)n * sizeof(PairDesc), 256);
  L.ovf = o;
  o = align_up(o + (size_t)n * sizeof(PairDesc), 256);
  L.ovf2 = o;
  o = align_up(o + (size_t)n * sizeof(PairDesc), 256);
  L.total = o;
  return L;
}

int check_params(const bsw_params* params, int32_t n_params) {
  if (!params) return fail(BSW_EINVAL, "params is NULL");
  if (n_params < 1 || n_params > 256)
    return fail(BSW_EINVAL, "n_params = %d (must be 1..256)", n_params);
  for (int i = 0; i < n_params; ++i) {
    const bsw_params& p = params[i];
    if (p.o_del < 0 || p.o_ins < 0 || p.o_del > BSW_MAX_GAP || p.o_ins > BSW_MAX_GAP)
      return fail(BSW_EINVAL, "params[%d]: gap open must be 0..%d", i, BSW_MAX_GAP);
    if (p.e_del < 1 || p.e_ins < 1 || p.e_del > BSW_MAX_GAP || p.e_ins > BSW_MAX_GAP)
      return fail(BSW_EINVAL, "params[%d]: gap extend must be 1..%d", i, BSW_MAX_GAP);
    if (p.w < 0) return fail(BSW_EINVAL, "params[%d]: w < 0", i);
    if (p.end_bonus < 0 || p.end_bonus > BSW_MAX_BONUS)
      return fail(BSW_EINVAL, "params[%d]: end_bonus out of range", i);
  }
  return BSW_OK;
}

KParams to_kparams(const bsw_params& p) {
  KParams k;
  std::memset(&k, 0, sizeof k);
  int amax = 0;
  for (int a = 0; a < 5; ++a) {
    uint32_t lo = 0;
    for (int b = 0; b < 4; ++b) lo |= (uint32_t)(uint8_t)p.mat[a * 5 + b] << (8 * b);
    k.prow[a][0] = lo;
    k.prow[a][1] = (uint32_t)(uint8_t)p.mat[a * 5 + 4];
  }
  for (int i = 0; i < 25; ++i) amax = std::max(amax, (int)p.mat[i]);
  k.o_del = p.o_del;
  k.e_del = p.e_del;
  k.o_ins = p.o_ins;
  k.e_ins = p.e_ins;
  k.oe_del = p.o_del + p.e_del;
  k.oe_ins = p.o_ins + p.e_ins;
  k.w = p.w;
  k.zdrop = p.zdrop;
  k.end_bonus = p.end_bonus;
  k.amax = amax;
  return k;
}

}  // namespace

struct bsw_ctx {
  bsw_ctx_opts opts;
  int device = 0;
  int num_cu = 0;
  hipStream_t stream = nullptr;
  // ev[0] start, ev[1] binning done, ev[2] before the DP kernels, ev[3] end
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  // start and end events of each DP launch (on the launch's stream), and
  // what each launch ran
  static constexpr int MAXL = NCLS + 3;
  hipEvent_t lev[MAXL] = {};
  hipEvent_t lev0[MAXL] = {};
  // side streams of the batched path: classes run concurrently
  static constexpr int NSIDE = 4;
  hipStream_t side[NSIDE] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[NSIDE] = {};
  int lcls[MAXL] = {};
  int n_launch = 0;
  double lms[MAXL] = {};
  unsigned long long lcells[MAXL] = {};
  DevBuf ws;       // workspace
  DevBuf in;       // staged host inputs
  DevBuf res;      // staged results (host API)
  DevBuf longbuf;  // row buffers of the long class
  DevBuf qtiles;   // column-major query tiles of the 8-bit lane kernels
  KParams* h_kp = nullptr;  // pinned
  KParams* d_kp = nullptr;
  Status* h_status = nullptr;  // pinned
  long long* h_cls = nullptr;  // pinned [NCLS][2]
  int blocks_per_cu[2][NCLS] = {};
  // occupancy of the chunked classes by (symmetric variant, ring chunks)
  int occc[2][NCLS][80] = {};
  int last_status = BSW_OK;
  bool pending = false;
  hipStream_t pending_stream = nullptr;
  double timing[4] = {0, 0, 0, 0};
  int n_dp_launches = 0;
};

namespace {

int set_device(bsw_ctx* c) {
  HIPCHK(hipSetDevice(c->device));
  return BSW_OK;
}

// Enqueue prepare + bin, wait for the class counts, then enqueue the DP
// kernels.  All pointers are device pointers.
int run_pipeline(bsw_ctx* c, int64_t n, const uint8_t* q, const uint64_t* q_off,
                 const uint8_t* t, const uint64_t* t_off, const int32_t* h0,
                 const uint8_t* pid, int32_t n_params, bsw_result* out,
                 bsw_diag* diag, hipStream_t s) {
  int wmax = 0;
  bool sym = true;
  for (int i = 0; i < n_params; ++i) {
    wmax = std::max(wmax, c->h_kp[i].w);
    sym = sym && c->h_kp[i].o_del == c->h_kp[i].o_ins && c->h_kp[i].e_del == c->h_kp[i].e_ins;
  }
  const Layout L = layout_for(n);
  int rc = c->ws.ensure(L.total);
  if (rc) return rc;
  char* base = (char*)c->ws.p;
  uint32_t* hist = (uint32_t*)(base + L.hist);
  Status* st = (Status*)(base + L.status);
  uint32_t* ctr = (uint32_t*)(base + L.ctr);
  uint32_t* cursor = (uint32_t*)(base + L.cursor);
  long long* cls_range = (long long*)(base + L.cls_range);
  PairDesc* ovf = (PairDesc*)(base + L.ovf);
  PairDesc* ovf2 = (PairDesc*)(base + L.ovf2);
  uint32_t* keys = (uint32_t*)(base + L.keys);
  PairDesc* desc = (PairDesc*)(base + L.desc);

  HIPCHK(hipMemcpyAsync(c->d_kp, c->h_kp, sizeof(KParams) * n_params,
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipEventRecord(c->ev[0], s));
  launch_fill((uint32_t*)(base + L.zero_beg), (int64_t)((L.zero_end - L.zero_beg) / 4), s);
  launch_prep(n, q, t, q_off, t_off, h0, pid, n_params, c->d_kp, c->opts.min_lane_bits,
              c->opts.force_mode, keys, hist, st, s);
  launch_codes(q, q_off, n, st, s);
  launch_codes(t, t_off, n, st, s);
  launch_scan(hist, cursor, cls_range, s);
  launch_scatter(n, q_off, t_off, h0, pid, keys, cursor, desc, st, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(c->ev[1], s));
  HIPCHK(hipMemcpyAsync(c->h_status, st, sizeof(Status), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(c->h_cls, cls_range, sizeof(long long) * 2 * NCLS,
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (c->h_status->bad)
    return fail(BSW_EINVAL, "pair %llu is invalid (lengths, h0, param_id or a code > 4)",
                ~(unsigned long long)c->h_status->first_bad_inv);

  const bool persist = c->opts.path != BSW_PATH_PLAIN;
  // occupancy of a chunked class with a given ring (cached per context)
  auto chunked_per_cu = [&](int cls, int rg) {
    int& occ = c->occc[sym ? 1 : 0][cls][rg];
    if (!occ) occ = lane_blocks_per_cu(cls, sym, (size_t)rg * lane_chunk_row_bytes(cls));
    return occ;
  };
  // grid of every lane class, and the query-tile space of the chunked ones;
  // the 16-bit rerun of 8-bit overflows gets the last query-tile region
  const int r1cls = CLS_W16 + NLW - 1, r2cls = CLS_W32 + NLW - 1;
  int64_t blocks[NCLS] = {};
  int ring[NCLS] = {};
  size_t qt_off[NCLS] = {}, qt_words = 0;
  bool any8 = false, any16 = false;
  for (int cls = 0; cls < CLS_LONG; ++cls) {
    const int64_t count = c->h_cls[2 * cls + 1];
    if (count <= 0) continue;
    const int wpb = lane_waves_per_block(cls);
    const int64_t tiles = (count + 63) / 64;
    blocks[cls] = (tiles + wpb - 1) / wpb;
    int per_cu = c->blocks_per_cu[1][cls];
    if (cls < CLS_W32) {
      ring[cls] = lane8_ring_chunks(cls, wmax);
      per_cu = chunked_per_cu(cls, ring[cls]);
    }
    if (persist) blocks[cls] = std::min(blocks[cls], (int64_t)per_cu * c->num_cu);
    if (cls < CLS_W32) {
      (cls < CLS_W16 ? any8 : any16) = true;
      qt_off[cls] = qt_words;
      qt_words += (size_t)blocks[cls] * lane8_qtile_words(cls);
    }
  }
  const int r1ring = lane8_ring_chunks(r1cls, wmax);
  const int64_t r1blocks = any8 ? (int64_t)chunked_per_cu(r1cls, r1ring) * c->num_cu : 0;
  const size_t r1qt = qt_words;
  qt_words += (size_t)r1blocks * lane8_qtile_words(r1cls);
  if (qt_words && (rc = c->qtiles.ensure(qt_words * 4))) return rc;
  uint32_t* qt = (uint32_t*)c->qtiles.p;
  c->n_dp_launches = 0;
  c->n_launch = 0;
  HIPCHK(hipEventRecord(c->ev[2], s));
  // launch bracketing: start/end events on the launch's stream
  auto begin_launch = [&](int cls, hipStream_t ls) -> int {
    c->lcls[c->n_launch] = cls;
    HIPCHK(hipEventRecord(c->lev0[c->n_launch], ls));
    return BSW_OK;
  };
  auto end_launch = [&](hipStream_t ls) -> int {
    HIPCHK(hipEventRecord(c->lev[c->n_launch], ls));
    ++c->n_launch;
    ++c->n_dp_launches;
    return BSW_OK;
  };
  // batched path: the classes run concurrently on side streams, widest
  // first, so that one class's tail overlaps the next class's work; the
  // reruns wait for all of them.  Plain path: one stream, in order.
  int nside_used = 0;
  if (persist) {
    HIPCHK(hipEventRecord(c->fork_ev, s));
    for (int k = 0; k < bsw_ctx::NSIDE; ++k) HIPCHK(hipStreamWaitEvent(c->side[k], c->fork_ev, 0));
  }
  int order[NCLS], no = 0;
  for (int cls = CLS_W16 - 1; cls >= CLS_L8; --cls) order[no++] = cls;   // 8-bit, widest first
  for (int cls = CLS_W16; cls < CLS_LONG; ++cls) order[no++] = cls;
  for (int oi = 0; oi < no; ++oi) {
    const int cls = order[oi];
    if (blocks[cls] <= 0) continue;
    hipStream_t ls = persist ? c->side[nside_used++ % bsw_ctx::NSIDE] : s;
    if ((rc = begin_launch(cls, ls))) return rc;
    // 8-bit overflows go to the first rerun list, 16-bit ones to the second
    launch_lane(cls, persist, (unsigned)blocks[cls], desc, cls_range + 2 * cls, q, t,
                c->d_kp, out, diag, ctr + cls, st, qt ? qt + qt_off[cls] : nullptr,
                cls < CLS_W16 ? ovf : ovf2,
                cls < CLS_W16 ? &st->ovf_range[1] : &st->ovf2_range[1], ring[cls], sym,
                &st->cls_cells[cls], ls);
    if ((rc = end_launch(ls))) return rc;
  }
  if (persist) {
    for (int k = 0; k < bsw_ctx::NSIDE; ++k) {
      HIPCHK(hipEventRecord(c->join_ev[k], c->side[k]));
      HIPCHK(hipStreamWaitEvent(s, c->join_ev[k], 0));
    }
  }
  if (c->h_cls[2 * CLS_LONG + 1] > 0) {
    const size_t need = (size_t)LONG_SLOTS * LONG_SLOT_COLS * (sizeof(int2) + 1);
    rc = c->longbuf.ensure(need);
    if (rc) return rc;
    int2* gbuf = (int2*)c->longbuf.p;
    uint8_t* gq = (uint8_t*)(gbuf + (size_t)LONG_SLOTS * LONG_SLOT_COLS);
    if ((rc = begin_launch(CLS_LONG, s))) return rc;
    launch_long(desc, cls_range + 2 * CLS_LONG, q, t, c->d_kp, out, diag, ctr + CLS_LONG,
                gbuf, gq, st, &st->cls_cells[CLS_LONG], s);
    if ((rc = end_launch(s))) return rc;
  }
  // reruns: the counts are only known on the device, so the grids are
  // persistent and exit at once when their list is empty
  if (any8) {
    // 16-bit chunked rerun of the pairs the 8-bit kernels could not settle
    if ((rc = begin_launch(NCLS, s))) return rc;
    launch_lane(r1cls, true, (unsigned)r1blocks, ovf, st->ovf_range, q, t, c->d_kp, out,
                diag, ctr + NCLS, st, qt + r1qt, ovf2, &st->ovf2_range[1], r1ring, sym,
                &st->cls_cells[NCLS], s);
    if ((rc = end_launch(s))) return rc;
  }
  if (any8 || any16) {
    // 32-bit rerun of the pairs the 16-bit kernels could not settle
    if ((rc = begin_launch(NCLS + 1, s))) return rc;
    launch_lane(r2cls, true, (unsigned)(c->blocks_per_cu[1][r2cls] * c->num_cu), ovf2,
                st->ovf2_range, q, t, c->d_kp, out, diag, ctr + NCLS + 1, st, nullptr,
                nullptr, nullptr, 0, false, &st->cls_cells[NCLS + 1], s);
    if ((rc = end_launch(s))) return rc;
  }
  HIPCHK(hipMemcpyAsync(c->h_status, st, sizeof(Status), hipMemcpyDeviceToHost, s));
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(c->ev[3], s));
  return BSW_OK;
}

// device time of the last call: prepare+bin and DP kernels (the host wait
// between the two is not counted)
void record_timing(bsw_ctx* c) {
  float a = 0, b = 0;
  if (hipEventElapsedTime(&a, c->ev[0], c->ev[1]) == hipSuccess &&
      hipEventElapsedTime(&b, c->ev[2], c->ev[3]) == hipSuccess) {
    c->timing[0] = (double)a + b;
    c->timing[1] = a;
    c->timing[2] = b;
    c->timing[3] = c->n_dp_launches;
  }
  for (int k = 0; k < c->n_launch; ++k) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, c->lev0[k], c->lev[k]) != hipSuccess) ms = 0;
    c->lms[k] = ms;
    c->lcells[k] = c->h_status->cls_cells[c->lcls[k]];
  }
}

}  // namespace

extern "C" {

int bsw_abi_version(void) { return BSW_ABI_VERSION; }

const char* bsw_last_error(void) { return g_err.c_str(); }

int bsw_ctx_create(bsw_ctx** out, const bsw_ctx_opts* opts) {
  if (!out) return fail(BSW_EINVAL, "out is NULL");
  bsw_ctx_opts o;
  std::memset(&o, 0, sizeof o);
  if (opts) o = *opts;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return fail(BSW_EDEVICE, "no HIP device is visible");
  if (o.device < 0 || o.device >= ndev)
    return fail(BSW_EDEVICE, "device %d does not exist (%d visible)", o.device, ndev);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, o.device) != hipSuccess)
    return fail(BSW_EDEVICE, "cannot query device %d", o.device);
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(BSW_EDEVICE, "device %d is %s; this library is built for gfx950",
                o.device, prop.gcnArchName);
  if (o.min_lane_bits != 0 && o.min_lane_bits != 8 && o.min_lane_bits != 16 &&
      o.min_lane_bits != 32)
    return fail(BSW_EINVAL, "min_lane_bits must be 0, 8, 16 or 32");
  if (o.path != BSW_PATH_BATCHED && o.path != BSW_PATH_PLAIN)
    return fail(BSW_EINVAL, "unknown path %d", o.path);
  bsw_ctx* c = new (std::nothrow) bsw_ctx;
  if (!c) return fail(BSW_ENOMEM, "out of host memory");
  c->opts = o;
  c->device = o.device;
  c->num_cu = prop.multiProcessorCount;
  int rc = BSW_OK;
  if (hipSetDevice(c->device) != hipSuccess ||
      hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return fail(BSW_EDEVICE, "cannot create a stream on device %d", o.device);
  }
  for (auto& e : c->ev)
    if (hipEventCreate(&e) != hipSuccess) rc = BSW_EDEVICE;
  for (auto& e : c->lev)
    if (hipEventCreate(&e) != hipSuccess) rc = BSW_EDEVICE;
  for (auto& e : c->lev0)
    if (hipEventCreate(&e) != hipSuccess) rc = BSW_EDEVICE;
  for (auto& e : c->join_ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) rc = BSW_EDEVICE;
  if (hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming) != hipSuccess)
    rc = BSW_EDEVICE;
  for (auto& st : c->side)
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) rc = BSW_EDEVICE;
  if (hipHostMalloc((void**)&c->h_kp, sizeof(KParams) * 256, 0) != hipSuccess ||
      hipHostMalloc((void**)&c->h_status, sizeof(Status), 0) != hipSuccess ||
      hipHostMalloc((void**)&c->h_cls, sizeof(int64_t) * 2 * NCLS, 0) != hipSuccess ||
      hipMalloc((void**)&c->d_kp, sizeof(KParams) * 256) != hipSuccess)
    rc = BSW_ENOMEM;
  // raise the dynamic-LDS limit of the large lane classes; a refusal only
  // surfaces later as a launch error of that class
  for (int cls = 0; cls < CLS_LONG && rc == BSW_OK; ++cls)
    for (int p = 0; p < 2; ++p) {
      (void)lane_setup(cls, p == 1);
      c->blocks_per_cu[p][cls] = lane_blocks_per_cu(cls, p == 1, 0);
    }
  (void)hipGetLastError();
  if (rc != BSW_OK) {
    bsw_ctx_destroy(c);
    return fail(rc, "context set-up on device %d failed", o.device);
  }
  *out = c;
  return BSW_OK;
}

void bsw_ctx_destroy(bsw_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  c->ws.release();
  c->in.release();
  c->res.release();
  c->longbuf.release();
  c->qtiles.release();
  if (c->h_kp) (void)hipHostFree(c->h_kp);
  if (c->h_status) (void)hipHostFree(c->h_status);
  if (c->h_cls) (void)hipHostFree(c->h_cls);
  if (c->d_kp) (void)hipFree(c->d_kp);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : c->lev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : c->lev0)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : c->join_ev)
    if (e) (void)hipEventDestroy(e);
  if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
  for (auto& st : c->side)
    if (st) (void)hipStreamDestroy(st);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

int bsw_extend_batch_device(bsw_ctx* c, int64_t n, const uint8_t* q,
                            const uint64_t* q_off, const uint8_t* t,
                            const uint64_t* t_off, const int32_t* h0,
                            const uint8_t* param_id, const bsw_params* params,
                            int32_t n_params, bsw_result* out, bsw_diag* diag,
                            void* stream, int32_t async) {
  if (!c) return fail(BSW_EINVAL, "ctx is NULL");
  if (n < 0 || n > 0x7fffffffLL) return fail(BSW_EINVAL, "n = %lld out of range", (long long)n);
  if (n == 0) return BSW_OK;
  int rc = check_params(params, n_params);
  if (rc) return rc;
  if (!q_off || !t_off || !h0 || !out)
    return fail(BSW_EINVAL, "a required device pointer is NULL");
  if ((rc = set_device(c))) return rc;
  for (int i = 0; i < n_params; ++i) c->h_kp[i] = to_kparams(params[i]);
  hipStream_t s = stream ? (hipStream_t)stream : c->stream;
  rc = run_pipeline(c, n, q, q_off, t, t_off, h0, param_id, n_params, out, diag, s);
  if (rc) return rc;
  if (async) {
    c->pending = true;
    c->pending_stream = s;
    return BSW_OK;
  }
  HIPCHK(hipStreamSynchronize(s));
  record_timing(c);
  return BSW_OK;
}

int bsw_ctx_wait(bsw_ctx* c) {
  if (!c) return fail(BSW_EINVAL, "ctx is NULL");
  if (!c->pending) return BSW_OK;
  c->pending = false;
  HIPCHK(hipStreamSynchronize(c->pending_stream));
  record_timing(c);
  return BSW_OK;
}

int bsw_ctx_last_kernels(bsw_ctx* c, int32_t* cls, int64_t* cells, double* ms,
                         int32_t max) {
  if (!c) return fail(BSW_EINVAL, "ctx is NULL");
  const int n = std::min((int)max, c->n_launch);
  for (int k = 0; k < n; ++k) {
    if (cls) cls[k] = c->lcls[k];
    if (cells) cells[k] = (int64_t)c->lcells[k];
    if (ms) ms[k] = c->lms[k];
  }
  return c->n_launch;
}

const char* bsw_class_name(int32_t cls) {
  static const char* names[NCLS + 2] = {
      "lane8_q32",  "lane8_q64",  "lane8_q96",  "lane8_q128", "lane8_q160",
      "lane8_q192", "lane8_q224", "lane8_q256", "lane16_q32", "lane16_q64",
      "lane16_q128", "lane16_q256", "lane32_q32", "lane32_q64", "lane32_q128",
      "lane32_q256", "long", "rerun16", "rerun32"};
  return cls >= 0 && cls <= NCLS + 1 ? names[cls] : "?";
}

int bsw_ctx_last_timing(bsw_ctx* c, double out4[4]) {
  if (!c || !out4) return fail(BSW_EINVAL, "NULL argument");
  for (int i = 0; i < 4; ++i) out4[i] = c->timing[i];
  return BSW_OK;
}

int bsw_extend_batch(bsw_ctx* c, int64_t n, const uint8_t* q, const uint64_t* q_off,
                     const uint8_t* t, const uint64_t* t_off, const int32_t* h0,
                     const uint8_t* param_id, const bsw_params* params,
                     int32_t n_params, bsw_result* out, bsw_diag* diag) {
  if (!c) return fail(BSW_EINVAL, "ctx is NULL");
  if (n < 0 || n > 0x7fffffffLL) return fail(BSW_EINVAL, "n = %lld out of range", (long long)n);
  if (n == 0) return BSW_OK;
  int rc = check_params(params, n_params);
  if (rc) return rc;
  if (!q_off || !t_off || !h0 || !out) return fail(BSW_EINVAL, "a required pointer is NULL");
  // host-side validation of every pair before anything is staged
  for (int64_t k = 0; k < n; ++k) {
    if (q_off[k + 1] < q_off[k] || t_off[k + 1] < t_off[k] ||
        q_off[k + 1] - q_off[k] > BSW_MAX_LEN || t_off[k + 1] - t_off[k] > BSW_MAX_LEN)
      return fail(BSW_EINVAL, "pair %lld: bad offsets or length > %d", (long long)k, BSW_MAX_LEN);
    if (h0[k] < 1 || h0[k] > BSW_MAX_H0)
      return fail(BSW_EINVAL, "pair %lld: h0 = %d out of range", (long long)k, h0[k]);
    if (param_id && param_id[k] >= n_params)
      return fail(BSW_EINVAL, "pair %lld: param_id %d >= n_params", (long long)k, param_id[k]);
    for (uint64_t x = q_off[k]; x < q_off[k + 1]; ++x)
      if (q[x] > 4) return fail(BSW_EINVAL, "pair %lld: query code > 4", (long long)k);
    for (uint64_t x = t_off[k]; x < t_off[k + 1]; ++x)
      if (t[x] > 4) return fail(BSW_EINVAL, "pair %lld: target code > 4", (long long)k);
  }
  if ((rc = set_device(c))) return rc;
  // stage: q bytes, t bytes, rebased offsets, h0, param_id
  const uint64_t q0 = q_off[0], t0 = t_off[0];
  const size_t qb = q_off[n] - q0, tb = t_off[n] - t0;
  size_t o = 0;
  const size_t o_q = o; o = align_up(o + qb + 1, 256);
  const size_t o_t = o; o = align_up(o + tb + 1, 256);
  const size_t o_qo = o; o = align_up(o + 8 * (size_t)(n + 1), 256);
  const size_t o_to = o; o = align_up(o + 8 * (size_t)(n + 1), 256);
  const size_t o_h0 = o; o = align_up(o + 4 * (size_t)n, 256);
  const size_t o_pid = o; o = align_up(o + (size_t)n, 256);
  const size_t total_in = o;
  const size_t o_out = 0;
  size_t r = align_up(sizeof(bsw_result) * (size_t)n, 256);
  const size_t o_diag = r;
  r += diag ? sizeof(bsw_diag) * (size_t)n : 0;
  if ((rc = c->in.ensure(total_in)) || (rc = c->res.ensure(r))) return rc;
  char* din = (char*)c->in.p;
  char* dres = (char*)c->res.p;
  std::vector<uint64_t> qo((size_t)n + 1), to((size_t)n + 1);
  for (int64_t k = 0; k <= n; ++k) {
    qo[k] = q_off[k] - q0;
    to[k] = t_off[k] - t0;
  }
  hipStream_t s = c->stream;
  HIPCHK(hipMemcpyAsync(din + o_q, q + q0, qb, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(din + o_t, t + t0, tb, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(din + o_qo, qo.data(), 8 * (size_t)(n + 1), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(din + o_to, to.data(), 8 * (size_t)(n + 1), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(din + o_h0, h0, 4 * (size_t)n, hipMemcpyHostToDevice, s));
  if (param_id)
    HIPCHK(hipMemcpyAsync(din + o_pid, param_id, (size_t)n, hipMemcpyHostToDevice, s));
  for (int i = 0; i < n_params; ++i) c->h_kp[i] = to_kparams(params[i]);
  rc = run_pipeline(c, n, (const uint8_t*)(din + o_q), (const uint64_t*)(din + o_qo),
                    (const uint8_t*)(din + o_t), (const uint64_t*)(din + o_to),
                    (const int32_t*)(din + o_h0),
                    param_id ? (const uint8_t*)(din + o_pid) : nullptr, n_params,
                    (bsw_result*)(dres + o_out), diag ? (bsw_diag*)(dres + o_diag) : nullptr,
                    s);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(out, dres + o_out, sizeof(bsw_result) * (size_t)n,
                        hipMemcpyDeviceToHost, s));
  if (diag)
    HIPCHK(hipMemcpyAsync(diag, dres + o_diag, sizeof(bsw_diag) * (size_t)n,
                          hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  record_timing(c);
  return BSW_OK;
}

}  // extern "C"
