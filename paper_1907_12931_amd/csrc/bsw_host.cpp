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
#include <cstdlib>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <utility>
#include <string>
#include <vector>

#include "../../include/bsw.h"
#include "bsw_internal.h"
#include "bsw_runtime.h"

namespace bsw {
size_t lane_lds_per_wave(int cls);
int lane_waves_per_block(int cls);
hipError_t lane_setup(int cls, bool persist);
int lane_blocks_per_cu(int cls, bool persist, size_t lds);
int lane8_ring_chunks(int cls, int wmax);
size_t lane8_qtile_words(int cls);
size_t lane_chunk_row_bytes(int cls);
void launch_prep(int64_t n, const uint8_t* q, const uint8_t* t, const uint64_t* q_off,
                 const uint64_t* q_end, const uint64_t* t_off, const uint64_t* t_end,
                 const int32_t* h0, const uint8_t* pid, int n_params, const KParams* kp,
                 int min_bits, int spec16, uint32_t* keys, uint32_t* hist, Status* st,
                 hipStream_t s);
void launch_scan(const uint32_t* hist, uint32_t* cursor, long long* cls_range,
                 hipStream_t s);
void launch_scatter(int64_t n, const uint64_t* q_off, const uint64_t* q_end,
                    const uint64_t* t_off, const uint64_t* t_end, const int32_t* h0,
                    const uint8_t* pid, const uint32_t* keys, uint32_t* cursor,
                    PairDesc* desc, const Status* st, hipStream_t s);

void launch_lane(int cls, bool persist, unsigned blocks, const PairDesc* desc,
                 const long long* range, const uint8_t* q, const uint8_t* t,
                 const KParams* kp, bsw_result* out, bsw_diag* diag,
                 uint32_t* tile_ctr, const Status* st, uint32_t* qtiles,
                 PairDesc* ovf, long long* ovf_count, int ring, bool sym,
                 unsigned long long* cls_cells, unsigned long long* work_cells,
                 hipStream_t s);
void launch_wave(unsigned blocks, const PairDesc* desc, const long long* range,
                 const uint8_t* q, const uint8_t* t, const KParams* kp, bsw_result* out,
                 bsw_diag* diag, uint32_t* ctr, const Status* st,
                 unsigned long long* cls_cells, hipStream_t s);
int wave_blocks_per_cu();
int wavev_blocks_per_cu(int cls);
void launch_wavev(int cls, unsigned blocks, const PairDesc* desc, const long long* range,
                  const uint8_t* q, const uint8_t* t, const KParams* kp, bsw_result* out,
                  bsw_diag* diag, uint32_t* ctr, const Status* st,
                  unsigned long long* cls_cells, unsigned long long* work_cells,
                  hipStream_t s);
void launch_long(int slots, const PairDesc* desc, const long long* range, const uint8_t* q,
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

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Workspace carve-up for n pairs.
struct Layout {
  size_t keys, desc, ovf, hist, cursor, cls_range, status, ctr, zero_beg, zero_end,
      total;
};

constexpr int NCTR = NCLS + 2;  // one tile counter per class, the rerun, spare

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
  L.total = o;
  return L;
}

int check_params(const bsw_params* params, int32_t n_params) {
  if (!params) return fail(BSW_EINVAL, "params is NULL");
  if (n_params < 1 || n_params > 256)
    return fail(BSW_EINVAL, "n_params = %d (must be 1..256)", n_params);
  for (int i = 0; i < n_params; ++i)
    if (const char* why = params_problem(params[i]))
      return fail(BSW_EINVAL, "params[%d]: %s", i, why);
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


// What a captured batched pipeline depends on besides the scoring values.
struct GraphKey {
  Args a;
  hipStream_t s;
  void* ws;
  void* qt;
  void* lb;
  int wmax;
  bool sym;
  Tune tune;
};

bool same_key(const GraphKey& x, const GraphKey& y) {
  const Args &a = x.a, &b = y.a;
  return a.n == b.n && a.q == b.q && a.q_off == b.q_off && a.t == b.t && a.t_off == b.t_off &&
         a.h0 == b.h0 && a.pid == b.pid && a.n_params == b.n_params && a.out == b.out &&
         a.diag == b.diag && a.q_end == b.q_end && a.t_end == b.t_end &&
         a.codes_checked == b.codes_checked && x.s == y.s && x.ws == y.ws && x.qt == y.qt &&
         x.lb == y.lb && x.wmax == y.wmax && x.sym == y.sym && x.tune == y.tune;
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
  unsigned long long lwork[MAXL] = {};
  Budget budget;
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
  int wave_per_cu = 1;  // resident groups per CU of the rerun kernel
  int wavev_per_cu[NCLS] = {};  // of the wave-mode kernel of each 32-bit class
  // occupancy of the chunked classes by (symmetric variant, ring chunks)
  int occc[2][NCLS][80] = {};
  bool noalloc = false;     // the call being enqueued uses the scratch
  void* scratch = nullptr;  // device address of this device's scratch array
  bool pending = false;
  hipStream_t pending_stream = nullptr;
  int (*pending_done)(bsw_ctx*) = nullptr;  // completion check of that call
  SeedState* seed = nullptr;                // read-level seed driver
  SalState* sal = nullptr;                  // suffix-array lookup
  FmState* fm = nullptr;                    // FM-index search
  bool graph_call = false;  // the last call ran as a graph replay
  Status* last_st = nullptr;  // device status block of the last call
  double timing[4] = {0, 0, 0, 0};
  unsigned long long last_cells = 0;  // band cells of the last finished call
  // captured batched pipeline and what it was captured for
  hipGraphExec_t gexec = nullptr;
  hipStream_t gexec_stream = nullptr;  // stream of the graph's last launch
  GraphKey gkey;
  int n_graph_launch = 0;
  // launch shapes of the batched path (defaults, a cache entry or
  // bsw_ctx_tune's choice)
  // (per workload kind: pair batches, and the seed driver's two passes)
  Tune tunes[NKIND];
  int kind = KIND_PAIRS;  // kind of the call being enqueued
  char dev_name[64] = {0};
  std::string tune_keys[NKIND];  // cache entry each kind's shape came from
  std::string tune_cache;  // copy of opts.tune_cache (which points here)
};

namespace {

int set_device(bsw_ctx* c) {
  HIPCHK(hipSetDevice(c->device));
  return BSW_OK;
}


// Workspace pointers of a call with n pairs.
struct Work {
  uint32_t* hist;
  Status* st;
  uint32_t* ctr;
  uint32_t* cursor;
  long long* cls_range;
  PairDesc* ovf;
  uint32_t* keys;
  PairDesc* desc;
  uint32_t* zero;
  int64_t zero_words;
};

Work carve(char* base, const Layout& L) {
  Work w;
  w.hist = (uint32_t*)(base + L.hist);
  w.st = (Status*)(base + L.status);
  w.ctr = (uint32_t*)(base + L.ctr);
  w.cursor = (uint32_t*)(base + L.cursor);
  w.cls_range = (long long*)(base + L.cls_range);
  w.ovf = (PairDesc*)(base + L.ovf);
  w.keys = (uint32_t*)(base + L.keys);
  w.desc = (PairDesc*)(base + L.desc);
  w.zero = (uint32_t*)(base + L.zero_beg);
  w.zero_words = (int64_t)((L.zero_end - L.zero_beg) / 4);
  return w;
}

// Scoring facts the launch shapes depend on.
void scan_params(const bsw_ctx* c, int n_params, int* wmax, bool* sym) {
  *wmax = 0;
  *sym = true;
  for (int i = 0; i < n_params; ++i) {
    *wmax = std::max(*wmax, c->h_kp[i].w);
    *sym = *sym && c->h_kp[i].o_del == c->h_kp[i].o_ins &&
           c->h_kp[i].e_del == c->h_kp[i].e_ins;
  }
}

// Resident groups per CU of a chunked class with a ring of rg chunks
// (cached per context).
int chunked_per_cu(bsw_ctx* c, int cls, bool sym, int rg) {
  int& occ = c->occc[sym ? 1 : 0][cls][rg];
  if (!occ) occ = lane_blocks_per_cu(cls, sym, (size_t)rg * lane_chunk_row_bytes(cls));
  return occ;
}

// validation, histogram, scan and scatter into class lists
void enqueue_prep_bin(bsw_ctx* c, const Args& a, const Work& w, hipStream_t s) {
  launch_fill(w.zero, w.zero_words, s);
  const uint64_t* qe = a.q_end ? a.q_end : a.q_off + 1;
  const uint64_t* te = a.t_end ? a.t_end : a.t_off + 1;
  launch_prep(a.n, a.q, a.t, a.q_off, qe, a.t_off, te, a.h0, a.pid, a.n_params, c->d_kp,
              c->opts.min_lane_bits, c->tunes[c->kind].spec16, w.keys, w.hist, w.st, s);
  if (!a.codes_checked) {
    launch_codes(a.q, a.q_off, a.n, w.st, 0, s);
    launch_codes(a.t, a.t_off, a.n, w.st, 0, s);
  }
  launch_scan(w.hist, w.cursor, w.cls_range, s);
  launch_scatter(a.n, a.q_off, qe, a.t_off, te, a.h0, a.pid, w.keys, w.cursor, w.desc, w.st,
                 s);
}

// launch bracketing: start/end events on the launch's stream (not inside
// a graph capture, where events carry no timestamps)
int begin_launch(bsw_ctx* c, int cls, hipStream_t ls) {
  c->lcls[c->n_launch] = cls;
  if (!c->graph_call) HIPCHK(hipEventRecord(c->lev0[c->n_launch], ls));
  return BSW_OK;
}
int end_launch(bsw_ctx* c, hipStream_t ls) {
  if (!c->graph_call) HIPCHK(hipEventRecord(c->lev[c->n_launch], ls));
  ++c->n_launch;
  return BSW_OK;
}

// Whether a class runs in wave mode (one pair per wave) under the tuned
// threshold: the 32-bit classes whose query cap reaches it.
bool wave_mode(const bsw_ctx* c, int cls) {
  static const int caps[NLW] = {LW_CAP[0], LW_CAP[1], LW_CAP[2], LW_CAP[3]};
  return cls >= CLS_W32 && cls < CLS_LONG && caps[cls - CLS_W32] >= c->tunes[c->kind].wave32;
}

// One DP launch of a class, lane or wave mode.
void launch_class(bsw_ctx* c, int cls, bool persist, unsigned blocks, const Work& w,
                  const Args& a, uint32_t* qt, int ring, bool sym, hipStream_t ls) {
  Status* st = w.st;
  if (wave_mode(c, cls))
    launch_wavev(cls, blocks, w.desc, w.cls_range + 2 * cls, a.q, a.t, c->d_kp, a.out, a.diag,
                 w.ctr + cls, st, &st->cls_cells[cls], &st->work_cells[cls], ls);
  else
    launch_lane(cls, persist, blocks, w.desc, w.cls_range + 2 * cls, a.q, a.t, c->d_kp, a.out,
                a.diag, w.ctr + cls, st, qt, w.ovf, &st->ovf_range[1], ring, sym,
                &st->cls_cells[cls], &st->work_cells[cls], ls);
}

// persistent groups per CU of a class: what fits, scaled for the 8-bit
// classes by the tuned share
int tuned_per_cu(const bsw_ctx* c, int cls, int fit) {
  if (cls >= CLS_W16) return fit;
  const int t = fit * c->tunes[c->kind].occ8 / 100;
  return t < 1 ? 1 : t;
}

// Launch shapes of the batched path.  They depend only on the band limit,
// the gap symmetry and the device, never on the data: every class gets a
// full persistent grid that drains its list from a device-side counter and
// exits at once when the list is empty.
struct BatchedPlan {
  int64_t blocks[NCLS + 1] = {};  // per class, then the rerun
  int ring[NCLS + 1] = {};
  size_t qt_off[NCLS + 1] = {};
  size_t qt_words = 0;
  // device buffers of the call: query tiles of the 16-bit classes and the
  // row-buffer slots of the long class
  uint32_t* qt = nullptr;
  int2* gbuf = nullptr;
  uint8_t* gq = nullptr;
  int long_slots = LONG_SLOTS;
};

// The fixed-size device scratch of the allocation-free entry point: one
// array per device, the same for every context on it (its address is taken
// once per device, with that device current).  It holds a call's
// workspace for up to BSW_NOALLOC_MAX_PAIRS pairs, the query tiles of the
// 16-bit classes with their grids capped at NOALLOC_GROUPS groups, and
// NOALLOC_LONG_SLOTS row-buffer slots for queries longer than 256.
constexpr int NOALLOC_GROUPS = 64;
constexpr int NOALLOC_LONG_SLOTS = 4;
constexpr size_t NOALLOC_BYTES = (size_t)16 << 20;

}  // namespace

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[128] = {};

// Device address of the scratch array on the current device `dev`.
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= 128) return fail(BSW_EDEVICE, "device %d: no scratch slot", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(BSW_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return BSW_OK;
}

BatchedPlan plan_batched(bsw_ctx* c, int wmax, bool sym) {
  BatchedPlan p;
  for (int cls = 0; cls < CLS_LONG; ++cls) {
    int per_cu = c->blocks_per_cu[1][cls];
    if (cls < CLS_W16) {
      // register-row kernels: occupancy set by registers and the mirror
      per_cu = c->blocks_per_cu[sym ? 1 : 0][cls];
    } else if (cls < CLS_W32) {
      p.ring[cls] = lane8_ring_chunks(cls, wmax);
      per_cu = chunked_per_cu(c, cls, sym, p.ring[cls]);
    } else if (wave_mode(c, cls)) {
      per_cu = c->wavev_per_cu[cls];
    }
    p.blocks[cls] = (int64_t)tuned_per_cu(c, cls, per_cu) * c->num_cu;
    if (c->opts.max_groups > 0) p.blocks[cls] = std::min<int64_t>(p.blocks[cls], c->opts.max_groups);
    if (c->noalloc && cls >= CLS_W16 && cls < CLS_W32)
      p.blocks[cls] = std::min<int64_t>(p.blocks[cls], NOALLOC_GROUPS);
    if (cls >= CLS_W16 && cls < CLS_W32) {
      p.qt_off[cls] = p.qt_words;
      p.qt_words += (size_t)p.blocks[cls] * lane8_qtile_words(cls);
    }
  }
  p.blocks[NCLS] = (int64_t)c->wave_per_cu * c->num_cu;
  if (c->opts.max_groups > 0) p.blocks[NCLS] = std::min<int64_t>(p.blocks[NCLS], c->opts.max_groups);
  return p;
}

// Every step of the batched path, with no host wait in between.  The
// classes run concurrently on the side streams (8-bit widest first, then
// 16-bit, 32-bit), so that one class's tail overlaps the next class's
// work; the long class and the two reruns follow on the main stream.
int enqueue_batched(bsw_ctx* c, const Args& a, const Work& w, const BatchedPlan& p,
                    bool sym, hipStream_t s) {
  int rc;
  uint32_t* qt = p.qt;
  int2* gbuf = p.gbuf;
  uint8_t* gq = p.gq;
  Status* st = w.st;
  const bool ev = !c->graph_call;
  if (ev) HIPCHK(hipEventRecord(c->ev[0], s));
  enqueue_prep_bin(c, a, w, s);
  HIPCHK(hipGetLastError());
  if (ev) HIPCHK(hipEventRecord(c->ev[1], s));
  if (ev) HIPCHK(hipEventRecord(c->ev[2], s));
  c->n_launch = 0;
  // nside = 0: every class on the call's stream, in order
  const int nside = c->tunes[c->kind].nside;
  if (nside > 0) HIPCHK(hipEventRecord(c->fork_ev, s));
  for (int k = 0; k < nside; ++k) HIPCHK(hipStreamWaitEvent(c->side[k], c->fork_ev, 0));
  int order[NCLS], no = 0;
  for (int cls = CLS_W16 - 1; cls >= CLS_L8; --cls) order[no++] = cls;
  for (int cls = CLS_W16; cls < CLS_LONG; ++cls) order[no++] = cls;
  for (int oi = 0; oi < no; ++oi) {
    const int cls = order[oi];
    // with 16-bit pairs tried at 8 bits first, the 16-bit classes hold only
    // the few pairs that cannot start there: they run on the call's own
    // stream, idle until the join, beside the 8-bit classes
    const bool beside = nside > 0 && c->tunes[c->kind].spec16 && cls >= CLS_W16 &&
                        cls < CLS_W32;
    hipStream_t ls = nside > 0 && !beside ? c->side[oi % nside] : s;
    if ((rc = begin_launch(c, cls | (wave_mode(c, cls) ? WAVE_TAG : 0), ls))) return rc;
    // pairs a narrow class cannot settle in its record width go to the
    // rerun list
    launch_class(c, cls, true, (unsigned)p.blocks[cls], w, a,
                 cls >= CLS_W16 && cls < CLS_W32 ? qt + p.qt_off[cls] : nullptr, p.ring[cls],
                 sym, ls);
    if ((rc = end_launch(c, ls))) return rc;
  }
  for (int k = 0; k < nside; ++k) {
    HIPCHK(hipEventRecord(c->join_ev[k], c->side[k]));
    HIPCHK(hipStreamWaitEvent(s, c->join_ev[k], 0));
  }
  if ((rc = begin_launch(c, CLS_LONG, s))) return rc;
  launch_long(p.long_slots, w.desc, w.cls_range + 2 * CLS_LONG, a.q, a.t, c->d_kp, a.out,
              a.diag, w.ctr + CLS_LONG, gbuf, gq, st, &st->cls_cells[CLS_LONG], s);
  if ((rc = end_launch(c, s))) return rc;
  // the rerun, one pair per wave with 32-bit values
  if ((rc = begin_launch(c, NCLS, s))) return rc;
  launch_wave((unsigned)p.blocks[NCLS], w.ovf, st->ovf_range, a.q, a.t, c->d_kp, a.out,
              a.diag, w.ctr + NCLS, st, &st->cls_cells[NCLS], s);
  if ((rc = end_launch(c, s))) return rc;
  HIPCHK(hipGetLastError());
  if (ev) HIPCHK(hipEventRecord(c->ev[3], s));
  return BSW_OK;
}

// Tuned shapes are cached per device, band limit, gap symmetry and lane
// width floor in a small JSON file, one entry per line:
//   "gfx950:cu256:w100:sym1:mb0": {"nside": 4, "occ8": 100, "spec16": 1, "ms": 57.1},
std::string tune_key(const bsw_ctx* c, int wmax, bool sym, int kind) {
  char k[160];
  std::snprintf(k, sizeof k, "%s:cu%d:w%d:sym%d:mb%d%s", c->dev_name, c->num_cu, wmax,
                sym ? 1 : 0, c->opts.min_lane_bits, kind == KIND_SEEDS ? ":seeds" : "");
  return k;
}

bool cache_lookup(const char* path, const std::string& key, Tune* t) {
  for (auto& kv : cache_read(path))
    if (kv.first == key) return parse_tune(kv.second, bsw_ctx::NSIDE, t);
  return false;
}

int cache_store(const char* path, const std::string& key, const Tune& t, double ms) {
  if (!cache_put(path, key, format_tune(t, ms)))
    return fail(BSW_EINVAL, "cannot write the tune cache %s", path);
  return BSW_OK;
}

// Shapes for this call's scoring: from the cache when it has an entry.
void pick_tune(bsw_ctx* c, int wmax, bool sym) {
  if (!c->opts.tune_cache) return;
  const std::string key = tune_key(c, wmax, sym, c->kind);
  if (key == c->tune_keys[c->kind]) return;
  c->tune_keys[c->kind] = key;
  Tune t;
  if (cache_lookup(c->opts.tune_cache, key, &t)) c->tunes[c->kind] = t;
}

// Batched path: plan, make sure every buffer exists, then run the steps
// eagerly or as a graph.  The graph is captured on the first call with a
// given set of pointers and shapes and replayed while they stay the same;
// the scoring table is uploaded outside it, before every replay.
// The side streams a shape uses, created on first need (before any graph
// capture): a context that never uses them (a server slot) keeps every
// class on its own stream and so holds one hardware queue, not five.
int ensure_side(bsw_ctx* c, int nside) {
  for (int k = 0; k < nside; ++k)
    if (!c->side[k] && hipStreamCreateWithFlags(&c->side[k], hipStreamNonBlocking) != hipSuccess)
      return fail(BSW_EDEVICE, "cannot create a side stream");
  return BSW_OK;
}

int run_batched(bsw_ctx* c, const Args& a, hipStream_t s) {
  int wmax;
  bool sym;
  scan_params(c, a.n_params, &wmax, &sym);
  const Layout L = layout_for(a.n);
  int rc;
  if (c->noalloc) {
    // everything in the device scratch, no graph of our own, no cache read
    BatchedPlan p = plan_batched(c, wmax, sym);
    char* base = (char*)c->scratch;
    const size_t qt_at = align_up(L.total, 256);
    const size_t lb_at = align_up(qt_at + p.qt_words * 4, 256);
    const size_t lb_bytes = (size_t)NOALLOC_LONG_SLOTS * LONG_SLOT_COLS * (sizeof(int2) + 1);
    if (lb_at + lb_bytes > NOALLOC_BYTES)
      return fail(BSW_ETOOBIG, "%lld pairs need more than the %zu-byte scratch", (long long)a.n,
                  NOALLOC_BYTES);
    p.qt = (uint32_t*)(base + qt_at);
    p.gbuf = (int2*)(base + lb_at);
    p.gq = (uint8_t*)(p.gbuf + (size_t)NOALLOC_LONG_SLOTS * LONG_SLOT_COLS);
    p.long_slots = NOALLOC_LONG_SLOTS;
    const Work w = carve(base, L);
    c->last_st = w.st;
    HIPCHK(hipMemcpyAsync(c->d_kp, c->h_kp, sizeof(KParams) * a.n_params,
                          hipMemcpyHostToDevice, s));
    c->graph_call = false;
    if ((rc = ensure_side(c, c->tunes[c->kind].nside))) return rc;
    return enqueue_batched(c, a, w, p, sym, s);
  }
  pick_tune(c, wmax, sym);
  if ((rc = ensure_side(c, c->tunes[c->kind].nside))) return rc;
  if ((rc = c->ws.ensure(L.total))) return rc;
  BatchedPlan p = plan_batched(c, wmax, sym);
  if ((rc = c->qtiles.ensure(p.qt_words * 4))) return rc;
  if ((rc = c->longbuf.ensure((size_t)LONG_SLOTS * LONG_SLOT_COLS * (sizeof(int2) + 1))))
    return rc;
  p.qt = (uint32_t*)c->qtiles.p;
  p.gbuf = (int2*)c->longbuf.p;
  p.gq = (uint8_t*)(p.gbuf + (size_t)LONG_SLOTS * LONG_SLOT_COLS);
  const Work w = carve((char*)c->ws.p, L);
  c->last_st = w.st;
  HIPCHK(hipMemcpyAsync(c->d_kp, c->h_kp, sizeof(KParams) * a.n_params,
                        hipMemcpyHostToDevice, s));
  c->graph_call = !c->opts.no_graph;
  if (!c->graph_call) return enqueue_batched(c, a, w, p, sym, s);
  GraphKey key;
  key.a = a;
  key.s = s;
  key.ws = c->ws.p;
  key.qt = c->qtiles.p;
  key.lb = c->longbuf.p;
  key.wmax = wmax;
  key.sym = sym;
  key.tune = c->tunes[c->kind];
  if (!c->gexec || !same_key(key, c->gkey)) {
    // an executable graph is destroyed only once its last launch has
    // finished: the runtime may still be walking it otherwise
    if (c->gexec) {
      HIPCHK(hipStreamSynchronize(c->gexec_stream));
      (void)hipGraphExecDestroy(c->gexec);
    }
    c->gexec = nullptr;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    rc = enqueue_batched(c, a, w, p, sym, s);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess)
      return fail(BSW_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    const hipError_t ei = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      c->gexec = nullptr;
      return fail(BSW_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(ei));
    }
    c->gkey = key;
    c->n_graph_launch = c->n_launch;
  }
  c->n_launch = c->n_graph_launch;
  HIPCHK(hipEventRecord(c->ev[0], s));
  c->gexec_stream = s;
  HIPCHK(hipGraphLaunch(c->gexec, s));
  HIPCHK(hipEventRecord(c->ev[3], s));
  return BSW_OK;
}

// The tuning loop (see ctx_tune_shapes).  The kind's cache key is set
// first, so that the calls leave the candidate shapes alone.
int tune_shapes(bsw_ctx* c, int kind, int n_params, int reps, int (*run)(bsw_ctx*, void*),
                void* arg, double* best_ms) {
  int wmax;
  bool sym;
  scan_params(c, n_params, &wmax, &sym);
  const std::string key = tune_key(c, wmax, sym, kind);
  c->tune_keys[kind] = key;
  // coordinate descent from the default shape: each knob in turn takes
  // every value with the others held at the best so far; a shape must beat
  // the best by more than 1% (timing noise between near-equal shapes)
  std::vector<double> ts;
  int rc = BSW_OK;
  auto score = [&](const Tune& x, double* med) {
    c->tunes[kind] = x;
    ts.clear();
    for (int r = 0; r <= reps && rc == BSW_OK; ++r) {
      rc = run(c, arg);
      if (rc == BSW_OK && r > 0) ts.push_back(c->timing[0]);
    }
    if (rc) return;
    std::sort(ts.begin(), ts.end());
    *med = ts[ts.size() / 2];
  };
  static const int nsides[] = {4, 2, 1}, occs[] = {100, 75, 50}, specs[] = {1, 0},
                   waves[] = {64, 128, 256, 512, 32};
  // more streams than hardware queues share queues: a side stream then
  // waits behind another stream's work (the graph replay of such a shape
  // lost about 1 ms against two side streams, where eager timing showed
  // no loss), so the tuner keeps the caller's stream, the runtime's default
  // stream and the side streams within the queues the process has
  // (GPU_MAX_HW_QUEUES, 4 unless set)
  const char* hwq_env = std::getenv("GPU_MAX_HW_QUEUES");
  const int hwq = hwq_env && std::atoi(hwq_env) > 0 ? std::atoi(hwq_env) : 4;
  const int nside_max = std::max(1, std::min(bsw_ctx::NSIDE, hwq - 2));
  Tune best;
  best.nside = std::min(best.nside, nside_max);
  double best_t = 1e300;
  score(best, &best_t);
  for (int knob = 0; knob < 4 && rc == BSW_OK; ++knob) {
    const int* vals = knob == 0 ? nsides : knob == 1 ? occs : knob == 2 ? specs : waves;
    const int nv = knob == 0 ? 3 : knob == 1 ? 3 : knob == 2 ? 2 : 5;
    const Tune base = best;
    for (int v = 0; v < nv && rc == BSW_OK; ++v) {
      Tune x = base;
      int& field = knob == 0 ? x.nside : knob == 1 ? x.occ8 : knob == 2 ? x.spec16 : x.wave32;
      if (field == vals[v] || (knob == 0 && vals[v] > nside_max)) continue;
      field = vals[v];
      double med = 0;
      score(x, &med);
      if (rc == BSW_OK && med < best_t * 0.99) {
        best_t = med;
        best = x;
      }
    }
  }
  c->tunes[kind] = best;
  if (rc) return rc;
  if (best_ms) *best_ms = best_t;
  if (c->opts.tune_cache && (rc = cache_store(c->opts.tune_cache, key, best, best_t)))
    return rc;
  return BSW_OK;
}

// Plain path: prepare + bin, wait for the class counts, then one ordinary
// launch per non-empty class on the caller's stream, in order.
int run_plain(bsw_ctx* c, const Args& a, hipStream_t s) {
  int wmax;
  bool sym;
  scan_params(c, a.n_params, &wmax, &sym);
  const Layout L = layout_for(a.n);
  int rc = c->ws.ensure(L.total);
  if (rc) return rc;
  const Work w = carve((char*)c->ws.p, L);
  Status* st = w.st;
  c->last_st = st;
  c->graph_call = false;
  HIPCHK(hipMemcpyAsync(c->d_kp, c->h_kp, sizeof(KParams) * a.n_params,
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipEventRecord(c->ev[0], s));
  enqueue_prep_bin(c, a, w, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(c->ev[1], s));
  HIPCHK(hipMemcpyAsync(c->h_status, st, sizeof(Status), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(c->h_cls, w.cls_range, sizeof(long long) * 2 * NCLS,
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (c->h_status->bad) return BSW_OK;  // reported when the call completes
  int64_t blocks[NCLS] = {};
  int ring[NCLS] = {};
  size_t qt_off[NCLS] = {}, qt_words = 0;
  bool any8 = false, any16 = false;
  for (int cls = 0; cls < CLS_LONG; ++cls) {
    const int64_t count = c->h_cls[2 * cls + 1];
    if (count <= 0) continue;
    const int wpb = lane_waves_per_block(cls);
    blocks[cls] = ((count + 63) / 64 + wpb - 1) / wpb;
    // wave mode: a persistent grid that takes one pair per wave at a time
    if (wave_mode(c, cls))
      blocks[cls] = std::min<int64_t>(count, (int64_t)c->wavev_per_cu[cls] * c->num_cu);
    if (cls < CLS_W32) (cls < CLS_W16 ? any8 : any16) = true;
    if (cls >= CLS_W16 && cls < CLS_W32) {
      ring[cls] = lane8_ring_chunks(cls, wmax);
      qt_off[cls] = qt_words;
      qt_words += (size_t)blocks[cls] * lane8_qtile_words(cls);
    }
  }
  if (qt_words && (rc = c->qtiles.ensure(qt_words * 4))) return rc;
  uint32_t* qt = (uint32_t*)c->qtiles.p;
  c->n_launch = 0;
  HIPCHK(hipEventRecord(c->ev[2], s));
  int order[NCLS], no = 0;  // same order as the batched path
  for (int cls = CLS_W16 - 1; cls >= CLS_L8; --cls) order[no++] = cls;
  for (int cls = CLS_W16; cls < CLS_LONG; ++cls) order[no++] = cls;
  for (int oi = 0; oi < no; ++oi) {
    const int cls = order[oi];
    if (blocks[cls] <= 0) continue;
    if ((rc = begin_launch(c, cls | (wave_mode(c, cls) ? WAVE_TAG : 0), s))) return rc;
    launch_class(c, cls, false, (unsigned)blocks[cls], w, a, qt ? qt + qt_off[cls] : nullptr,
                 ring[cls], sym, s);
    if ((rc = end_launch(c, s))) return rc;
  }
  if (c->h_cls[2 * CLS_LONG + 1] > 0) {
    rc = c->longbuf.ensure((size_t)LONG_SLOTS * LONG_SLOT_COLS * (sizeof(int2) + 1));
    if (rc) return rc;
    int2* gbuf = (int2*)c->longbuf.p;
    uint8_t* gq = (uint8_t*)(gbuf + (size_t)LONG_SLOTS * LONG_SLOT_COLS);
    if ((rc = begin_launch(c, CLS_LONG, s))) return rc;
    launch_long(LONG_SLOTS, w.desc, w.cls_range + 2 * CLS_LONG, a.q, a.t, c->d_kp, a.out,
                a.diag, w.ctr + CLS_LONG, gbuf, gq, st, &st->cls_cells[CLS_LONG], s);
    if ((rc = end_launch(c, s))) return rc;
  }
  // the rerun: its count is only known on the device, so the grid is
  // persistent and exits at once when the list is empty
  if (any8 || any16) {
    if ((rc = begin_launch(c, NCLS, s))) return rc;
    launch_wave((unsigned)(c->wave_per_cu * c->num_cu), w.ovf, st->ovf_range, a.q, a.t,
                c->d_kp, a.out, a.diag, w.ctr + NCLS, st, &st->cls_cells[NCLS], s);
    if ((rc = end_launch(c, s))) return rc;
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipEventRecord(c->ev[3], s));
  return BSW_OK;
}

// Enqueue a whole call on stream s, then the copy of its status to the
// host.  All pointers are device pointers.
int run_pipeline(bsw_ctx* c, const Args& a, hipStream_t s) {
  int rc = c->opts.path == BSW_PATH_PLAIN ? run_plain(c, a, s) : run_batched(c, a, s);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(c->h_status, c->last_st, sizeof(Status), hipMemcpyDeviceToHost, s));
  return BSW_OK;
}

// device time of the last call: prepare+bin and DP kernels (the host wait
// between the two is not counted)
// (a graph replay has only its whole span: the steps inside carry no
// events).  A failed query is cleared so that it does not linger as the
// thread's last HIP error.
float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
    (void)hipGetLastError();
    ms = 0;
  }
  return ms;
}

void record_timing(bsw_ctx* c) {
  c->timing[3] = c->n_launch;
  if (c->graph_call) {
    c->timing[0] = elapsed(c->ev[0], c->ev[3]);
    c->timing[1] = c->timing[2] = 0;
  } else {
    const float a = elapsed(c->ev[0], c->ev[1]), b = elapsed(c->ev[2], c->ev[3]);
    c->timing[0] = (double)a + b;
    c->timing[1] = a;
    c->timing[2] = b;
  }
  for (int k = 0; k < c->n_launch; ++k) {
    c->lms[k] = c->graph_call ? 0.0 : elapsed(c->lev0[k], c->lev[k]);
    c->lcells[k] = c->h_status->cls_cells[c->lcls[k] & (WAVE_TAG - 1)];
    c->lwork[k] = c->h_status->work_cells[c->lcls[k] & (WAVE_TAG - 1)];
  }
}

// After the stream has passed a call: its status (a rejected pair is
// reported here), then its timing.
int finish_call(bsw_ctx* c) {
  if (c->h_status->bad)
    return fail(BSW_EINVAL, "pair %llu is invalid (lengths, h0, param_id or a code > 4)",
                ~(unsigned long long)c->h_status->first_bad_inv);
  record_timing(c);
  c->last_cells = 0;
  for (int k = 0; k <= NCLS; ++k) c->last_cells += c->h_status->cls_cells[k];
  return BSW_OK;
}

}  // namespace

namespace bsw {

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

void ctx_set_side_streams(bsw_ctx* c, int nside) {
  c->tunes[KIND_PAIRS].nside = nside < 0 ? 0 : (nside > bsw_ctx::NSIDE ? bsw_ctx::NSIDE : nside);
}

int ctx_set_params(bsw_ctx* c, const bsw_params* params, int32_t n_params) {
  const int rc = check_params(params, n_params);
  if (rc) return rc;
  for (int i = 0; i < n_params; ++i) c->h_kp[i] = to_kparams(params[i]);
  return BSW_OK;
}

int ctx_reserve(bsw_ctx* c, int64_t n, int32_t n_params) {
  int rc = set_device(c);
  if (rc) return rc;
  int wmax;
  bool sym;
  scan_params(c, n_params, &wmax, &sym);
  if ((rc = c->ws.ensure(layout_for(n).total))) return rc;
  if (c->opts.path == BSW_PATH_BATCHED) {
    const BatchedPlan p = plan_batched(c, wmax, sym);
    if ((rc = c->qtiles.ensure(p.qt_words * 4))) return rc;
    if ((rc = c->longbuf.ensure((size_t)LONG_SLOTS * LONG_SLOT_COLS * (sizeof(int2) + 1))))
      return rc;
  }
  return BSW_OK;
}

int ctx_enqueue(bsw_ctx* c, const Args& a, hipStream_t s) {
  int rc = set_device(c);
  if (rc) return rc;
  return run_pipeline(c, a, s);
}

int ctx_finish(bsw_ctx* c) { return finish_call(c); }

int ctx_enqueue_eager(bsw_ctx* c, const Args& a, hipStream_t s) {
  const int32_t saved = c->opts.no_graph;
  c->opts.no_graph = 1;
  const int rc = run_pipeline(c, a, s);
  c->opts.no_graph = saved;
  return rc;
}

Status* ctx_status_dev(const bsw_ctx* c) { return c->last_st; }

Budget* ctx_budget(bsw_ctx* c) { return &c->budget; }

int ctx_launches(const bsw_ctx* c) { return c->n_launch; }

double* ctx_timing(bsw_ctx* c) { return c->timing; }

void ctx_add_cells(bsw_ctx* c, unsigned long long cells) { c->last_cells += cells; }

void ctx_set_cells(bsw_ctx* c, unsigned long long cells) { c->last_cells = cells; }

int ctx_set_device(bsw_ctx* c) { return set_device(c); }

int ctx_num_cu(const bsw_ctx* c) { return c->num_cu; }

int ctx_check_idle(const bsw_ctx* c) {
  if (c->pending)
    return fail(BSW_EBUSY,
                "an asynchronous call is still pending on this context: call "
                "bsw_ctx_wait first");
  return BSW_OK;
}

void ctx_set_pending(bsw_ctx* c, hipStream_t s, int (*done)(bsw_ctx*)) {
  c->pending = true;
  c->pending_stream = s;
  c->pending_done = done;
}

SeedState*& ctx_seed_state(bsw_ctx* c) { return c->seed; }

SalState*& ctx_sal_state(bsw_ctx* c) { return c->sal; }

FmState*& ctx_fm_state(bsw_ctx* c) { return c->fm; }

void ctx_set_kind(bsw_ctx* c, int kind) { c->kind = kind; }

int ctx_tune_shapes(bsw_ctx* c, int kind, int n_params, int reps,
                    int (*run)(bsw_ctx*, void*), void* arg, double* best_ms) {
  const int saved = c->kind;
  c->kind = kind;
  const int rc = tune_shapes(c, kind, n_params, reps, run, arg, best_ms);
  c->kind = saved;
  return rc;
}

Tune ctx_shape(const bsw_ctx* c, int kind) { return c->tunes[kind]; }

unsigned long long ctx_last_cells(const bsw_ctx* c) {
  unsigned long long sum = 0;
  for (int k = 0; k <= NCLS; ++k) sum += c->h_status->cls_cells[k];
  return sum;
}

hipStream_t ctx_stream(const bsw_ctx* c) { return c->stream; }

}  // namespace bsw

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
  if (o.max_groups < 0) return fail(BSW_EINVAL, "max_groups must be >= 0");
  if (o.path != BSW_PATH_BATCHED && o.path != BSW_PATH_PLAIN)
    return fail(BSW_EINVAL, "unknown path %d", o.path);
  bsw_ctx* c = new (std::nothrow) bsw_ctx;
  if (!c) return fail(BSW_ENOMEM, "out of host memory");
  c->opts = o;
  if (o.tune_cache) {
    c->tune_cache = o.tune_cache;
    c->opts.tune_cache = c->tune_cache.c_str();
  }
  c->device = o.device;
  c->num_cu = prop.multiProcessorCount;
  std::snprintf(c->dev_name, sizeof c->dev_name, "%s", prop.gcnArchName);
  c->budget.limit = o.hbm_budget;
  for (DevBuf* d : {&c->ws, &c->in, &c->res, &c->longbuf, &c->qtiles}) d->b = &c->budget;
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
  c->wave_per_cu = wave_blocks_per_cu();
  if (rc == BSW_OK) {
    const int rs = scratch_address(c->device, &c->scratch);
    if (rs != BSW_OK) rc = rs;
  }
  for (int cls = CLS_W32; cls < CLS_LONG; ++cls) c->wavev_per_cu[cls] = wavev_blocks_per_cu(cls);
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
  if (c->pending) (void)hipStreamSynchronize(c->pending_stream);
  seed_state_free(c->seed);
  sal_state_free(c->sal);
  fm_state_free(c->fm);
  c->ws.release();
  c->in.release();
  c->res.release();
  c->longbuf.release();
  c->qtiles.release();
  if (c->gexec) {
    (void)hipStreamSynchronize(c->gexec_stream);
    (void)hipGraphExecDestroy(c->gexec);
  }
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
  if (int rc0 = ctx_check_idle(c)) return rc0;
  if (n < 0 || n > 0x7fffffffLL) return fail(BSW_EINVAL, "n = %lld out of range", (long long)n);
  if (n == 0) return BSW_OK;
  int rc = check_params(params, n_params);
  if (rc) return rc;
  if (!q_off || !t_off || !h0 || !out)
    return fail(BSW_EINVAL, "a required device pointer is NULL");
  if ((rc = set_device(c))) return rc;
  for (int i = 0; i < n_params; ++i) c->h_kp[i] = to_kparams(params[i]);
  hipStream_t s = stream ? (hipStream_t)stream : c->stream;
  const Args a = {n, q, q_off, t, t_off, h0, param_id, n_params, out, diag,
                 nullptr, nullptr, false};
  rc = run_pipeline(c, a, s);
  if (rc) return rc;
  if (async) {
    ctx_set_pending(c, s, finish_call);
    return BSW_OK;
  }
  HIPCHK(hipStreamSynchronize(s));
  return finish_call(c);
}

int bsw_extend_batch_device_noalloc(bsw_ctx* c, int64_t n, const uint8_t* q,
                                    const uint64_t* q_off, const uint8_t* t,
                                    const uint64_t* t_off, const int32_t* h0,
                                    const uint8_t* param_id, const bsw_params* params,
                                    int32_t n_params, bsw_result* out, bsw_diag* diag,
                                    void* stream, int32_t async) {
  if (!c) return fail(BSW_EINVAL, "ctx is NULL");
  if (int rc0 = ctx_check_idle(c)) return rc0;
  if (n < 0) return fail(BSW_EINVAL, "n = %lld out of range", (long long)n);
  if (n > BSW_NOALLOC_MAX_PAIRS)
    return fail(BSW_ETOOBIG, "n = %lld exceeds the allocation-free limit of %d pairs",
                (long long)n, BSW_NOALLOC_MAX_PAIRS);
  if (n == 0) return BSW_OK;
  int rc = check_params(params, n_params);
  if (rc) return rc;
  if (!q_off || !t_off || !h0 || !out)
    return fail(BSW_EINVAL, "a required device pointer is NULL");
  if (c->opts.path != BSW_PATH_BATCHED)
    return fail(BSW_EINVAL, "the allocation-free entry runs the batched path");
  if ((rc = set_device(c))) return rc;
  for (int i = 0; i < n_params; ++i) c->h_kp[i] = to_kparams(params[i]);
  hipStream_t s = stream ? (hipStream_t)stream : c->stream;
  const Args a = {n, q, q_off, t, t_off, h0, param_id, n_params, out, diag,
                 nullptr, nullptr, false};
  c->noalloc = true;
  rc = run_pipeline(c, a, s);
  c->noalloc = false;
  if (rc) return rc;
  if (async) {
    ctx_set_pending(c, s, finish_call);
    return BSW_OK;
  }
  HIPCHK(hipStreamSynchronize(s));
  return finish_call(c);
}

int bsw_ctx_tune(bsw_ctx* c, int64_t n, const uint8_t* q, const uint64_t* q_off,
                 const uint8_t* t, const uint64_t* t_off, const int32_t* h0,
                 const uint8_t* param_id, const bsw_params* params, int32_t n_params,
                 bsw_result* out, int32_t reps, double* best_ms) {
  if (!c) return fail(BSW_EINVAL, "ctx is NULL");
  if (int rc0 = ctx_check_idle(c)) return rc0;
  if (c->opts.path != BSW_PATH_BATCHED)
    return fail(BSW_EINVAL, "tuning applies to the batched path");
  if (n < 1 || n > 0x7fffffffLL) return fail(BSW_EINVAL, "n = %lld out of range", (long long)n);
  if (reps < 1 || reps > 100) return fail(BSW_EINVAL, "reps must be 1..100");
  int rc = check_params(params, n_params);
  if (rc) return rc;
  if (!q_off || !t_off || !h0 || !out)
    return fail(BSW_EINVAL, "a required device pointer is NULL");
  if ((rc = set_device(c))) return rc;
  for (int i = 0; i < n_params; ++i) c->h_kp[i] = to_kparams(params[i]);
  Args a = {n, q, q_off, t, t_off, h0, param_id, n_params, out, nullptr,
            nullptr, nullptr, false};
  // every candidate runs eagerly, one whole call at a time
  auto run = [](bsw_ctx* cc, void* arg) {
    int r = run_pipeline(cc, *(const Args*)arg, cc->stream);
    if (r == BSW_OK && hipStreamSynchronize(cc->stream) != hipSuccess)
      r = fail(BSW_EDEVICE, "stream synchronisation failed");
    return r == BSW_OK ? finish_call(cc) : r;
  };
  const int32_t saved = c->opts.no_graph;
  c->opts.no_graph = 1;
  c->kind = KIND_PAIRS;
  rc = tune_shapes(c, KIND_PAIRS, n_params, reps, run, &a, best_ms);
  c->opts.no_graph = saved;
  return rc;
}

int bsw_ctx_tune_info(bsw_ctx* c, int32_t out3[3]) {
  if (!c || !out3) return fail(BSW_EINVAL, "NULL argument");
  out3[0] = c->tunes[KIND_PAIRS].nside;
  out3[1] = c->tunes[KIND_PAIRS].occ8;
  out3[2] = c->tunes[KIND_PAIRS].spec16;
  return BSW_OK;
}

int bsw_ctx_shape(bsw_ctx* c, int32_t* out, int32_t n) {
  if (!c || (!out && n > 0)) return fail(BSW_EINVAL, "NULL argument");
  const Tune& t = c->tunes[KIND_PAIRS];
  const int32_t v[4] = {t.nside, t.occ8, t.spec16, t.wave32};
  for (int k = 0; k < n && k < 4; ++k) out[k] = v[k];
  return 4;
}

int bsw_ctx_wait(bsw_ctx* c) {
  if (!c) return fail(BSW_EINVAL, "ctx is NULL");
  if (!c->pending) return BSW_OK;
  c->pending = false;
  HIPCHK(hipStreamSynchronize(c->pending_stream));
  return c->pending_done ? c->pending_done(c) : finish_call(c);
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

int bsw_ctx_last_work(bsw_ctx* c, int64_t* work, int32_t max) {
  if (!c) return fail(BSW_EINVAL, "ctx is NULL");
  const int n = std::min((int)max, c->n_launch);
  for (int k = 0; k < n && work; ++k) work[k] = (int64_t)c->lwork[k];
  return c->n_launch;
}

const char* bsw_class_name(int32_t cls) {
  static const char* names[NCLS + 1] = {
      "lane8_q32",  "lane8_q64",  "lane8_q96",  "lane8_q128", "lane8_q160",
      "lane8_q192", "lane8_q224", "lane8_q256", "lane16_q32", "lane16_q64",
      "lane16_q128", "lane16_q256", "lane32_q32", "lane32_q64", "lane32_q128",
      "lane32_q256", "long", "rerun"};
  static const char* wave_names[NLW] = {"wave32_q32", "wave32_q64", "wave32_q128",
                                        "wave32_q256"};
  if (cls >= CLS_W32 + WAVE_TAG && cls < CLS_LONG + WAVE_TAG)
    return wave_names[cls - WAVE_TAG - CLS_W32];
  return cls >= 0 && cls <= NCLS ? names[cls] : "?";
}

int bsw_ctx_last_cells(bsw_ctx* c, int64_t* cells) {
  if (!c || !cells) return fail(BSW_EINVAL, "NULL argument");
  *cells = (int64_t)c->last_cells;
  return BSW_OK;
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
  if (int rc0 = ctx_check_idle(c)) return rc0;
  if (n < 0 || n > 0x7fffffffLL) return fail(BSW_EINVAL, "n = %lld out of range", (long long)n);
  if (n == 0) return BSW_OK;
  int rc = check_params(params, n_params);
  if (rc) return rc;
  if (!q_off || !t_off || !h0 || !out) return fail(BSW_EINVAL, "a required pointer is NULL");
  // host-side validation of every pair before anything is staged
  int why = PF_NONE;
  const int64_t k = first_bad_pair(n, q, q_off, t, t_off, h0, param_id, n_params, &why);
  if (k >= 0) {
    switch (why) {
      case PF_OFFSETS:
        return fail(BSW_EINVAL, "pair %lld: bad offsets, length > %d or sequence NULL",
                    (long long)k, BSW_MAX_LEN);
      case PF_H0:
        return fail(BSW_EINVAL, "pair %lld: h0 = %d out of range", (long long)k, h0[k]);
      case PF_PID:
        return fail(BSW_EINVAL, "pair %lld: param_id %d >= n_params", (long long)k,
                    param_id[k]);
      case PF_QCODE:
        return fail(BSW_EINVAL, "pair %lld: query code > 4", (long long)k);
      default:
        return fail(BSW_EINVAL, "pair %lld: target code > 4", (long long)k);
    }
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
  const Args a = {n,
                 (const uint8_t*)(din + o_q),
                 (const uint64_t*)(din + o_qo),
                 (const uint8_t*)(din + o_t),
                 (const uint64_t*)(din + o_to),
                 (const int32_t*)(din + o_h0),
                 param_id ? (const uint8_t*)(din + o_pid) : nullptr,
                 n_params,
                 (bsw_result*)(dres + o_out),
                 diag ? (bsw_diag*)(dres + o_diag) : nullptr,
                 nullptr,
                 nullptr,
                 false};
  rc = run_pipeline(c, a, s);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(s));
  if ((rc = finish_call(c))) return rc;
  HIPCHK(hipMemcpyAsync(out, dres + o_out, sizeof(bsw_result) * (size_t)n,
                        hipMemcpyDeviceToHost, s));
  if (diag)
    HIPCHK(hipMemcpyAsync(diag, dres + o_diag, sizeof(bsw_diag) * (size_t)n,
                          hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return BSW_OK;
}

}  // extern "C"
