// bsw_server.cpp -- serving loop of libbsw.so.
//
// Requests of many pairs arrive over time.  One scheduler thread owns all
// device work of the server and runs three steps in a loop:
//  1. admission: the oldest waiting request is given a region of the arena
//     when it fits (strict arrival order, so a large request is never
//     overtaken);
//  2. completion: a slot whose batch has finished frees its requests'
//     regions and is free again at once; a copier thread hands the results
//     to each request;
//  3. dispatch: a free slot takes every admitted request, copies their data
//     to their regions on its own stream, checks their codes, gathers their
//     pairs into one batch on the device and runs the batched path over it.
// A slot's uploads run on its own stream, so they never wait behind the
// other slot's kernels on a shared hardware queue; while one slot uploads,
// the other computes.  Batches form from whatever is admitted when a slot
// frees up, so new requests join the work between batches while the other
// slots keep the GPU busy (continuous batching at batch granularity).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/bsw.h"
#include "bsw_internal.h"
#include "bsw_runtime.h"

using namespace bsw;

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

enum ReqState { QUEUED, ADMITTED, RUNNING, DONE };

struct Req {
  uint64_t ticket = 0;
  int64_t n = 0;
  const uint8_t* q = nullptr;
  const uint64_t* q_off = nullptr;
  const uint8_t* t = nullptr;
  const uint64_t* t_off = nullptr;
  const int32_t* h0 = nullptr;
  const uint8_t* pid = nullptr;
  bsw_result* out = nullptr;
  bsw_diag* diag = nullptr;
  uint64_t qbytes = 0, tbytes = 0;
  // region layout (offsets from the region start) and placement
  size_t o_q = 0, o_t = 0, o_qo = 0, o_to = 0, o_h0 = 0, o_pid = 0, bytes = 0;
  size_t at = 0;
  // the device's view of the request's arrays when they are in pinned host
  // memory (read by k_gather), else null (copied with hipMemcpyAsync):
  // query bytes, target bytes, q_off, t_off, h0, param_id
  const uint8_t* dsrc[6] = {};
  ReqState state = QUEUED;
  int rc = BSW_OK;
  char err[160] = {0};
  Clock::time_point t_submit, t_admit, t_done;
};

enum SlotState { SLOT_FREE, SLOT_RUNNING };

// A pinned host buffer for a batch's results (and diagnostics).
struct ResBuf {
  void* p = nullptr;
  size_t cap = 0;
};

// A finished batch whose results wait to be handed to its requests: the
// slot that ran it and the requests' device regions are already free.
struct Handoff {
  std::vector<Req*> reqs;
  ResBuf buf;
  int64_t n = 0;
  int rc = BSW_OK;
  unsigned long long cells = 0;
  std::string err;
};

struct Slot {
  bsw_ctx* ctx = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t done = nullptr;
  std::atomic<int> state{SLOT_FREE};
  bool want_diag = false;  // some request of the batch asked for diagnostics
  std::vector<Req*> reqs;
  int64_t n = 0;
  // device: assembled batch arrays and the request table
  void* dev = nullptr;
  size_t dev_cap = 0;
  // pinned host: request table, and the results buffer of the running
  // batch (taken from the server's pool at launch, handed on at completion)
  ReqSlice* h_tab = nullptr;
  int tab_cap = 0;
  CopySeg* h_seg = nullptr;  // pinned: the batch's copy list (6 per request)
  ResBuf res;
};

}  // namespace

struct bsw_server {
  bsw_server_opts opts;
  std::vector<bsw_params> params;
  char* arena_base = nullptr;
  Arena arena;
  std::deque<Slot> slots;  // a deque: slots hold atomics and never move

  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_copy;
  std::deque<Handoff> copy_q;  // finished batches whose results wait to be handed out
  std::vector<ResBuf> res_pool;  // pinned result buffers not in use
  bool copier_stop = false;
  std::thread copier;
  std::deque<Req*> pending;   // submitted, waiting for admission
  std::deque<Req*> admitted;  // admitted, not yet in a batch (arrival order)
  std::unordered_map<uint64_t, Req*> by_ticket;
  uint64_t next_ticket = 1;
  bool stop = false;
  int sched_err = BSW_OK;
  std::thread th;

  // measurement window
  int64_t submitted = 0, completed = 0, failed = 0, batches = 0, pairs = 0;
  unsigned long long cells = 0;
  double batch_pairs_sum = 0;
  std::vector<double> lat, admit_wait;
  bool have_first = false;
  Clock::time_point first_submit, last_done;
};

namespace {

#define SRVCHK(expr)                                                          \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess)                                                     \
      return set_error(e_ == hipErrorOutOfMemory ? BSW_ENOMEM : BSW_EDEVICE,  \
                       "%s failed: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

// Bytes of a request's region: sequences, offsets, h0, param_id.
void plan_region(Req* r) {
  size_t o = 0;
  r->o_q = o;
  o = align_up(o + r->qbytes + 4, 256);
  r->o_t = o;
  o = align_up(o + r->tbytes + 4, 256);
  r->o_qo = o;
  o = align_up(o + 8 * (size_t)(r->n + 1), 256);
  r->o_to = o;
  o = align_up(o + 8 * (size_t)(r->n + 1), 256);
  r->o_h0 = o;
  o = align_up(o + 4 * (size_t)r->n, 256);
  r->o_pid = o;
  o = align_up(o + (size_t)r->n + 4, 256);
  r->bytes = o;
}

// The device address of host memory the device can read (pinned and
// mapped), else null.  A failed query leaves no error behind.
const uint8_t* device_view(const void* p) {
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  if (at.type != hipMemoryTypeHost || !at.devicePointer) return nullptr;
  return (const uint8_t*)at.devicePointer;
}

// Queue an admitted request's data for its region: short ranges the device
// can read go to the copy list (one k_gather for the batch), the others are
// copied with hipMemcpyAsync on stream s (long ranges from pinned memory go
// to the copy engines, which run beside the other slot's kernels).
constexpr size_t GATHER_MAX = (size_t)1 << 20;
int upload(bsw_server* v, Req* r, CopySeg* segs, int* ns, unsigned long long* chunks,
           hipStream_t s) {
  char* base = v->arena_base + r->at;
  const void* src[6] = {r->q + r->q_off[0], r->t + r->t_off[0], r->q_off, r->t_off, r->h0,
                        r->pid};
  const size_t dst[6] = {r->o_q, r->o_t, r->o_qo, r->o_to, r->o_h0, r->o_pid};
  const size_t len[6] = {r->qbytes, r->tbytes, 8 * (size_t)(r->n + 1),
                         8 * (size_t)(r->n + 1), 4 * (size_t)r->n,
                         r->pid ? (size_t)r->n : 0};
  for (int k = 0; k < 6; ++k) {
    if (!len[k]) continue;
    if (r->dsrc[k] && len[k] < GATHER_MAX) {
      CopySeg& g = segs[(*ns)++];
      g.src = r->dsrc[k];
      g.dst = (uint8_t*)base + dst[k];
      g.bytes = len[k];
      g.chunk0 = *chunks;
      *chunks += (len[k] + 4095) / 4096;
    } else {
      SRVCHK(hipMemcpyAsync(base + dst[k], src[k], len[k], hipMemcpyHostToDevice, s));
    }
  }
  return BSW_OK;
}

// Grow a slot's buffers for a batch of n pairs from m requests.
int slot_reserve(Slot& sl, int64_t n, int m) {
  const size_t need = align_up(32 * (size_t)n, 256) + align_up(5 * (size_t)n, 256) +
                      align_up(40 * (size_t)n, 256) + align_up(sizeof(ReqSlice) * m, 256) +
                      align_up(8 * (size_t)m, 256) + align_up(sizeof(CopySeg) * 6 * m, 256);
  if (need > sl.dev_cap) {
    if (sl.dev) (void)hipFree(sl.dev);
    sl.dev = nullptr;
    sl.dev_cap = 0;
    const size_t want = std::max(need + need / 2, (size_t)1 << 20);
    SRVCHK(hipMalloc(&sl.dev, want));
    sl.dev_cap = want;
  }
  if (m > sl.tab_cap) {
    if (sl.h_tab) (void)hipHostFree(sl.h_tab);
    if (sl.h_seg) (void)hipHostFree(sl.h_seg);
    sl.h_tab = nullptr;
    sl.h_seg = nullptr;
    sl.tab_cap = 0;
    const int want = std::max(m * 2, 64);
    SRVCHK(hipHostMalloc((void**)&sl.h_tab, sizeof(ReqSlice) * want, 0));
    SRVCHK(hipHostMalloc((void**)&sl.h_seg, sizeof(CopySeg) * 6 * want, 0));
    sl.tab_cap = want;
  }
  return BSW_OK;
}

// A pinned results buffer of at least `bytes` for a slot's next batch: the
// slot's own, else one from the pool, else a new one (a too-small buffer
// goes back to the pool; pinned memory is only freed with the server).
int take_res(bsw_server* v, Slot& sl, size_t bytes) {
  if (sl.res.p && sl.res.cap >= bytes) return BSW_OK;
  std::lock_guard<std::mutex> g(v->mu);
  if (sl.res.p) v->res_pool.push_back(sl.res);
  sl.res = ResBuf();
  for (size_t k = 0; k < v->res_pool.size(); ++k)
    if (v->res_pool[k].cap >= bytes) {
      sl.res = v->res_pool[k];
      v->res_pool.erase(v->res_pool.begin() + (long)k);
      return BSW_OK;
    }
  const size_t want = std::max(bytes + bytes / 2, (size_t)1 << 20);
  SRVCHK(hipHostMalloc(&sl.res.p, want, 0));
  sl.res.cap = want;
  return BSW_OK;
}

// Gather the slot's requests into one batch and enqueue it.
int launch_batch(bsw_server* v, Slot& sl) {
  const int m = (int)sl.reqs.size();
  int64_t n = 0;
  for (Req* r : sl.reqs) n += r->n;
  int rc = slot_reserve(sl, n, m);
  if (rc) return rc;
  // results and diagnostics (40 B per pair), then each request's code flag
  if ((rc = take_res(v, sl, 40 * (size_t)n + 8 * (size_t)m))) return rc;
  sl.n = n;
  char* d = (char*)sl.dev;
  uint64_t* qb = (uint64_t*)d;
  uint64_t* qe = qb + n;
  uint64_t* tb = qe + n;
  uint64_t* te = tb + n;
  size_t o = align_up(32 * (size_t)n, 256);
  int32_t* h0 = (int32_t*)(d + o);
  uint8_t* pid = (uint8_t*)(h0 + n);
  o += align_up(5 * (size_t)n, 256);
  bsw_result* out = (bsw_result*)(d + o);
  bsw_diag* diag = (bsw_diag*)(out + n);
  o += align_up(40 * (size_t)n, 256);
  ReqSlice* tab = (ReqSlice*)(d + o);
  o += align_up(sizeof(ReqSlice) * m, 256);
  unsigned long long* bad = (unsigned long long*)(d + o);
  o += align_up(8 * (size_t)m, 256);
  CopySeg* segs = (CopySeg*)(d + o);
  hipStream_t s = sl.s;
  int ns = 0;
  unsigned long long chunks = 0;
  for (Req* r : sl.reqs)
    if ((rc = upload(v, r, sl.h_seg, &ns, &chunks, s))) return rc;
  if (ns) {
    SRVCHK(hipMemcpyAsync(segs, sl.h_seg, sizeof(CopySeg) * ns, hipMemcpyHostToDevice, s));
    launch_gather(segs, ns, chunks, s);
  }
  int64_t base = 0;
  for (int k = 0; k < m; ++k) {
    Req* r = sl.reqs[k];
    char* rb = v->arena_base + r->at;
    ReqSlice& e = sl.h_tab[k];
    e.base = base;
    e.n = r->n;
    e.q_at = (unsigned long long)(r->at + r->o_q);
    e.t_at = (unsigned long long)(r->at + r->o_t);
    e.q_off = (const uint64_t*)(rb + r->o_qo);
    e.t_off = (const uint64_t*)(rb + r->o_to);
    e.h0 = (const int32_t*)(rb + r->o_h0);
    e.pid = r->pid ? (const uint8_t*)(rb + r->o_pid) : nullptr;
    base += r->n;
  }
  SRVCHK(hipMemcpyAsync(tab, sl.h_tab, sizeof(ReqSlice) * m, hipMemcpyHostToDevice, s));
  // every byte must be a code 0..4; a request with a bad byte is flagged
  // and gets no bytes in the batch (it fails alone at completion)
  launch_fill((uint32_t*)bad, 2 * (int64_t)m, s);
  launch_req_codes(tab, m, n, (const uint8_t*)v->arena_base, bad, s);
  launch_assemble(tab, m, n, qb, qe, tb, te, h0, pid, bad, s);
  SRVCHK(hipGetLastError());
  const uint8_t* ab = (const uint8_t*)v->arena_base;
  const Args a = {n,  ab,  qb,   ab, tb, h0, pid, (int32_t)v->params.size(),
                  out, diag, qe, te, true};
  if ((rc = ctx_enqueue(sl.ctx, a, s))) return rc;
  sl.want_diag = false;
  for (Req* r : sl.reqs) sl.want_diag = sl.want_diag || r->diag;
  // results, then diagnostics (contiguous after them) when asked for
  SRVCHK(hipMemcpyAsync(sl.res.p, out, (sl.want_diag ? 40 : 24) * (size_t)n,
                        hipMemcpyDeviceToHost, s));
  SRVCHK(hipMemcpyAsync((char*)sl.res.p + 40 * (size_t)n, bad, 8 * (size_t)m,
                        hipMemcpyDeviceToHost, s));
  SRVCHK(hipEventRecord(sl.done, s));
  sl.state = SLOT_RUNNING;
  return BSW_OK;
}

// Release a request's device region (caller holds the lock).
void release_req(bsw_server* v, Req* r) {
  if (r->bytes) v->arena.release(r->at, r->bytes);
  r->bytes = 0;
}

// Mark a request finished (caller holds the lock); its region must already
// be released.
void done_req(bsw_server* v, Req* r, int rc, Clock::time_point now) {
  r->rc = rc;
  r->state = DONE;
  r->t_done = now;
  if (rc == BSW_OK) {
    ++v->completed;
    v->pairs += r->n;
    v->lat.push_back(ms_between(r->t_submit, now));
  } else {
    ++v->failed;
  }
  v->last_done = now;
}

// Both of the above (caller holds the lock).
void finish_req(bsw_server* v, Req* r, int rc, Clock::time_point now) {
  release_req(v, r);
  done_req(v, r, rc, now);
}

// Hand a finished batch's results to its requests (copier thread).
void hand_out(bsw_server* v, Handoff& h) {
  const bsw_result* res = (const bsw_result*)h.buf.p;
  const bsw_diag* dg = (const bsw_diag*)(res + h.n);
  const unsigned long long* bad =
      (const unsigned long long*)((const char*)h.buf.p + 40 * (size_t)h.n);
  std::vector<int> rc(h.reqs.size(), h.rc);
  int64_t base = 0;
  for (size_t k = 0; k < h.reqs.size(); ++k) {
    Req* r = h.reqs[k];
    if (h.rc == BSW_OK && bad[k]) {  // a code > 4: the request fails alone
      rc[k] = BSW_EINVAL;
      std::snprintf(r->err, sizeof r->err, "pair %llu is invalid (a code > 4)", ~bad[k]);
    } else if (h.rc == BSW_OK) {
      std::memcpy(r->out, res + base, sizeof(bsw_result) * (size_t)r->n);
      if (r->diag) std::memcpy(r->diag, dg + base, sizeof(bsw_diag) * (size_t)r->n);
    } else {
      std::snprintf(r->err, sizeof r->err, "%s", h.err.c_str());
    }
    base += r->n;
  }
  const auto now = Clock::now();
  {
    std::lock_guard<std::mutex> g(v->mu);
    for (size_t k = 0; k < h.reqs.size(); ++k) done_req(v, h.reqs[k], rc[k], now);
    ++v->batches;
    v->batch_pairs_sum += (double)h.n;
    v->cells += h.cells;
    v->res_pool.push_back(h.buf);
  }
  v->cv_done.notify_all();
}

// Hands finished batches' results to their requests, so that the copies
// into the callers' buffers never hold up the scheduler.
void copier(bsw_server* v) {
  (void)hipSetDevice(v->opts.device);
  for (;;) {
    Handoff h;
    {
      std::unique_lock<std::mutex> lk(v->mu);
      v->cv_copy.wait(lk, [&] { return !v->copy_q.empty() || v->copier_stop; });
      if (v->copy_q.empty()) return;
      h = std::move(v->copy_q.front());
      v->copy_q.pop_front();
    }
    hand_out(v, h);
  }
}

void scheduler(bsw_server* v) {
  (void)hipSetDevice(v->opts.device);
  for (;;) {
    bool progress = false;
    {
      std::unique_lock<std::mutex> lk(v->mu);
      // 1. admission, strictly in arrival order
      while (!v->pending.empty()) {
        Req* r = v->pending.front();
        size_t at = 0;
        if (!v->arena.alloc(r->bytes, &at)) break;
        v->pending.pop_front();
        r->at = at;
        r->state = ADMITTED;
        r->t_admit = Clock::now();
        v->admit_wait.push_back(ms_between(r->t_submit, r->t_admit));
        v->admitted.push_back(r);
        progress = true;
      }
      bool busy = false;
      for (auto& sl : v->slots) busy = busy || sl.state != SLOT_FREE;
      if (v->stop && v->pending.empty() && v->admitted.empty() && !busy) break;
      if (!progress && !busy && v->admitted.empty())
        v->cv_work.wait_for(lk, std::chrono::milliseconds(5));
    }
    // 2. completion: a finished batch frees its slot and its requests'
    //    regions at once; its results (in pinned memory) go to the copier
    for (auto& sl : v->slots) {
      if (sl.state != SLOT_RUNNING || hipEventQuery(sl.done) != hipSuccess) continue;
      Handoff h;
      h.rc = ctx_finish(sl.ctx);
      h.cells = h.rc == BSW_OK ? ctx_last_cells(sl.ctx) : 0;
      if (h.rc != BSW_OK) h.err = bsw_last_error();
      h.n = sl.n;
      h.reqs.swap(sl.reqs);
      h.buf = sl.res;
      sl.res = ResBuf();
      {
        std::lock_guard<std::mutex> g(v->mu);
        for (Req* r : h.reqs) release_req(v, r);
        v->copy_q.push_back(std::move(h));
      }
      sl.state = SLOT_FREE;
      v->cv_copy.notify_one();
      progress = true;
    }
    // 3. dispatch: a free slot takes the admitted requests in order, up to
    //    max_batch_pairs (a larger request runs alone)
    for (auto& sl : v->slots) {
      if (sl.state != SLOT_FREE) continue;
      std::vector<Req*> batch;
      {
        std::lock_guard<std::mutex> g(v->mu);
        int64_t n = 0;
        while (!v->admitted.empty()) {
          Req* r = v->admitted.front();
          if (!batch.empty() && n + r->n > v->opts.max_batch_pairs) break;
          n += r->n;
          r->state = RUNNING;
          batch.push_back(r);
          v->admitted.pop_front();
        }
      }
      if (batch.empty()) break;
      sl.reqs = batch;
      const int rc = launch_batch(v, sl);
      if (rc) {
        std::lock_guard<std::mutex> g(v->mu);
        for (Req* r : sl.reqs) {
          std::snprintf(r->err, sizeof r->err, "%s", bsw_last_error());
          finish_req(v, r, rc, Clock::now());
        }
        sl.reqs.clear();
        sl.state = SLOT_FREE;
        v->sched_err = rc;
        v->cv_done.notify_all();
      }
      progress = true;
    }
    if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

double percentile(std::vector<double> v, double p) {
  if (v.empty()) return 0;
  std::sort(v.begin(), v.end());
  const size_t k = (size_t)std::min<double>((double)v.size() - 1, p * (double)(v.size() - 1) + 0.5);
  return v[k];
}

void destroy_server(bsw_server* v) {
  (void)hipSetDevice(v->opts.device);
  for (auto& sl : v->slots) {
    if (sl.s) (void)hipStreamSynchronize(sl.s);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.dev) (void)hipFree(sl.dev);
    if (sl.h_tab) (void)hipHostFree(sl.h_tab);
    if (sl.h_seg) (void)hipHostFree(sl.h_seg);
    if (sl.res.p) (void)hipHostFree(sl.res.p);
    if (sl.ctx) bsw_ctx_destroy(sl.ctx);
  }
  for (auto& b : v->res_pool) (void)hipHostFree(b.p);
  for (auto& h : v->copy_q) (void)hipHostFree(h.buf.p);
  if (v->arena_base) (void)hipFree(v->arena_base);
  for (auto& kv : v->by_ticket) delete kv.second;
  delete v;
}

}  // namespace

extern "C" {

int bsw_server_create(bsw_server** out, const bsw_server_opts* opts,
                      const bsw_params* params, int32_t n_params) {
  if (!out) return set_error(BSW_EINVAL, "out is NULL");
  bsw_server_opts o;
  std::memset(&o, 0, sizeof o);
  if (opts) o = *opts;
  if (o.max_inflight == 0) o.max_inflight = 3;
  if (o.max_inflight < 1 || o.max_inflight > 8)
    return set_error(BSW_EINVAL, "max_inflight must be 1..8");
  if (o.max_batch_pairs == 0) o.max_batch_pairs = (int64_t)1 << 22;
  if (o.max_batch_pairs < 1 || o.max_batch_pairs > 0x7fffffffLL)
    return set_error(BSW_EINVAL, "max_batch_pairs out of range");
  if (o.hbm_budget == 0) o.hbm_budget = (size_t)16 << 30;
  if (o.max_queued == 0) o.max_queued = 65536;
  if (o.max_queued < 1) return set_error(BSW_EINVAL, "max_queued must be >= 1");
  bsw_server* v = new (std::nothrow) bsw_server;
  if (!v) return set_error(BSW_ENOMEM, "out of host memory");
  v->opts = o;
  int rc = BSW_OK;
  bsw_ctx_opts co;
  std::memset(&co, 0, sizeof co);
  co.device = o.device;
  co.min_lane_bits = o.min_lane_bits;
  co.path = BSW_PATH_BATCHED;
  co.no_graph = 1;  // every batch has its own shapes and pointers
  for (int k = 0; k < o.max_inflight; ++k) v->slots.emplace_back();
  for (auto& sl : v->slots) {
    if ((rc = bsw_ctx_create(&sl.ctx, &co))) break;
    if ((rc = ctx_set_params(sl.ctx, params, n_params))) break;
    // a slot runs its classes in order on its own stream: with one stream
    // per slot the slots hold separate hardware queues, so one slot's
    // uploads and kernels never wait behind the other's
    ctx_set_side_streams(sl.ctx, 0);
    // workspaces for a full batch up front: growing them later would free
    // device memory, which waits for all work on the device
    if ((rc = ctx_reserve(sl.ctx, o.max_batch_pairs, n_params))) break;
    if ((rc = slot_reserve(sl, o.max_batch_pairs, 1024))) break;
    sl.s = ctx_stream(sl.ctx);
    if (hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
      rc = set_error(BSW_EDEVICE, "event creation failed");
      break;
    }
  }
  // pinned results buffers for a full batch: one per slot and a spare, so
  // that a slot can start its next batch while the copier still hands out
  // the last one
  for (auto& sl : v->slots) {
    if (rc != BSW_OK) break;
    rc = take_res(v, sl, 40 * (size_t)o.max_batch_pairs);
  }
  if (rc == BSW_OK) {
    Slot spare;
    if ((rc = take_res(v, spare, 40 * (size_t)o.max_batch_pairs)) == BSW_OK)
      v->res_pool.push_back(spare.res);
  }
  if (rc == BSW_OK) {
    v->params.assign(params, params + n_params);
    if (hipMalloc((void**)&v->arena_base, o.hbm_budget) != hipSuccess) {
      v->arena_base = nullptr;
      rc = set_error(BSW_ENOMEM, "arena of %zu bytes does not fit", o.hbm_budget);
    }
  }
  if (rc != BSW_OK) {
    const std::string msg = bsw_last_error();
    destroy_server(v);
    return set_error(rc, "%s", msg.c_str());
  }
  v->arena.reset(o.hbm_budget);
  v->copier = std::thread(copier, v);
  v->th = std::thread(scheduler, v);
  *out = v;
  return BSW_OK;
}

void bsw_server_destroy(bsw_server* v) {
  if (!v) return;
  {
    std::lock_guard<std::mutex> g(v->mu);
    v->stop = true;
  }
  v->cv_work.notify_all();
  if (v->th.joinable()) v->th.join();
  {
    std::lock_guard<std::mutex> g(v->mu);
    v->copier_stop = true;
  }
  v->cv_copy.notify_all();
  if (v->copier.joinable()) v->copier.join();
  destroy_server(v);
}

int bsw_server_submit(bsw_server* v, int64_t n, const uint8_t* q, const uint64_t* q_off,
                      const uint8_t* t, const uint64_t* t_off, const int32_t* h0,
                      const uint8_t* param_id, bsw_result* out, bsw_diag* diag,
                      uint64_t* ticket) {
  if (!v || !ticket) return set_error(BSW_EINVAL, "server or ticket is NULL");
  if (n < 1 || n > 0x7fffffffLL) return set_error(BSW_EINVAL, "n = %lld out of range", (long long)n);
  if (!q || !q_off || !t || !t_off || !h0 || !out)
    return set_error(BSW_EINVAL, "a required pointer is NULL");
  const int np = (int)v->params.size();
  for (int64_t k = 0; k < n; ++k) {
    if (q_off[k + 1] < q_off[k] || t_off[k + 1] < t_off[k] ||
        q_off[k + 1] - q_off[k] > BSW_MAX_LEN || t_off[k + 1] - t_off[k] > BSW_MAX_LEN)
      return set_error(BSW_EINVAL, "pair %lld: bad offsets or length > %d", (long long)k,
                       BSW_MAX_LEN);
    if (h0[k] < 1 || h0[k] > BSW_MAX_H0)
      return set_error(BSW_EINVAL, "pair %lld: h0 = %d out of range", (long long)k, h0[k]);
    if (param_id && param_id[k] >= np)
      return set_error(BSW_EINVAL, "pair %lld: param_id %d >= n_params", (long long)k,
                       param_id[k]);
  }
  Req* r = new (std::nothrow) Req;
  if (!r) return set_error(BSW_ENOMEM, "out of host memory");
  r->n = n;
  r->q = q;
  r->q_off = q_off;
  r->t = t;
  r->t_off = t_off;
  r->h0 = h0;
  r->pid = param_id;
  r->out = out;
  r->diag = diag;
  r->qbytes = q_off[n] - q_off[0];
  r->tbytes = t_off[n] - t_off[0];
  {
    const void* src[6] = {q + q_off[0], t + t_off[0], q_off, t_off, h0, param_id};
    for (int k = 0; k < 6; ++k) r->dsrc[k] = src[k] ? device_view(src[k]) : nullptr;
  }
  plan_region(r);
  if (r->bytes > v->arena.size()) {
    const size_t b = r->bytes;
    delete r;
    return set_error(BSW_ETOOBIG, "request needs %zu bytes of the %zu-byte arena", b,
                     v->arena.size());
  }
  {
    std::lock_guard<std::mutex> g(v->mu);
    if ((int64_t)v->pending.size() >= v->opts.max_queued) {
      delete r;
      return set_error(BSW_EBUSY, "%d requests are waiting for admission", v->opts.max_queued);
    }
    r->ticket = v->next_ticket++;
    r->t_submit = Clock::now();
    if (!v->have_first) {
      v->have_first = true;
      v->first_submit = r->t_submit;
    }
    ++v->submitted;
    v->pending.push_back(r);
    v->by_ticket[r->ticket] = r;
    *ticket = r->ticket;
  }
  v->cv_work.notify_one();
  return BSW_OK;
}

int bsw_server_wait(bsw_server* v, uint64_t ticket, int32_t timeout_ms) {
  if (!v) return set_error(BSW_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(v->mu);
  auto it = v->by_ticket.find(ticket);
  if (it == v->by_ticket.end())
    return set_error(BSW_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  Req* r = it->second;
  auto done = [&] { return r->state == DONE; };
  if (timeout_ms < 0) {
    v->cv_done.wait(lk, done);
  } else if (!v->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done)) {
    return set_error(BSW_ETIMEOUT, "ticket %llu not complete after %d ms",
                     (unsigned long long)ticket, timeout_ms);
  }
  const int rc = r->rc;
  if (rc != BSW_OK) set_error(rc, "%s", r->err);
  v->by_ticket.erase(r->ticket);
  delete r;
  return rc;
}

int bsw_server_stats(bsw_server* v, bsw_server_report* out, int32_t reset) {
  if (!v || !out) return set_error(BSW_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> g(v->mu);
  std::memset(out, 0, sizeof *out);
  out->submitted = v->submitted;
  out->completed = v->completed;
  out->failed = v->failed;
  out->batches = v->batches;
  out->pairs = v->pairs;
  out->cells = (int64_t)v->cells;
  out->mean_batch_pairs = v->batches ? v->batch_pairs_sum / (double)v->batches : 0;
  out->lat_p50_ms = percentile(v->lat, 0.50);
  out->lat_p99_ms = percentile(v->lat, 0.99);
  out->lat_p999_ms = percentile(v->lat, 0.999);
  out->lat_max_ms = v->lat.empty() ? 0 : *std::max_element(v->lat.begin(), v->lat.end());
  double s = 0;
  for (double x : v->admit_wait) s += x;
  out->admit_wait_mean_ms = v->admit_wait.empty() ? 0 : s / (double)v->admit_wait.size();
  out->admit_wait_p99_ms = percentile(v->admit_wait, 0.99);
  out->window_s = v->have_first && v->completed + v->failed > 0
                      ? ms_between(v->first_submit, v->last_done) / 1e3
                      : 0;
  out->gcups = out->window_s > 0 ? (double)v->cells / out->window_s / 1e9 : 0;
  if (reset) {
    v->submitted = v->completed = v->failed = v->batches = v->pairs = 0;
    v->cells = 0;
    v->batch_pairs_sum = 0;
    v->lat.clear();
    v->admit_wait.clear();
    v->have_first = false;
  }
  return BSW_OK;
}

}  // extern "C"
