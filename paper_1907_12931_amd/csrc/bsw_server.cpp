// bsw_server.cpp -- serving loop of libbsw.so.
//
// Requests of many pairs arrive over time.  One scheduler thread owns all
// device work of the server and runs three steps in a loop:
//  1. admission: the oldest waiting request is given a region of the arena
//     when it fits (strict arrival order, so a large request is never
//     overtaken); its data is copied to the device on the upload stream and
//     its codes are checked there;
//  2. completion: a slot whose batch has finished hands each request its
//     results and releases the request's region;
//  3. dispatch: a free slot takes every admitted request whose data is
//     resident and valid, gathers their pairs into one batch on the device
//     and runs the batched path over it.
// Batches form from whatever is ready when a slot frees up, so new requests
// join the work between batches while the other slots keep the GPU busy
// (continuous batching at batch granularity).
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
  size_t o_st = 0, o_q = 0, o_t = 0, o_qo = 0, o_to = 0, o_h0 = 0, o_pid = 0, bytes = 0;
  size_t at = 0;
  Status* h_st = nullptr;  // pinned copy of the device status after the code check
  hipEvent_t ready = nullptr;
  ReqState state = QUEUED;
  int rc = BSW_OK;
  char err[160] = {0};
  Clock::time_point t_submit, t_admit, t_done;
};

enum SlotState { SLOT_FREE, SLOT_RUNNING, SLOT_COPYING };

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
  // pinned host: request table and results of the batch
  ReqSlice* h_tab = nullptr;
  int tab_cap = 0;
  void* h_res = nullptr;
  size_t h_res_cap = 0;
};

}  // namespace

struct bsw_server {
  bsw_server_opts opts;
  std::vector<bsw_params> params;
  char* arena_base = nullptr;
  Arena arena;
  hipStream_t up = nullptr;  // uploads and code checks
  std::deque<Slot> slots;  // a deque: slots hold atomics and never move
  std::vector<hipEvent_t> free_events;
  std::vector<Status*> free_status;
  std::vector<Status*> status_blocks;  // pinned allocations (freed at the end)

  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_copy;
  std::deque<int> copy_q;  // finished slots whose results wait to be handed out
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

// Bytes of a request's region: status, sequences, offsets, h0, param_id.
void plan_region(Req* r) {
  size_t o = 0;
  r->o_st = o;
  o = align_up(o + sizeof(Status), 256);
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
  o = align_up(o + (size_t)r->n, 256);
  r->bytes = o;
}

// Pinned status records, allocated in blocks and reused.
int take_status(bsw_server* v, Status** out) {
  if (v->free_status.empty()) {
    Status* blk = nullptr;
    SRVCHK(hipHostMalloc((void**)&blk, sizeof(Status) * 64, 0));
    v->status_blocks.push_back(blk);
    for (int i = 0; i < 64; ++i) v->free_status.push_back(blk + i);
  }
  *out = v->free_status.back();
  v->free_status.pop_back();
  return BSW_OK;
}

int take_event(bsw_server* v, hipEvent_t* out) {
  if (v->free_events.empty()) {
    hipEvent_t e = nullptr;
    SRVCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    v->free_events.push_back(e);
  }
  *out = v->free_events.back();
  v->free_events.pop_back();
  return BSW_OK;
}

// Copy an admitted request to its region and check its codes there; the
// request's ready event follows the copy of its status to the host.
int upload(bsw_server* v, Req* r) {
  char* base = v->arena_base + r->at;
  Status* st = (Status*)(base + r->o_st);
  uint8_t* dq = (uint8_t*)(base + r->o_q);
  uint8_t* dt = (uint8_t*)(base + r->o_t);
  uint64_t* dqo = (uint64_t*)(base + r->o_qo);
  uint64_t* dto = (uint64_t*)(base + r->o_to);
  int rc = take_status(v, &r->h_st);
  if (rc) return rc;
  if ((rc = take_event(v, &r->ready))) return rc;
  hipStream_t s = v->up;
  launch_fill((uint32_t*)st, sizeof(Status) / 4, s);
  if (r->qbytes) SRVCHK(hipMemcpyAsync(dq, r->q + r->q_off[0], r->qbytes, hipMemcpyHostToDevice, s));
  if (r->tbytes) SRVCHK(hipMemcpyAsync(dt, r->t + r->t_off[0], r->tbytes, hipMemcpyHostToDevice, s));
  SRVCHK(hipMemcpyAsync(dqo, r->q_off, 8 * (size_t)(r->n + 1), hipMemcpyHostToDevice, s));
  SRVCHK(hipMemcpyAsync(dto, r->t_off, 8 * (size_t)(r->n + 1), hipMemcpyHostToDevice, s));
  SRVCHK(hipMemcpyAsync(base + r->o_h0, r->h0, 4 * (size_t)r->n, hipMemcpyHostToDevice, s));
  if (r->pid)
    SRVCHK(hipMemcpyAsync(base + r->o_pid, r->pid, (size_t)r->n, hipMemcpyHostToDevice, s));
  // the code check indexes seq[off[k]] with the caller's offsets, so the
  // bytes are addressed through a base shifted back by the first offset
  launch_codes(dq - r->q_off[0], dqo, r->n, st, r->qbytes, s);
  launch_codes(dt - r->t_off[0], dto, r->n, st, r->tbytes, s);
  SRVCHK(hipGetLastError());
  SRVCHK(hipMemcpyAsync(r->h_st, st, sizeof(Status), hipMemcpyDeviceToHost, s));
  SRVCHK(hipEventRecord(r->ready, s));
  return BSW_OK;
}

// Grow a slot's buffers for a batch of n pairs from m requests.
int slot_reserve(Slot& sl, int64_t n, int m) {
  const size_t need = align_up(32 * (size_t)n, 256) + align_up(5 * (size_t)n, 256) +
                      align_up(40 * (size_t)n, 256) + align_up(sizeof(ReqSlice) * m, 256);
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
    sl.h_tab = nullptr;
    sl.tab_cap = 0;
    const int want = std::max(m * 2, 64);
    SRVCHK(hipHostMalloc((void**)&sl.h_tab, sizeof(ReqSlice) * want, 0));
    sl.tab_cap = want;
  }
  const size_t res = 40 * (size_t)n;
  if (res > sl.h_res_cap) {
    if (sl.h_res) (void)hipHostFree(sl.h_res);
    sl.h_res = nullptr;
    sl.h_res_cap = 0;
    const size_t want = std::max(res + res / 2, (size_t)1 << 20);
    SRVCHK(hipHostMalloc(&sl.h_res, want, 0));
    sl.h_res_cap = want;
  }
  return BSW_OK;
}

// Gather the slot's requests into one batch and enqueue it.
int launch_batch(bsw_server* v, Slot& sl) {
  const int m = (int)sl.reqs.size();
  int64_t n = 0;
  for (Req* r : sl.reqs) n += r->n;
  int rc = slot_reserve(sl, n, m);
  if (rc) return rc;
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
  hipStream_t s = sl.s;
  SRVCHK(hipMemcpyAsync(tab, sl.h_tab, sizeof(ReqSlice) * m, hipMemcpyHostToDevice, s));
  launch_assemble(tab, m, n, qb, qe, tb, te, h0, pid, s);
  SRVCHK(hipGetLastError());
  const uint8_t* ab = (const uint8_t*)v->arena_base;
  const Args a = {n,  ab,  qb,   ab, tb, h0, pid, (int32_t)v->params.size(),
                  out, diag, qe, te, true};
  if ((rc = ctx_enqueue(sl.ctx, a, s))) return rc;
  sl.want_diag = false;
  for (Req* r : sl.reqs) sl.want_diag = sl.want_diag || r->diag;
  // results, then diagnostics (contiguous after them) when asked for
  SRVCHK(hipMemcpyAsync(sl.h_res, out, (sl.want_diag ? 40 : 24) * (size_t)n,
                        hipMemcpyDeviceToHost, s));
  SRVCHK(hipEventRecord(sl.done, s));
  sl.state = SLOT_RUNNING;
  return BSW_OK;
}

// Mark a request finished (caller holds the lock) and release its region.
void finish_req(bsw_server* v, Req* r, int rc, Clock::time_point now) {
  r->rc = rc;
  r->state = DONE;
  r->t_done = now;
  v->arena.release(r->at, r->bytes);
  if (r->h_st) v->free_status.push_back(r->h_st);
  r->h_st = nullptr;
  if (r->ready) v->free_events.push_back(r->ready);
  r->ready = nullptr;
  if (rc == BSW_OK) {
    ++v->completed;
    v->pairs += r->n;
    v->lat.push_back(ms_between(r->t_submit, now));
  } else {
    ++v->failed;
  }
  v->last_done = now;
}

// Hand a finished batch's results to its requests.
void complete_slot(bsw_server* v, Slot& sl) {
  const int rc = ctx_finish(sl.ctx);
  const unsigned long long cells = rc == BSW_OK ? ctx_last_cells(sl.ctx) : 0;
  const bsw_result* res = (const bsw_result*)sl.h_res;
  const bsw_diag* dg = (const bsw_diag*)(res + sl.n);
  int64_t base = 0;
  for (Req* r : sl.reqs) {
    if (rc == BSW_OK) {
      std::memcpy(r->out, res + base, sizeof(bsw_result) * (size_t)r->n);
      if (r->diag) std::memcpy(r->diag, dg + base, sizeof(bsw_diag) * (size_t)r->n);
    }
    base += r->n;
  }
  const auto now = Clock::now();
  {
    std::lock_guard<std::mutex> g(v->mu);
    for (Req* r : sl.reqs) {
      if (rc != BSW_OK) std::snprintf(r->err, sizeof r->err, "%s", bsw_last_error());
      finish_req(v, r, rc, now);
    }
    ++v->batches;
    v->batch_pairs_sum += (double)sl.n;
    v->cells += cells;
  }
  v->cv_done.notify_all();
  sl.reqs.clear();
  sl.state = SLOT_FREE;
  v->cv_work.notify_one();
}

// Hands finished batches' results to their requests, so that the copies
// into the callers' buffers never hold up the scheduler.
void copier(bsw_server* v) {
  (void)hipSetDevice(v->opts.device);
  for (;;) {
    int k;
    {
      std::unique_lock<std::mutex> lk(v->mu);
      v->cv_copy.wait(lk, [&] { return !v->copy_q.empty() || v->copier_stop; });
      if (v->copy_q.empty()) return;
      k = v->copy_q.front();
      v->copy_q.pop_front();
    }
    complete_slot(v, v->slots[k]);
  }
}

void scheduler(bsw_server* v) {
  (void)hipSetDevice(v->opts.device);
  std::vector<Req*> to_upload;
  for (;;) {
    bool progress = false;
    to_upload.clear();
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
        to_upload.push_back(r);
      }
      bool busy = false;
      for (auto& sl : v->slots) busy = busy || sl.state != SLOT_FREE;
      if (v->stop && v->pending.empty() && v->admitted.empty() && !busy) break;
      if (to_upload.empty() && !busy && v->admitted.empty())
        v->cv_work.wait_for(lk, std::chrono::milliseconds(5));
    }
    for (Req* r : to_upload) {
      const int rc = upload(v, r);
      if (rc) {
        std::lock_guard<std::mutex> g(v->mu);
        std::snprintf(r->err, sizeof r->err, "%s", bsw_last_error());
        v->admitted.erase(std::find(v->admitted.begin(), v->admitted.end(), r));
        finish_req(v, r, rc, Clock::now());
        v->cv_done.notify_all();
      }
      progress = true;
    }
    // 2. completion: finished slots go to the copier
    for (size_t k = 0; k < v->slots.size(); ++k) {
      Slot& sl = v->slots[k];
      if (sl.state == SLOT_RUNNING && hipEventQuery(sl.done) == hipSuccess) {
        sl.state = SLOT_COPYING;
        {
          std::lock_guard<std::mutex> g(v->mu);
          v->copy_q.push_back((int)k);
        }
        v->cv_copy.notify_one();
        progress = true;
      }
    }
    // 3. dispatch: a free slot takes every ready admitted request
    for (auto& sl : v->slots) {
      if (sl.state != SLOT_FREE) continue;
      std::vector<Req*> batch;
      {
        std::lock_guard<std::mutex> g(v->mu);
        int64_t n = 0;
        for (auto it = v->admitted.begin(); it != v->admitted.end();) {
          Req* r = *it;
          if (hipEventQuery(r->ready) != hipSuccess) {
            ++it;
            continue;
          }
          if (r->h_st->bad) {  // a code > 4: the request fails alone
            std::snprintf(r->err, sizeof r->err,
                          "pair %llu is invalid (a code > 4)",
                          ~(unsigned long long)r->h_st->first_bad_inv);
            it = v->admitted.erase(it);
            finish_req(v, r, BSW_EINVAL, Clock::now());
            v->cv_done.notify_all();
            progress = true;
            continue;
          }
          if (!batch.empty() && n + r->n > v->opts.max_batch_pairs) break;
          n += r->n;
          r->state = RUNNING;
          batch.push_back(r);
          it = v->admitted.erase(it);
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
    if (sl.h_res) (void)hipHostFree(sl.h_res);
    if (sl.ctx) bsw_ctx_destroy(sl.ctx);
  }
  if (v->up) {
    (void)hipStreamSynchronize(v->up);
    (void)hipStreamDestroy(v->up);
  }
  for (auto e : v->free_events) (void)hipEventDestroy(e);
  for (auto b : v->status_blocks) (void)hipHostFree(b);
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
  if (o.max_inflight == 0) o.max_inflight = 2;
  if (o.max_inflight < 1 || o.max_inflight > 8)
    return set_error(BSW_EINVAL, "max_inflight must be 1..8");
  if (o.max_batch_pairs == 0) o.max_batch_pairs = (int64_t)1 << 22;
  if (o.max_batch_pairs < 1 || o.max_batch_pairs > 0x7fffffffLL)
    return set_error(BSW_EINVAL, "max_batch_pairs out of range");
  if (o.hbm_budget == 0) o.hbm_budget = (size_t)8 << 30;
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
  if (rc == BSW_OK) {
    v->params.assign(params, params + n_params);
    if (hipStreamCreateWithFlags(&v->up, hipStreamNonBlocking) != hipSuccess)
      rc = set_error(BSW_EDEVICE, "stream creation failed");
    else if (hipMalloc((void**)&v->arena_base, o.hbm_budget) != hipSuccess) {
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
