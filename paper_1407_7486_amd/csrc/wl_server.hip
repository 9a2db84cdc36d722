// Serving loop: continuous batching of uneven Wilson-loop requests against a
// device-resident ensemble.
//
// A scheduler thread owns `slots` batch slots.  Each slot has its own stream
// (default priority), pinned host staging, a device region for descriptors,
// grids and results, a work counter, and one captured hipGraph per precision
// (H2D of the staging -> counter reset -> persistent batch kernel ->
// sub-range reduction -> statistics).  The batch kernels read the batch's
// composition from device memory, so a slot's graph is replayed for every
// batch.  Requests are admitted first-come first-served into a free slot
// while their partial-sum memory (group sums, sub-range partials, means,
// errors) fits the slot's budget; with two slots in flight the next batch's
// workgroups take over the compute units as the previous batch drains.
// Every request is decomposed exactly as when evaluated alone, so its result
// does not depend on what it was batched with.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "wl_host.h"

using Clock = std::chrono::steady_clock;

namespace {

struct Ticket {
  int64_t id = 0;
  wl_request req{};  // rho / T point into the owned copies below
  std::vector<double> rho, T;
  wl::FieldArgs fa{};
  wl::ReqPlan plan;
  int32_t state = 1;  // 1 queued, 2 running, 0 done, < 0 error
  Clock::time_point t_submit, t_launch, t_done;
};

struct Slot {
  hipStream_t stream = nullptr;
  void* h_in = nullptr;  // pinned staging of header, descriptors, grids
  void* d_in = nullptr;
  void* d_res = nullptr;
  double* h_res = nullptr;  // pinned copy of sums, means, errors
  unsigned int* d_counter = nullptr;
  hipEvent_t ev_done = nullptr;  // recorded after the batch's results are copied
  hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};
  hipGraph_t graph[3] = {nullptr, nullptr, nullptr};
  bool busy = false;
  std::atomic<bool> done{false};
  std::vector<Ticket*> reqs;
  wl::BatchLayout lay;
  int prec = 0;
};

}  // namespace

struct wl_server {
  wl_ctx* ctx = nullptr;
  const wl_ens* ens = nullptr;
  wl_server_config cfg{};
  std::vector<std::unique_ptr<Slot>> slots;
  std::deque<Ticket*> pending;
  std::map<int64_t, std::unique_ptr<Ticket>> tickets;
  std::mutex mu;
  std::condition_variable cv;       // scheduler wake-ups
  std::condition_variable cv_done;  // request completions
  std::thread th;
  bool stop = false;
  int64_t next_id = 1;
  int fatal = WL_OK;  // first HIP failure: the server then fails everything
  std::string err;
  int64_t n_batches = 0;
  Slot* last = nullptr;  // the slot launched most recently (in-order mode)
};

namespace {

int sfail(wl_server* s, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  s->err = buf;
  return code;
}

void host_done(void* p) {
  // runs on a HIP runtime thread: no HIP calls, no locks
  static_cast<Slot*>(p)->done.store(true, std::memory_order_release);
}

int32_t persistent_wgs(const wl_server* s) { return s->ctx->num_cu * 8; }

// Captures the device work of one batch of precision `prec` on slot `sl`.
hipError_t capture(wl_server* s, Slot* sl, int prec) {
  const wl_ens* e = s->ens;
  if (prec == WL_FP64) {
    // the FP64 segment array is built (once, outside the capture) before
    // the first FP64 batch
    const hipError_t b = wl::ensure_seg64(e, sl->stream);
    if (b != hipSuccess) return b;
  }
  hipError_t st = hipStreamBeginCapture(sl->stream, hipStreamCaptureModeThreadLocal);
  if (st != hipSuccess) return st;
  hipError_t r = hipMemcpyAsync(sl->d_in, sl->h_in, s->cfg.input_bytes, hipMemcpyHostToDevice,
                                sl->stream);
  if (r == hipSuccess)
    r = wl::launch_batch(prec, e->d_seg, e->d_seg64, e->d_norm, e->d_x, e->d_y, e->n_ppl,
                         sl->d_in, e->n_groups, e->n_loops, sl->d_counter,
                         (double*)sl->d_res, persistent_wgs(s), sl->stream);
  hipGraph_t g = nullptr;
  st = hipStreamEndCapture(sl->stream, &g);
  if (r != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return r;
  }
  if (st != hipSuccess) return st;
  st = hipGraphInstantiate(&sl->exec[prec], g, nullptr, nullptr, 0);
  if (st != hipSuccess) {
    (void)hipGraphDestroy(g);
    return st;
  }
  sl->graph[prec] = g;
  return hipSuccess;
}

void finish_ticket(wl_server* s, Ticket* t, int32_t state) {
  t->state = state;
  t->t_done = Clock::now();
  (void)s;
}

// Picks the next batch for a free slot (called with the lock held): the
// oldest pending request fixes the precision; later requests of that
// precision join in arrival order while they fit the slot's budget.
void pick_batch(wl_server* s, Slot* sl) {
  sl->reqs.clear();
  if (s->pending.empty()) return;
  const int prec = s->pending.front()->req.precision;
  size_t in_b = wl::kBatchDescOffset + 256, res_b = 0;
  for (auto it = s->pending.begin(); it != s->pending.end();) {
    Ticket* t = *it;
    if (t->req.precision != prec) {
      ++it;
      continue;
    }
    if ((int32_t)sl->reqs.size() >= s->cfg.max_batch ||
        in_b + t->plan.in_bytes > s->cfg.input_bytes ||
        res_b + t->plan.res_bytes > s->cfg.result_bytes)
      break;  // keep arrival order: later requests wait behind this one
    in_b += t->plan.in_bytes;
    res_b += t->plan.res_bytes;
    sl->reqs.push_back(t);
    t->state = 2;
    it = s->pending.erase(it);
  }
  sl->prec = prec;
}

// Launches the slot's batch (without the lock).  prev: the slot launched
// before it, whose batch this one waits for on the device (in-order mode;
// nullptr: no wait).
hipError_t launch_slot(wl_server* s, Slot* sl, Slot* prev) {
  std::vector<const wl_request*> rq;
  std::vector<wl::FieldArgs> fa;
  std::vector<wl::ReqPlan> pl;
  for (Ticket* t : sl->reqs) {
    rq.push_back(&t->req);
    fa.push_back(t->fa);
    pl.push_back(t->plan);
  }
  if (!wl::build_batch(s->ens, rq.data(), fa.data(), pl.data(), (int32_t)rq.size(), sl->h_in,
                       s->cfg.input_bytes, sl->d_in, sl->d_res, s->cfg.result_bytes,
                       &sl->lay))
    return hipErrorInvalidValue;  // admission guarantees the fit
  hipError_t e = hipSuccess;
  if (!sl->exec[sl->prec]) e = capture(s, sl, sl->prec);
  // read under the lock only once the ticket is done (its state is set
  // under the lock after this)
  const Clock::time_point now = Clock::now();
  for (Ticket* t : sl->reqs) t->t_launch = now;
  if (e == hipSuccess && prev) e = hipStreamWaitEvent(sl->stream, prev->ev_done, 0);
  if (e == hipSuccess) e = hipGraphLaunch(sl->exec[sl->prec], sl->stream);
  const size_t out_b = sl->lay.head_bytes;
  if (e == hipSuccess)
    e = hipMemcpyAsync(sl->h_res, sl->d_res, out_b, hipMemcpyDeviceToHost, sl->stream);
  if (e == hipSuccess) e = hipEventRecord(sl->ev_done, sl->stream);
  sl->done.store(false, std::memory_order_relaxed);
  if (e == hipSuccess) e = hipLaunchHostFunc(sl->stream, host_done, sl);
  return e;
}

void scheduler(wl_server* s) {
  wl::DeviceGuard g(s->ctx->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    bool any_busy = false;
    // harvest finished batches
    for (auto& up : s->slots) {
      Slot* sl = up.get();
      if (!sl->busy || !sl->done.load(std::memory_order_acquire)) {
        any_busy |= sl->busy;
        continue;
      }
      for (size_t i = 0; i < sl->reqs.size(); ++i) {
        wl::scatter_results(sl->reqs[i]->req, sl->lay, (int32_t)i, sl->h_res,
                            s->ens->n_groups);
        finish_ticket(s, sl->reqs[i], 0);
      }
      sl->reqs.clear();
      sl->busy = false;
      s->cv_done.notify_all();
    }
    if (s->fatal != WL_OK) {
      for (Ticket* t : s->pending) finish_ticket(s, t, s->fatal);
      s->pending.clear();
      s->cv_done.notify_all();
    }
    // start batches in free slots
    for (auto& up : s->slots) {
      Slot* sl = up.get();
      if (sl->busy || s->pending.empty() || s->fatal != WL_OK) continue;
      pick_batch(s, sl);
      if (sl->reqs.empty()) continue;
      sl->busy = true;
      any_busy = true;
      s->n_batches++;
      // the previous slot's event is recorded by its own launch, which
      // happened before this one (same thread)
      Slot* prev = s->cfg.in_order && s->last && s->last != sl ? s->last : nullptr;
      s->last = sl;
      lk.unlock();
      const hipError_t e = launch_slot(s, sl, prev);
      lk.lock();
      if (e != hipSuccess) {
        sfail(s, WL_EHIP, "batch launch: %s", hipGetErrorString(e));
        s->fatal = WL_EHIP;
        for (Ticket* t : sl->reqs) finish_ticket(s, t, WL_EHIP);
        sl->reqs.clear();
        sl->busy = false;
        s->cv_done.notify_all();
      }
    }
    if (s->stop && s->pending.empty() && !any_busy) break;
    // completions are signalled by a flag (no lock in the HIP callback), so
    // poll them at a short interval while batches are in flight
    s->cv.wait_for(lk, any_busy ? std::chrono::microseconds(200)
                                : std::chrono::milliseconds(20));
  }
}

}  // namespace

extern "C" {

int wl_server_create(wl_ctx* ctx, const wl_ens* ens, const wl_server_config* cfg,
                     wl_server** out) {
  if (!ctx) return WL_EINVAL;
  ctx->err.clear();
  if (!out) return wl::fail(ctx, WL_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = wl::check_common(ctx, ens, 0, WL_FP32C);
  if (rc) return rc;
  wl_server_config c{};
  c.slots = 2;
  c.max_batch = 1024;
  c.input_bytes = (size_t)8 << 20;
  c.result_bytes = (size_t)512 << 20;
  if (cfg) {
    if (cfg->slots < 1 || cfg->slots > 8) return wl::fail(ctx, WL_EINVAL, "slots must be 1..8");
    if (cfg->max_batch < 1) return wl::fail(ctx, WL_EINVAL, "max_batch must be >= 1");
    if (cfg->input_bytes < 4096 || cfg->result_bytes < 4096)
      return wl::fail(ctx, WL_EINVAL, "slot budgets must be >= 4096 bytes");
    if (cfg->in_order != 0 && cfg->in_order != 1)
      return wl::fail(ctx, WL_EINVAL, "in_order must be 0 or 1");
    c = *cfg;
  }
  c.input_bytes = (c.input_bytes + 255) & ~(size_t)255;
  c.result_bytes = (c.result_bytes + 255) & ~(size_t)255;
  wl::DeviceGuard g(ctx->device);
  if (g.status != hipSuccess) return wl::hip_fail(ctx, g.status, "hipSetDevice");
  auto s = std::make_unique<wl_server>();
  s->ctx = ctx;
  s->ens = ens;
  s->cfg = c;
  for (int i = 0; i < c.slots; ++i) {
    auto sl = std::make_unique<Slot>();
    hipError_t e = hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipHostMalloc(&sl->h_in, c.input_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&sl->h_res, c.result_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc(&sl->d_in, c.input_bytes);
    if (e == hipSuccess) e = hipMalloc(&sl->d_res, c.result_bytes);
    if (e == hipSuccess)
      e = hipMalloc((void**)&sl->d_counter, wl::kBatchCounters * sizeof(unsigned int));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl->ev_done, hipEventDisableTiming);
    s->slots.push_back(std::move(sl));
    if (e != hipSuccess) {
      wl_server* raw = s.release();
      raw->stop = true;
      wl_server_destroy(raw);
      (void)hipGetLastError();
      return wl::fail(ctx, WL_ENOMEM, "server slot allocation: %s", hipGetErrorString(e));
    }
  }
  s->th = std::thread(scheduler, s.get());
  *out = s.release();
  return WL_OK;
}

int wl_server_submit(wl_server* s, const wl_request* req, int64_t* ticket) {
  if (!s || !req || !ticket) return WL_EINVAL;
  wl_ctx* ctx = s->ctx;
  auto t = std::make_unique<Ticket>();
  std::lock_guard<std::mutex> lk(s->mu);
  s->err.clear();
  if (s->stop) return sfail(s, WL_EINVAL, "server is stopping");
  if (s->fatal != WL_OK) return sfail(s, s->fatal, "server failed earlier");
  // validation reuses the context's checks; their message is copied here
  int rc = wl::check_common(ctx, s->ens, req->spin, req->precision);
  if (!rc) rc = wl::check_not_study(ctx, req->precision);
  if (!rc) rc = wl::check_field(ctx, &req->field, &t->fa);
  if (!rc) rc = wl::check_grid(ctx, req->rho, req->n_rho, req->T, req->n_T);
  if (rc) return sfail(s, rc, "%s", ctx->err.c_str());
  t->req = *req;
  t->rho.assign(req->rho, req->rho + req->n_rho);
  t->T.assign(req->T, req->T + req->n_T);
  t->req.rho = t->rho.data();
  t->req.T = t->T.data();
  t->plan = wl::plan_request(ctx, s->ens, t->req);
  t->id = s->next_id++;
  t->t_submit = Clock::now();
  const size_t in_need = wl::kBatchDescOffset + 512 + t->plan.in_bytes;
  if (t->plan.n_pts > 0 &&
      (in_need > s->cfg.input_bytes || t->plan.res_bytes > s->cfg.result_bytes))
    return sfail(s, WL_ENOMEM,
                 "request needs %zu result / %zu input bytes, above the slot budget "
                 "(%zu / %zu)",
                 t->plan.res_bytes, in_need, s->cfg.result_bytes, s->cfg.input_bytes);
  *ticket = t->id;
  Ticket* raw = t.get();
  s->tickets[t->id] = std::move(t);
  if (raw->plan.n_pts == 0) {
    finish_ticket(s, raw, 0);  // empty grid: nothing to compute
  } else {
    s->pending.push_back(raw);
    s->cv.notify_all();
  }
  return WL_OK;
}

int wl_server_poll(wl_server* s, int64_t ticket, int32_t* status, double* latency_ms) {
  if (!s || !status) return WL_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return sfail(s, WL_EINVAL, "unknown ticket %lld", (long long)ticket);
  Ticket* t = it->second.get();
  *status = t->state;
  if (latency_ms)
    *latency_ms = (t->state <= 0)
                      ? std::chrono::duration<double, std::milli>(t->t_done - t->t_submit).count()
                      : -1.0;
  return WL_OK;
}

int wl_server_wait(wl_server* s, int64_t ticket, double timeout_s, int32_t* status,
                   double* latency_ms) {
  if (!s || !status) return WL_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return sfail(s, WL_EINVAL, "unknown ticket %lld", (long long)ticket);
  Ticket* t = it->second.get();
  const auto deadline =
      Clock::now() + std::chrono::duration_cast<Clock::duration>(
                         std::chrono::duration<double>(timeout_s < 0 ? 1e9 : timeout_s));
  while (t->state > 0) {
    if (s->cv_done.wait_until(lk, deadline) == std::cv_status::timeout && t->state > 0) break;
  }
  *status = t->state;
  if (latency_ms)
    *latency_ms = (t->state <= 0)
                      ? std::chrono::duration<double, std::milli>(t->t_done - t->t_submit).count()
                      : -1.0;
  return WL_OK;
}

int wl_server_timing(wl_server* s, int64_t ticket, double* queue_ms, double* service_ms) {
  if (!s || !queue_ms || !service_ms) return WL_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return sfail(s, WL_EINVAL, "unknown ticket %lld", (long long)ticket);
  const Ticket* t = it->second.get();
  using Ms = std::chrono::duration<double, std::milli>;
  // (a request with no grid points finishes without a launch)
  const bool ran = t->state <= 0 && t->t_launch >= t->t_submit;
  *queue_ms = ran ? Ms(t->t_launch - t->t_submit).count() : -1.0;
  *service_ms = ran ? Ms(t->t_done - t->t_launch).count() : -1.0;
  return WL_OK;
}

int wl_server_release(wl_server* s, int64_t ticket) {
  if (!s) return WL_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return sfail(s, WL_EINVAL, "unknown ticket %lld", (long long)ticket);
  if (it->second->state > 0) return sfail(s, WL_EINVAL, "ticket %lld is not finished", (long long)ticket);
  s->tickets.erase(it);
  return WL_OK;
}

int wl_server_info(wl_server* s, int64_t* pending, int64_t* running, int64_t* batches) {
  if (!s) return WL_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  int64_t run = 0;
  for (auto& sl : s->slots) run += (int64_t)sl->reqs.size();
  if (pending) *pending = (int64_t)s->pending.size();
  if (running) *running = run;
  if (batches) *batches = s->n_batches;
  return WL_OK;
}

const char* wl_server_last_error(const wl_server* s) { return s ? s->err.c_str() : ""; }

int wl_server_destroy(wl_server* s) {
  if (!s) return WL_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  if (s->th.joinable()) s->th.join();  // drains pending and in-flight work
  wl::DeviceGuard g(s->ctx->device);
  for (auto& sl : s->slots) {
    if (sl->stream) (void)hipStreamSynchronize(sl->stream);
    for (int p = 0; p < 3; ++p) {
      if (sl->exec[p]) (void)hipGraphExecDestroy(sl->exec[p]);
      if (sl->graph[p]) (void)hipGraphDestroy(sl->graph[p]);
    }
    if (sl->h_in) (void)hipHostFree(sl->h_in);
    if (sl->h_res) (void)hipHostFree(sl->h_res);
    if (sl->d_in) (void)hipFree(sl->d_in);
    if (sl->d_res) (void)hipFree(sl->d_res);
    if (sl->d_counter) (void)hipFree(sl->d_counter);
    if (sl->ev_done) (void)hipEventDestroy(sl->ev_done);
    if (sl->stream) (void)hipStreamDestroy(sl->stream);
  }
  delete s;
  return WL_OK;
}

}  // extern "C"
