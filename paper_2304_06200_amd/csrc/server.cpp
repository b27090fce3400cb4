// Serving loop of libhgrape: continuous admission of cost+gradient requests of
// different problems and shapes onto one GPU.
//
// A request is admitted when a worker slot is free and its device footprint
// (evaluation workspace plus its own input and gradient buffers) fits in the
// HBM budget next to the requests already running; admission is first come,
// first served.  Each worker owns one HIP stream (default priority) and runs
// admitted requests to completion with hg_eval, so kernels of concurrent
// requests overlap on the device and a request that arrives while others run
// starts as soon as a slot and memory free up.  Results are per request and
// deterministic: a request's numbers do not depend on what runs beside it.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "hg_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t id = 0;
  hg_problem* p = nullptr;
  hg_eval_desc desc{};
  std::vector<int32_t> schedule;  // private copy of a frozen schedule
  hg_result* results = nullptr;
  double* grad = nullptr;
  hipEvent_t ready = nullptr;     // recorded on the caller's stream at submit
  size_t bytes = 0;
  int state = 0;  // 0 queued, 1 running, 2 done
  hg_status status = HG_OK;
  std::string error;
  Clock::time_point t_submit, t_start, t_end;
};

}  // namespace

struct hg_server {
  hg_ctx* ctx = nullptr;
  size_t budget = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::map<uint64_t, std::shared_ptr<Request>> reqs;
  size_t in_use = 0;
  int running = 0;
  uint64_t next_id = 1;
  bool stopping = false;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
};

namespace {

constexpr size_t kMaxQueued = 1 << 16;

void worker_loop(hg_server* sv, int w) {
  (void)hipSetDevice(sv->ctx->device);
  for (;;) {
    std::shared_ptr<Request> r;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv_work.wait(lk, [&] {
        return (sv->stopping && sv->queue.empty()) ||
               (!sv->queue.empty() && sv->in_use + sv->queue.front()->bytes <= sv->budget);
      });
      if (sv->queue.empty()) return;  // stopping and drained
      r = sv->queue.front();
      sv->queue.pop_front();
      sv->in_use += r->bytes;
      sv->running += 1;
      r->state = 1;
      r->t_start = Clock::now();
    }
    if (!r->schedule.empty()) r->desc.schedule = r->schedule.data();
    hg_status st = HG_OK;
    std::string err;
    try {  // no exception may end a worker thread (or cross the C ABI)
      // the inputs are complete once the caller's stream reaches the submit point
      if (r->ready) {
        const hipError_t e = hipStreamWaitEvent(sv->streams[w], r->ready, 0);
        (void)hipEventDestroy(r->ready);
        r->ready = nullptr;
        if (e != hipSuccess) {
          st = HG_ERR_DEVICE;
          err = std::string("hipStreamWaitEvent: ") + hipGetErrorString(e);
        }
      }
      if (st == HG_OK) {
        st = hg_eval(r->p, &r->desc, r->results, r->grad, sv->streams[w]);
        if (st != HG_OK) err = hg_last_error();
      }
    } catch (const std::bad_alloc&) {
      st = HG_ERR_OUT_OF_MEMORY;
      err = "host allocation failed";
    } catch (...) {
      st = HG_ERR_DEVICE;
      err = "unexpected exception in the evaluation";
    }
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->in_use -= r->bytes;
      sv->running -= 1;
      r->status = st;
      r->error = err;
      r->state = 2;
      r->t_end = Clock::now();
    }
    sv->cv_done.notify_all();
    sv->cv_work.notify_all();
  }
}

size_t request_bytes(const hg_problem* p, const hg_eval_desc* d, size_t workspace) {
  const size_t B = (size_t)d->n_batch, N = (size_t)d->n_steps, S = (size_t)d->n_states;
  const size_t K = (size_t)p->n_ctrl, dim = (size_t)p->dim;
  return workspace + 8 * B * K * N /* u */ + 2 * 16 * B * S * dim /* psi0, targets */ +
         8 * B * K * N /* grad */;
}

}  // namespace

extern "C" {

hg_status hg_server_create(hg_ctx* ctx, size_t hbm_budget_bytes, int32_t max_inflight,
                           hg_server** out) {
  if (!ctx || !out || max_inflight < 1 || max_inflight > 256 || hbm_budget_bytes == 0) {
    hg::set_error("hg_server_create: bad argument");
    return HG_ERR_INVALID_ARG;
  }
  try {
  auto sv = std::make_unique<hg_server>();
  sv->ctx = ctx;
  sv->budget = hbm_budget_bytes;
  if (hipSetDevice(ctx->device) != hipSuccess) {
    hg::set_error("hipSetDevice failed");
    return HG_ERR_DEVICE;
  }
  for (int i = 0; i < max_inflight; ++i) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      for (auto x : sv->streams) (void)hipStreamDestroy(x);
      hg::set_error("hipStreamCreate failed");
      return HG_ERR_DEVICE;
    }
    sv->streams.push_back(s);
  }
  hg_server* raw = sv.get();
  try {
    for (int i = 0; i < max_inflight; ++i) sv->workers.emplace_back(worker_loop, raw, i);
  } catch (...) {  // stop the workers that did start before the server goes away
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->stopping = true;
    }
    sv->cv_work.notify_all();
    for (auto& t : sv->workers) t.join();
    for (auto x : sv->streams) (void)hipStreamDestroy(x);
    throw;
  }
  *out = sv.release();
  return HG_OK;
  } catch (const std::exception& e) {
    hg::set_error(std::string("hg_server_create: ") + e.what());
    return HG_ERR_OUT_OF_MEMORY;
  }
}

hg_status hg_server_submit(hg_server* sv, hg_problem* p, const hg_eval_desc* desc,
                           hg_result* results, double* grad, void* after_stream,
                           uint64_t* req_id) {
  if (!sv || !p || !desc || !results || !req_id) {
    hg::set_error("hg_server_submit: NULL argument");
    return HG_ERR_INVALID_ARG;
  }
  size_t ws = 0;
  hg_status st = hg_eval_footprint(p, desc, &ws);
  if (st != HG_OK) return st;
  try {
  auto r = std::make_shared<Request>();
  r->p = p;
  r->desc = *desc;
  if (desc->schedule) {
    const size_t n = (size_t)2 * desc->n_batch * desc->n_steps;
    r->schedule.assign(desc->schedule, desc->schedule + n);
  }
  r->results = results;
  r->grad = grad;
  r->bytes = request_bytes(p, desc, ws);
  if (r->bytes > sv->budget) {
    hg::set_error("request needs " + std::to_string(r->bytes) + " B of device memory; budget is " +
                  std::to_string(sv->budget) + " B");
    return HG_ERR_OUT_OF_MEMORY;
  }
  // the request's worker waits for what the caller queued on after_stream so far
  int prev_dev = -1;
  (void)hipGetDevice(&prev_dev);
  const bool made = hipSetDevice(sv->ctx->device) == hipSuccess &&
                    hipEventCreateWithFlags(&r->ready, hipEventDisableTiming) == hipSuccess;
  if (prev_dev >= 0 && prev_dev != sv->ctx->device) (void)hipSetDevice(prev_dev);
  if (!made) {
    r->ready = nullptr;
    hg::set_error("hg_server_submit: hipEventCreate failed");
    return HG_ERR_DEVICE;
  }
  if (hipEventRecord(r->ready, (hipStream_t)after_stream) != hipSuccess) {
    (void)hipEventDestroy(r->ready);
    r->ready = nullptr;
    hg::set_error("hg_server_submit: hipEventRecord on the caller's stream failed");
    return HG_ERR_DEVICE;
  }
  struct Unready {  // a request refused below never reaches a worker
    Request* r;
    bool armed = true;
    ~Unready() {
      if (armed && r->ready) {
        (void)hipEventDestroy(r->ready);
        r->ready = nullptr;
      }
    }
  } unready{r.get()};
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stopping) {
      hg::set_error("server is shutting down");
      return HG_ERR_BUSY;
    }
    if (sv->queue.size() >= kMaxQueued) {
      hg::set_error("request queue is full");
      return HG_ERR_BUSY;
    }
    r->id = sv->next_id++;
    r->t_submit = Clock::now();
    sv->queue.push_back(r);
    sv->reqs[r->id] = r;
    *req_id = r->id;
    unready.armed = false;
  }
  sv->cv_work.notify_one();
  return HG_OK;
  } catch (const std::bad_alloc&) {
    hg::set_error("hg_server_submit: host allocation failed");
    return HG_ERR_OUT_OF_MEMORY;
  }
}

hg_status hg_server_poll(hg_server* sv, uint64_t req_id, int32_t* done) {
  if (!sv || !done) return HG_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(req_id);
  if (it == sv->reqs.end()) {
    hg::set_error("unknown request id");
    return HG_ERR_INVALID_ARG;
  }
  *done = it->second->state == 2 ? 1 : 0;
  return HG_OK;
}

hg_status hg_server_wait(hg_server* sv, uint64_t req_id, double* latency_ms, double* queued_ms) {
  if (!sv) return HG_ERR_INVALID_ARG;
  std::shared_ptr<Request> r;
  {
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(req_id);
    if (it == sv->reqs.end()) {
      hg::set_error("unknown request id");
      return HG_ERR_INVALID_ARG;
    }
    r = it->second;
    sv->cv_done.wait(lk, [&] { return r->state == 2; });
    sv->reqs.erase(req_id);
  }
  using ms = std::chrono::duration<double, std::milli>;
  if (latency_ms) *latency_ms = ms(r->t_end - r->t_submit).count();
  if (queued_ms) *queued_ms = r->status == HG_ERR_CANCELLED ? 0.0 : ms(r->t_start - r->t_submit).count();
  if (r->status != HG_OK) hg::set_error(r->error);
  return r->status;
}

hg_status hg_server_cancel(hg_server* sv, uint64_t req_id) {
  if (!sv) return HG_ERR_INVALID_ARG;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(req_id);
    if (it == sv->reqs.end()) {
      hg::set_error("unknown request id");
      return HG_ERR_INVALID_ARG;
    }
    auto r = it->second;
    if (r->state != 0) {
      hg::set_error("request already started");
      return HG_ERR_BUSY;
    }
    for (auto q = sv->queue.begin(); q != sv->queue.end(); ++q)
      if ((*q)->id == req_id) {
        sv->queue.erase(q);
        break;
      }
    if (r->ready) {
      (void)hipEventDestroy(r->ready);
      r->ready = nullptr;
    }
    r->state = 2;
    r->status = HG_ERR_CANCELLED;
    r->error = "cancelled before it ran";
    r->t_start = r->t_end = Clock::now();
  }
  sv->cv_done.notify_all();
  sv->cv_work.notify_all();  // the new queue head may fit now
  return HG_OK;
}

hg_status hg_server_info(hg_server* sv, size_t* bytes_in_use, int32_t* queued, int32_t* running) {
  if (!sv) return HG_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  if (bytes_in_use) *bytes_in_use = sv->in_use;
  if (queued) *queued = (int32_t)sv->queue.size();
  if (running) *running = sv->running;
  return HG_OK;
}

hg_status hg_server_destroy(hg_server* sv) {
  if (!sv) return HG_OK;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stopping = true;
  }
  sv->cv_work.notify_all();
  for (auto& t : sv->workers) t.join();
  for (auto s : sv->streams) (void)hipStreamDestroy(s);
  delete sv;
  return HG_OK;
}

}  // extern "C"
