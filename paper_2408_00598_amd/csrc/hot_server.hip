// Continuous-batching solve service (hot_server_*, see include/hot.h).
//
// Requests wait in a FIFO queue.  A worker thread admits the head of the
// queue whenever a slot is free and the problem's device footprint fits in
// the HBM budget, sets it up on its own stream and keeps relaunching its
// captured iteration graph (one quantum = kGraphIters iterations of
// Algorithm 2) until the problem stops.  Problems admitted at different times
// run concurrently on their own streams, so their kernels overlap on the
// device; each one runs exactly the kernels and reduction order of hot_solve,
// so its result is the same as when solved alone.  Iterates stay on the
// device between quanta and across restarts.  Workspaces are pooled by
// shape and precision and reused (graph included).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/hot.h"
#include "hot_internal.h"
#include "hot_runtime.h"

using namespace hot;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Request {
  hot_problem prob;
  uint64_t tag;
  double t_submit;
  uint64_t gen;  // cancellation generation at submission
};

struct Slot {
  std::shared_ptr<Workspace> ws;
  Request req;
  size_t bytes;
  int64_t quanta;
  int64_t max_quanta;
  bool esc;          // HOT_FLAG_ESCALATE on an FP32-stream problem
  bool esc_next;     // stalled at the last quantum: widen after this one
  hot_status esc_err;  // a failed widening ends the request with this status
  StallWatch watch;
};

struct Done {
  hot_result res;
  uint64_t tag;
  double latency;
};

typedef std::tuple<int, int, int> ShapeKey;

}  // namespace

struct hot_server {
  hot_ctx* ctx = nullptr;
  size_t budget = 0;
  int max_slots = 1;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request> queue;
  std::vector<Done> done;
  std::vector<double> latencies;
  std::multimap<ShapeKey, std::pair<std::shared_ptr<Workspace>, size_t>> pool;
  size_t pool_count = 0;
  size_t pool_bytes = 0;  // device bytes held by pooled workspaces
  std::thread th;
  std::atomic<bool> stop{false};
  std::atomic<uint64_t> cancel_gen{0};  // requests of earlier generations are cancelled
  // counters (guarded by mu)
  int64_t submitted = 0, completed = 0;
  int active = 0, max_active = 0;
  size_t in_use = 0;
};

static size_t footprint_of(const hot_problem& p, const Tuning& tune) {
  Layout lay;
  std::string err;
  if (!build_layout({{p.m, p.n}}, p.prec == HOT_FP32_STREAM, tune, lay, err)) return 0;
  return lay.bytes(p.flags);
}

static void server_loop(hot_server* S) {
  (void)hipSetDevice(S->ctx->device);
  std::vector<Slot> slots;
  hot_ctx tmp;  // error sink of the worker
  tmp.device = S->ctx->device;
  tmp.tune = S->ctx->tune;
  for (;;) {
    bool progressed = false;
    // ---- admission ----------------------------------------------------
    for (;;) {
      Request req;
      size_t bytes = 0;
      std::shared_ptr<Workspace> ws;
      std::vector<std::shared_ptr<Workspace>> evicted;  // freed outside the lock
      {
        std::unique_lock<std::mutex> lk(S->mu);
        if (S->queue.empty() || (int)slots.size() >= S->max_slots) break;
        const Request& head = S->queue.front();
        bytes = footprint_of(head.prob, tmp.tune);
        // a pooled workspace of this shape is reused; pooled memory counts
        // against the budget, so others are freed when it would not fit
        const ShapeKey key{head.prob.m, head.prob.n, head.prob.prec};
        auto hit = S->pool.find(key);
        const size_t reuse = hit != S->pool.end() ? hit->second.second : 0;
        while (S->in_use + S->pool_bytes - reuse + bytes > S->budget) {
          auto victim = S->pool.begin();
          while (victim != S->pool.end() && victim == hit) ++victim;
          if (victim == S->pool.end()) break;
          S->pool_bytes -= victim->second.second;
          --S->pool_count;
          evicted.push_back(victim->second.first);
          S->pool.erase(victim);
        }
        if (!slots.empty() && S->in_use + S->pool_bytes - reuse + bytes > S->budget)
          break;  // wait for memory
        if (hit != S->pool.end()) {
          ws = hit->second.first;
          S->pool_bytes -= hit->second.second;
          --S->pool_count;
          S->pool.erase(hit);
        }
        req = S->queue.front();
        S->queue.pop_front();
        S->in_use += bytes;
        S->active = (int)slots.size() + 1;
        S->max_active = std::max(S->max_active, S->active);
      }
      evicted.clear();
      progressed = true;
      hot_status st = HOT_OK;
      if (!ws) st = make_workspace(&tmp, &req.prob, 1, ws);
      if (st == HOT_OK) st = ws->setup(&tmp, &req.prob, 1, ws->stream);
      if (st == HOT_OK) st = ws->ensure_graph(&tmp, ws->stream);
      if (st == HOT_OK && ws->launch_quantum(ws->stream) != hipSuccess) st = HOT_E_DEVICE;
      if (st != HOT_OK) {
        Done d;
        std::memset(&d.res, 0, sizeof(d.res));
        d.res.status = (int32_t)st;
        d.tag = req.tag;
        d.latency = now_s() - req.t_submit;
        std::lock_guard<std::mutex> lk(S->mu);
        S->in_use -= bytes;
        S->active = (int)slots.size();
        S->done.push_back(d);
        S->latencies.push_back(d.latency);
        ++S->completed;
        S->cv.notify_all();
        continue;
      }
      Slot sl;
      sl.ws = ws;
      sl.req = req;
      sl.bytes = bytes;
      sl.quanta = 1;
      sl.max_quanta = (int64_t)req.prob.max_iter * 2 / kGraphIters + 8;
      sl.esc = (req.prob.flags & HOT_FLAG_ESCALATE) && req.prob.prec == HOT_FP32_STREAM &&
               !(req.prob.flags & HOT_FLAG_FIXED_ITERS);
      sl.esc_next = false;
      sl.esc_err = HOT_OK;
      slots.push_back(sl);
    }
    // ---- progress of resident problems ---------------------------------
    for (size_t q = 0; q < slots.size();) {
      Slot& sl = slots[q];
      const hipError_t e = hipEventQuery(sl.ws->quantum_event);
      if (e == hipErrorNotReady) {
        ++q;
        continue;
      }
      progressed = true;
      const bool running = (e == hipSuccess) && sl.ws->host_ctl[0].status == ST_RUNNING;
      const bool cancel = S->stop.load() || sl.req.gen < S->cancel_gen.load();
      if (running && !cancel && sl.quanta < sl.max_quanta) {
        bool ok = true;
        if (sl.esc_next) {
          // stalled one quantum ago: widen the state to FP64 now and continue
          // with FP64 streams (hot_solve, which decides while its next graph
          // is in flight, widens at the same iteration)
          sl.esc_next = false;
          sl.esc_err = sl.ws->escalate(&tmp, sl.ws->stream);
          if (sl.esc_err == HOT_OK) sl.esc_err = sl.ws->ensure_graph(&tmp, sl.ws->stream);
          ok = sl.esc_err == HOT_OK;
          if (ok) sl.ws->escalated_at = sl.ws->host_ctl[0].it;
        } else if (sl.esc && sl.ws->lay.fp32 && sl.watch.stalled(sl.ws->host_ctl[0])) {
          sl.esc_next = true;
        }
        if (ok && sl.ws->launch_quantum(sl.ws->stream) == hipSuccess) {
          ++sl.quanta;
          ++q;
          continue;
        }
      }
      // finished (or failed): the final control block (with the finalize
      // pass's metrics) once the stream is idle
      if (e == hipSuccess && sl.ws->finalize(sl.ws->stream) == hipSuccess)
        (void)hipMemcpyAsync(sl.ws->host_ctl, sl.ws->ctl_d, sizeof(PairCtl),
                             hipMemcpyDeviceToHost, sl.ws->stream);
      (void)hipStreamSynchronize(sl.ws->stream);
      Done d;
      const double t = now_s();
      sl.ws->fill_result(0, &d.res, t - sl.req.t_submit);
      if (e != hipSuccess) d.res.status = HOT_E_DEVICE;
      else if (sl.esc_err != HOT_OK) d.res.status = sl.esc_err;
      else if (running) d.res.status = HOT_E_CANCELLED;
      d.tag = sl.req.tag;
      d.latency = t - sl.req.t_submit;
      {
        std::lock_guard<std::mutex> lk(S->mu);
        S->done.push_back(d);
        S->latencies.push_back(d.latency);
        ++S->completed;
        S->in_use -= sl.bytes;
        // (a workspace widened to FP64 no longer matches its FP32 key)
        const bool same_prec = sl.ws->lay.fp32 == (sl.req.prob.prec == HOT_FP32_STREAM ? 1 : 0);
        if (S->pool_count < (size_t)(2 * S->max_slots) && e == hipSuccess && same_prec) {
          S->pool.emplace(ShapeKey{sl.req.prob.m, sl.req.prob.n, sl.req.prob.prec},
                          std::make_pair(sl.ws, sl.bytes));
          ++S->pool_count;
          S->pool_bytes += sl.bytes;
        }
        S->active = (int)slots.size() - 1;
        S->cv.notify_all();
      }
      slots.erase(slots.begin() + q);
    }
    if (!progressed) {
      std::unique_lock<std::mutex> lk(S->mu);
      if (S->stop && S->queue.empty() && slots.empty()) break;
      if (slots.empty()) {
        S->cv.wait_for(lk, std::chrono::milliseconds(2));
      } else {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
      }
    }
  }
}

extern "C" {

hot_status hot_server_create(hot_ctx* ctx, const hot_server_config* cfg, hot_server** out) {
  if (!ctx || !cfg || !out) return HOT_E_INVALID;
  *out = nullptr;
  if (cfg->max_slots < 1 || cfg->max_slots > 1024) {
    ctx->err = "max_slots must be in [1, 1024]";
    return HOT_E_INVALID;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return HOT_E_DEVICE;
  size_t budget = cfg->hbm_budget_bytes;
  if (budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return HOT_E_DEVICE;
    budget = fr / 10 * 8;
  }
  hot_server* S = new hot_server();
  S->ctx = ctx;
  S->budget = budget;
  S->max_slots = cfg->max_slots;
  S->th = std::thread(server_loop, S);
  *out = S;
  return HOT_OK;
}

hot_status hot_server_submit(hot_server* S, const hot_problem* prob, uint64_t tag) {
  if (!S || !prob) return HOT_E_INVALID;
  if (prob->m < 1 || prob->n < 1 || prob->m > kMaxSide || prob->n > kMaxSide || !prob->mu1 ||
      !prob->mu2 || prob->max_iter < 1 || prob->check_every < 1 ||
      (prob->prec != HOT_FP64 && prob->prec != HOT_FP32_STREAM))
    return HOT_E_INVALID;
  if (!(prob->flags & HOT_FLAG_FIXED_ITERS) && !(prob->tol > 0)) return HOT_E_INVALID;
  if ((prob->flags & HOT_FLAG_ADMM) && !(prob->relax <= 0.0 || prob->relax < 2.0))
    return HOT_E_INVALID;
  if (footprint_of(*prob, S->ctx->tune) > S->budget) return HOT_E_NOMEM;
  Request r;
  r.prob = *prob;
  r.tag = tag;
  r.t_submit = now_s();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    r.gen = S->cancel_gen.load();
    S->queue.push_back(r);
    ++S->submitted;
  }
  S->cv.notify_all();
  return HOT_OK;
}

int32_t hot_server_poll(hot_server* S, hot_result* results, uint64_t* tags, double* latency_s,
                        int32_t max) {
  if (!S || max < 1) return 0;
  std::lock_guard<std::mutex> lk(S->mu);
  const int32_t k = (int32_t)std::min<size_t>(S->done.size(), (size_t)max);
  for (int32_t q = 0; q < k; ++q) {
    if (results) results[q] = S->done[q].res;
    if (tags) tags[q] = S->done[q].tag;
    if (latency_s) latency_s[q] = S->done[q].latency;
  }
  S->done.erase(S->done.begin(), S->done.begin() + k);
  return k;
}

hot_status hot_server_drain(hot_server* S, double timeout_s) {
  if (!S) return HOT_E_INVALID;
  std::unique_lock<std::mutex> lk(S->mu);
  const auto until = std::chrono::steady_clock::now() +
                     std::chrono::microseconds((int64_t)(std::max(0.0, timeout_s) * 1e6));
  while (S->completed < S->submitted) {
    if (S->cv.wait_until(lk, until) == std::cv_status::timeout && S->completed < S->submitted)
      return HOT_E_BUSY;
  }
  return HOT_OK;
}

hot_status hot_server_stats(hot_server* S, double* out) {
  if (!S || !out) return HOT_E_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  std::vector<double> lat = S->latencies;
  std::sort(lat.begin(), lat.end());
  auto pct = [&](double p) -> double {
    if (lat.empty()) return 0.0;
    const size_t idx = std::min(lat.size() - 1, (size_t)(p * (double)(lat.size() - 1) + 0.5));
    return lat[idx];
  };
  out[0] = (double)S->completed;
  out[1] = (double)S->submitted;
  out[2] = (double)S->queue.size();
  out[3] = (double)S->active;
  out[4] = (double)S->in_use;
  out[5] = (double)S->max_active;
  out[6] = pct(0.50);
  out[7] = pct(0.99);
  return HOT_OK;
}

hot_status hot_server_cancel(hot_server* S) {
  if (!S) return HOT_E_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  // resident problems submitted so far stop after their current quantum
  S->cancel_gen.fetch_add(1);
  const double t = now_s();
  for (const Request& r : S->queue) {  // queued ones finish now
    Done d;
    std::memset(&d.res, 0, sizeof(d.res));
    d.res.status = HOT_E_CANCELLED;
    d.tag = r.tag;
    d.latency = t - r.t_submit;
    S->done.push_back(d);
    S->latencies.push_back(d.latency);
    ++S->completed;
  }
  S->queue.clear();
  S->cv.notify_all();
  return HOT_OK;
}

void hot_server_destroy(hot_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->queue.clear();  // requests not yet admitted are dropped
  }
  S->stop = true;  // resident problems stop after their current quantum
  S->cv.notify_all();
  if (S->th.joinable()) S->th.join();
  delete S;
}

}  // extern "C"
