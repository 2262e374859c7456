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
//
// With HOT_SERVER_SHARED, problems of one precision, side class and sigma
// rule share launches instead: the class has a group of slots at fixed bases
// in one workspace; a problem is set up in a free slot at the group's next
// quantum boundary, the work tables of the occupied slots are installed and
// the graph re-captured, and every quantum iterates all of them at once.  A
// slot holds the problem's own single-problem geometry (place_in_slot), so
// its kernels and reduction order, hence its result, are those of a solve
// alone.
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

// side classes of the shared groups (the larger side of a problem, at most)
constexpr int kClassSides[] = {32, 48, 64, 96, 128, 192, 256};

struct GroupSlot {
  bool used = false;
  Request req;
  int64_t quanta = 0, max_quanta = 0;
  std::vector<SlabItem> items;
  std::vector<PBlock> blocks, sblocks;
};

struct Group {
  int prec = 0, side = 0, su = 0;
  std::shared_ptr<Workspace> ws;
  std::vector<GroupSlot> slots;
  std::deque<Request> pending;  // admitted, set up at the next quantum boundary
  bool in_flight = false;
  bool dirty = false;  // occupancy changed: new work tables before the next quantum
  size_t bytes = 0;
  int used() const {
    int u = 0;
    for (const GroupSlot& g : slots) u += g.used ? 1 : 0;
    return u;
  }
};

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
  // shared launches (HOT_SERVER_SHARED); groups are owned by the worker
  bool shared = false;
  size_t group_bytes = 0;  // device bytes of the groups (guarded by mu)
  int max_shared = 0;      // most problems one shared launch iterated
};

static size_t footprint_of(const hot_problem& p, const Tuning& tune) {
  Layout lay;
  std::string err;
  if (!build_layout({{p.m, p.n}}, p.prec == HOT_FP32_STREAM, tune, lay, err)) return 0;
  return lay.bytes(p.flags);
}

// The side class of a shared group a problem joins; false if it runs alone.
static bool group_class(const hot_server* S, const hot_problem& p, int& side, int& su) {
  if (!S->shared || (p.flags & HOT_FLAG_ESCALATE)) return false;
  const int big = std::max(p.m, p.n);
  side = 0;
  for (int c : kClassSides)
    if (big <= c) {
      side = c;
      break;
    }
  su = ((p.flags & HOT_FLAG_SIGMA_UPDATE) && (p.flags & HOT_FLAG_RESTART) &&
        !(p.flags & (HOT_FLAG_FIXED_ITERS | HOT_FLAG_ADMM)))
           ? 1
           : 0;
  return side > 0;
}

// Slot capacities of a class: the single-problem layout of its largest shape.
static bool class_caps(const Tuning& tune, int prec, int side, SlotCaps& caps) {
  Layout cap;
  std::string err;
  if (!build_layout({{side, side}}, prec == HOT_FP32_STREAM, tune, cap, err)) return false;
  caps = slot_caps(cap);
  return true;
}

static size_t group_bytes_of(const SlotCaps& caps, int K, int prec, int su) {
  Layout lay;
  group_layout(caps, K, prec == HOT_FP32_STREAM, lay);
  return lay.bytes(su ? HOT_FLAG_SIGMA_UPDATE : 0);
}

static hot_status make_group(hot_ctx* tmp, int prec, int side, int su, int K, const SlotCaps& caps,
                             std::unique_ptr<Group>& out) {
  auto ws = std::make_shared<Workspace>();
  ws->caps = caps;
  group_layout(caps, K, prec == HOT_FP32_STREAM, ws->lay);
  ws->group = true;
  ws->device = tmp->device;
  hot_status s = ws->alloc_all(tmp);
  if (s != HOT_OK) return s;
  const int64_t elems = 2 * (int64_t)side * side * side;  // the class shape's launch
  ws->args.unroll = tmp->tune.unroll_for(elems, 1, prec == HOT_FP32_STREAM);
  ws->args.nt_store = tmp->tune.nt_store;
  ws->args.fuse = tmp->tune.fuse;
  ws->args.solve_pre = tmp->tune.solve_pre;
  ws->args.fuse_pair = tmp->tune.fuse_pair;
  ws->args.bytes_ctr = nullptr;
  if (hipStreamCreateWithFlags(&ws->stream, hipStreamNonBlocking) != hipSuccess)
    return HOT_E_DEVICE;
  ws->own_stream = true;
  s = ws->init_group(tmp, ws->stream);
  if (s != HOT_OK) return s;
  auto g = std::make_unique<Group>();
  g->prec = prec;
  g->side = side;
  g->su = su;
  g->ws = ws;
  g->slots.resize(K);
  out = std::move(g);
  return HOT_OK;
}

static void server_loop(hot_server* S) {
  (void)hipSetDevice(S->ctx->device);
  std::vector<Slot> slots;
  std::vector<std::unique_ptr<Group>> groups;
  auto group_residents = [&]() {
    int r = 0;
    for (const auto& g : groups) r += g->used() + (int)g->pending.size();
    return r;
  };
  hot_ctx tmp;  // error sink of the worker
  tmp.device = S->ctx->device;
  tmp.tune = S->ctx->tune;
  auto finish = [&](const Request& req, const hot_result& res) {  // (takes the lock)
    Done d;
    d.res = res;
    d.tag = req.tag;
    d.latency = now_s() - req.t_submit;
    std::lock_guard<std::mutex> lk(S->mu);
    S->done.push_back(d);
    S->latencies.push_back(d.latency);
    ++S->completed;
    S->cv.notify_all();
  };
  for (;;) {
    bool progressed = false;
    // ---- admission ----------------------------------------------------
    for (;;) {
      {  // shared launches: the head joins its class's group when it has room
        std::vector<std::shared_ptr<Workspace>> freed;  // released after the lock
        std::unique_lock<std::mutex> lk(S->mu);
        if (S->queue.empty()) break;
        const Request head = S->queue.front();
        int side = 0, su = 0;
        Layout one;
        std::string err;
        Group* G = nullptr;
        bool route = group_class(S, head.prob, side, su) &&
                     build_layout({{head.prob.m, head.prob.n}}, head.prob.prec == HOT_FP32_STREAM,
                                  tmp.tune, one, err);
        if (route) {
          for (auto& g : groups)
            if (g->prec == head.prob.prec && g->side == side && g->su == su) G = g.get();
          if (!G) {
            SlotCaps caps;
            const int K = std::min(S->max_slots, 32);
            if (class_caps(tmp.tune, head.prob.prec, side, caps) && slot_fits(one, caps)) {
              const size_t gb = group_bytes_of(caps, K, head.prob.prec, su);
              while (S->in_use + S->pool_bytes + S->group_bytes + gb > S->budget &&
                     !S->pool.empty()) {
                auto victim = S->pool.begin();
                S->pool_bytes -= victim->second.second;
                --S->pool_count;
                freed.push_back(victim->second.first);
                S->pool.erase(victim);
              }
              std::unique_ptr<Group> ng;
              if (S->in_use + S->pool_bytes + S->group_bytes + gb <= S->budget &&
                  make_group(&tmp, head.prob.prec, side, su, K, caps, ng) == HOT_OK) {
                ng->bytes = gb;
                S->group_bytes += gb;
                groups.push_back(std::move(ng));
                G = groups.back().get();
              }
            }
          }
          route = G && slot_fits(one, G->ws->caps);
        }
        if (route) {
          if ((int)slots.size() + group_residents() >= S->max_slots) break;
          if (G->used() + (int)G->pending.size() >= (int)G->slots.size()) break;
          G->pending.push_back(head);
          S->queue.pop_front();
          S->active = (int)slots.size() + group_residents();
          S->max_active = std::max(S->max_active, S->active);
          progressed = true;
          continue;
        }
      }
      Request req;
      size_t bytes = 0;
      std::shared_ptr<Workspace> ws;
      std::vector<std::shared_ptr<Workspace>> evicted;  // freed outside the lock
      {
        std::unique_lock<std::mutex> lk(S->mu);
        if (S->queue.empty() || (int)slots.size() + group_residents() >= S->max_slots) break;
        const Request& head = S->queue.front();
        bytes = footprint_of(head.prob, tmp.tune);
        // a pooled workspace of this shape is reused; pooled memory counts
        // against the budget, so others are freed when it would not fit
        const ShapeKey key{head.prob.m, head.prob.n, head.prob.prec};
        auto hit = S->pool.find(key);
        const size_t reuse = hit != S->pool.end() ? hit->second.second : 0;
        while (S->in_use + S->pool_bytes + S->group_bytes - reuse + bytes > S->budget) {
          auto victim = S->pool.begin();
          while (victim != S->pool.end() && victim == hit) ++victim;
          if (victim == S->pool.end()) break;
          S->pool_bytes -= victim->second.second;
          --S->pool_count;
          evicted.push_back(victim->second.first);
          S->pool.erase(victim);
        }
        if ((!slots.empty() || group_residents() > 0) &&
            S->in_use + S->pool_bytes + S->group_bytes - reuse + bytes > S->budget)
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
        S->active = (int)slots.size() + 1 + group_residents();
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
        S->active = (int)slots.size() + group_residents();
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
        S->active = (int)slots.size() - 1 + group_residents();
        S->cv.notify_all();
      }
      slots.erase(slots.begin() + q);
    }
    // ---- shared groups: one quantum for all of a group's problems --------
    bool groups_busy = false;
    for (auto& gp : groups) {
      Group& G = *gp;
      Workspace& W = *G.ws;
      const int K = (int)G.slots.size();
      if (G.in_flight) {
        const hipError_t e = hipEventQuery(W.quantum_event);
        if (e == hipErrorNotReady) {
          groups_busy = true;
          continue;
        }
        G.in_flight = false;
        progressed = true;
        std::vector<int> leave;
        for (int s = 0; s < K; ++s) {
          const GroupSlot& gs = G.slots[s];
          if (!gs.used) continue;
          const bool running = e == hipSuccess && W.host_ctl[s].status == ST_RUNNING;
          const bool cancel = S->stop.load() || gs.req.gen < S->cancel_gen.load();
          if (!running || cancel || gs.quanta >= gs.max_quanta) leave.push_back(s);
        }
        if (!leave.empty()) {
          // the final control blocks (the finalize pass's metrics; it covers
          // every occupied slot and leaves the running ones' iterates alone)
          if (e == hipSuccess && W.finalize(W.stream) == hipSuccess)
            (void)hipMemcpyAsync(W.host_ctl, W.ctl_d, K * sizeof(PairCtl), hipMemcpyDeviceToHost,
                                 W.stream);
          (void)hipStreamSynchronize(W.stream);
          for (int s : leave) {
            GroupSlot& gs = G.slots[s];
            hot_result r;
            W.fill_result(s, &r, now_s() - gs.req.t_submit);
            if (e != hipSuccess) r.status = HOT_E_DEVICE;
            else if (W.host_ctl[s].status == ST_RUNNING) r.status = HOT_E_CANCELLED;
            finish(gs.req, r);
            gs.used = false;
            gs.items.clear();
            gs.blocks.clear();
            gs.sblocks.clear();
          }
          G.dirty = true;
        }
      }
      // set up the admitted problems in free slots, then launch
      while (!G.pending.empty()) {
        int s = 0;
        while (s < K && G.slots[s].used) ++s;
        if (s == K) break;
        const Request req = G.pending.front();
        G.pending.pop_front();
        progressed = true;
        if (S->stop.load() || req.gen < S->cancel_gen.load()) {
          hot_result r;
          std::memset(&r, 0, sizeof(r));
          r.status = HOT_E_CANCELLED;
          finish(req, r);
          continue;
        }
        Layout one;
        std::string err;
        GroupSlot& gs = G.slots[s];
        PairGeo g;
        hot_status st = build_layout({{req.prob.m, req.prob.n}}, req.prob.prec == HOT_FP32_STREAM,
                                     tmp.tune, one, err)
                            ? HOT_OK
                            : HOT_E_INVALID;
        if (st == HOT_OK) {
          place_in_slot(one, s, W.caps, g, gs.items, gs.blocks, gs.sblocks);
          st = W.setup_slot(&tmp, s, req.prob, g, W.stream);
        }
        if (st != HOT_OK) {
          hot_result r;
          std::memset(&r, 0, sizeof(r));
          r.status = (int32_t)st;
          finish(req, r);
          continue;
        }
        gs.used = true;
        gs.req = req;
        gs.quanta = 0;
        gs.max_quanta = (int64_t)req.prob.max_iter * 2 / kGraphIters + 8;
        G.dirty = true;
      }
      const int u = G.used();
      if (G.dirty && u > 0) {
        std::vector<SlabItem> items;
        std::vector<PBlock> blocks, sblocks;
        int coord = 0;
        for (const GroupSlot& gs : G.slots) {
          if (!gs.used) continue;
          items.insert(items.end(), gs.items.begin(), gs.items.end());
          blocks.insert(blocks.end(), gs.blocks.begin(), gs.blocks.end());
          sblocks.insert(sblocks.end(), gs.sblocks.begin(), gs.sblocks.end());
          if (gs.req.prob.coord_row || gs.req.prob.coord_col) coord = 1;
        }
        const hot_status ts = W.set_tables(&tmp, items, blocks, sblocks, coord, G.su, W.stream);
        G.dirty = false;
        if (ts != HOT_OK) {  // (capacities are checked at admission: not expected)
          for (GroupSlot& gs : G.slots) {
            if (!gs.used) continue;
            hot_result r;
            std::memset(&r, 0, sizeof(r));
            r.status = ts;
            finish(gs.req, r);
            gs.used = false;
          }
          continue;
        }
      }
      if (u > 0) {
        const bool ok = W.ensure_graph(&tmp, W.stream) == HOT_OK &&
                        W.launch_quantum(W.stream) == hipSuccess;
        if (ok) {
          G.in_flight = true;
          groups_busy = true;
          for (GroupSlot& gs : G.slots)
            if (gs.used) ++gs.quanta;
          std::lock_guard<std::mutex> lk(S->mu);
          S->max_shared = std::max(S->max_shared, u);
        } else {
          for (GroupSlot& gs : G.slots) {
            if (!gs.used) continue;
            hot_result r;
            std::memset(&r, 0, sizeof(r));
            r.status = HOT_E_DEVICE;
            finish(gs.req, r);
            gs.used = false;
          }
        }
        progressed = true;
      }
      std::lock_guard<std::mutex> lk(S->mu);
      S->active = (int)slots.size() + group_residents();
    }
    if (!progressed) {
      std::unique_lock<std::mutex> lk(S->mu);
      if (S->stop && S->queue.empty() && slots.empty() && group_residents() == 0) break;
      if (slots.empty() && !groups_busy) {
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
  S->shared = (cfg->flags & HOT_SERVER_SHARED) != 0;
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
  out[4] = (double)(S->in_use + S->group_bytes);
  out[5] = (double)S->max_active;
  out[6] = pct(0.50);
  out[7] = pct(0.99);
  out[8] = (double)S->max_shared;
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
