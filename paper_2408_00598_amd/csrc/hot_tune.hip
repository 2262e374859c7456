// Autotuner of the slab-pass launch shape (hot_autotune, hot_autotune_load).
//
// For a set of problem shapes, the built-in rule and every candidate of
// elements per slab-pass workgroup (2^11 .. 2^17) x row unroll (1, 2) x
// 16-byte vectors per lane (2, 4) are timed on a fixed number of iterations
// of uniform histograms: whole iterations (slab pass, reduce, solve) as the
// solver runs them, a batch's groups on their own streams, captured graphs,
// wall clock after the set-up.  The fastest is stored in the context for
// launches of that precision, size class and pair-count class, and optionally
// appended to a JSON-lines cache file keyed by device architecture.
#include <hip/hip_runtime.h>

#include <chrono>

#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/hot.h"
#include "hot_internal.h"
#include "hot_runtime.h"

using namespace hot;

static std::string arch_name(int dev) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  std::string a = p.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

extern "C" hot_status hot_autotune(hot_ctx* ctx, const hot_problem* probs, int32_t count,
                                   int32_t iters, const char* cache_path, double* out) {
  if (!ctx || !probs || count < 1 || iters < 1) return HOT_E_INVALID;
  if (hipSetDevice(ctx->device) != hipSuccess) return HOT_E_DEVICE;
  const int prec = probs[0].prec;
  // uniform histograms of every shape (values do not affect timing)
  std::vector<hot_problem> pr(probs, probs + count);
  std::vector<void*> bufs;
  int64_t total = 0;
  for (auto& p : pr) {
    if (p.m < 1 || p.n < 1 || p.m > kMaxSide || p.n > kMaxSide || p.prec != prec) {
      for (void* b : bufs) (void)hipFree(b);
      ctx->err = "autotune: bad shapes or mixed precision";
      return HOT_E_INVALID;
    }
    const int64_t M = (int64_t)p.m * p.n;
    total += (int64_t)p.m * p.m * p.n + (int64_t)p.m * p.n * p.n;
    std::vector<double> h((size_t)M, 1.0 / (double)M);
    void* d = nullptr;
    if (hipMalloc(&d, M * sizeof(double)) != hipSuccess ||
        hipMemcpy(d, h.data(), M * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipGetLastError();
      for (void* b : bufs) (void)hipFree(b);
      ctx->err = "autotune: allocation failed";
      return HOT_E_NOMEM;
    }
    bufs.push_back(d);
    p.mu1 = (const double*)d;
    p.mu2 = (const double*)d;
    p.tol = 1.0;
    p.max_iter = iters;
    p.check_every = 1 << 30;
    p.flags = HOT_FLAG_FIXED_ITERS;
    p.relax = 0.0;
    p.coord_row = nullptr;  // the uniform grid (the launch shape does not
    p.coord_col = nullptr;  // depend on the positions)
  }
  const int cls = size_class(total), pcls = size_class(count);
  const Tuning::Key key = tune_key(prec == HOT_FP32_STREAM, total, count);
  const Tuning saved = ctx->tune;
  double best = 1e300, dflt = 0.0;
  Tuning::Choice bestc{0, 1, 4};
  hot_status status = HOT_OK;
  std::vector<Tuning::Choice> cands;
  {  // the built-in rule, as an explicit choice (reference; may also win)
    Tuning t = saved;
    t.table.erase(key);
    const int fp32 = prec == HOT_FP32_STREAM;
    cands.push_back({t.item_elems_for(total, count, fp32), t.unroll_for(total, count, fp32),
                     t.vec_per_lane_for(total, count, fp32)});
  }
  for (int64_t e = 2048; e <= 131072; e *= 2)
    for (int u = 1; u <= 2; ++u)
      for (int v = 2; v <= 4; v += 2) cands.push_back({e, u, v});
  for (size_t c = 0; c < cands.size() && status == HOT_OK; ++c) {
    Tuning t = saved;
    t.table.erase(key);
    t.table[key] = cands[c];
    hot_ctx tmp;
    tmp.device = ctx->device;
    tmp.tune = t;
    tmp.tune.sep_anchor = 1;  // time the three-stream passes of the steady state
    tmp.profiling = false;
    // whole iterations (slab pass, reduce, solve) as the solver runs them:
    // the batch's groups on their streams, captured graphs, wall clock
    // around the run after the set-up has synchronised; the first run
    // captures the graphs
    GroupedBatch gb;
    double secs = 0.0;
    status = make_groups(&tmp, pr.data(), count, tmp.tune.batch_groups, gb);
    std::vector<std::vector<hot_problem>> sub(gb.wss.size());
    if (status == HOT_OK)
      for (int p = 0; p < count; ++p) sub[gb.where[p].first].push_back(pr[p]);
    for (int rep = 0; rep < 2 && status == HOT_OK; ++rep) {
      for (size_t g = 0; g < gb.wss.size() && status == HOT_OK; ++g)
        status = gb.wss[g]->setup(&tmp, sub[g].data(), (int)sub[g].size(), gb.wss[g]->stream);
      for (size_t g = 0; g < gb.wss.size() && status == HOT_OK; ++g)
        if (hipStreamSynchronize(gb.wss[g]->stream) != hipSuccess) status = HOT_E_DEVICE;
      const auto t0 = std::chrono::steady_clock::now();
      if (status == HOT_OK)
        status = run_concurrent(&tmp, gb.wss, (int64_t)iters * 2 / kGraphIters + 8);
      secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() /
             (double)iters;
    }
    if (status != HOT_OK) {
      ctx->err = "autotune: " + (tmp.err.empty() ? std::string("device error") : tmp.err);
      break;
    }
    if (c == 0) dflt = secs;
    if (secs < best) {
      best = secs;
      bestc = cands[c];
    }
  }
  for (void* b : bufs) (void)hipFree(b);
  if (status != HOT_OK) return status;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->tune.table[key] = bestc;
    ws_cache_clear(ctx);  // (layouts follow the tuning)
  }
  if (cache_path && cache_path[0]) {
    FILE* f = std::fopen(cache_path, "a");
    if (f) {
      std::fprintf(f,
                   "{\"arch\": \"%s\", \"fp32\": %d, \"size_class\": %d, \"pairs_class\": %d, "
                   "\"item_elems\": %lld, \"unroll\": %d, \"vec_per_lane\": %d, "
                   "\"us_per_iter\": %.3f, \"default_us_per_iter\": %.3f}\n",
                   arch_name(ctx->device).c_str(), std::get<0>(key), cls, pcls,
                   (long long)bestc.item_elems,
                   bestc.unroll, bestc.vec_per_lane, best * 1e6, dflt * 1e6);
      std::fclose(f);
    }
  }
  if (out) {
    out[0] = (double)bestc.item_elems;
    out[1] = (double)bestc.unroll;
    out[2] = best;
    out[3] = dflt;
    out[4] = (double)bestc.vec_per_lane;
  }
  return HOT_OK;
}

extern "C" hot_status hot_autotune_load(hot_ctx* ctx, const char* cache_path) {
  if (!ctx || !cache_path) return HOT_E_INVALID;
  FILE* f = std::fopen(cache_path, "r");
  if (!f) return HOT_E_INVALID;
  const std::string arch = arch_name(ctx->device);
  char line[512];
  int loaded = 0;
  while (std::fgets(line, sizeof(line), f)) {
    char a[64] = {0};
    int fp32 = 0, cls = 0, pcls = 0, u = 1, v = 4;
    long long e = 0;
    if (std::sscanf(line,
                    "{\"arch\": \"%63[^\"]\", \"fp32\": %d, \"size_class\": %d, \"pairs_class\": "
                    "%d, \"item_elems\": %lld, \"unroll\": %d, \"vec_per_lane\": %d",
                    a, &fp32, &cls, &pcls, &e, &u, &v) == 7 &&
        arch == a && e >= 1024 && (u == 1 || u == 2) && (v == 2 || v == 4)) {
      std::lock_guard<std::mutex> lk(ctx->mu);
      ctx->tune.table[Tuning::Key{fp32, cls, pcls}] = Tuning::Choice{(int64_t)e, u, v};  // later lines win
      ++loaded;
    }
  }
  std::fclose(f);
  if (loaded > 0) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ws_cache_clear(ctx);  // (layouts follow the tuning)
  }
  return loaded > 0 ? HOT_OK : HOT_E_INVALID;
}
