// Host runtime and C ABI of libhot (see include/hot.h).
//
// A "Batch" holds one or more problems laid out back to back in shared
// device buffers (flow state, sums, dual vectors, control blocks).  Every
// iteration is one slab pass + one pair reduce + one pair solve over all
// problems of the batch; the loop body is captured once into a HIP graph of
// kGraphIters iterations and relaunched until every problem has stopped.
// The stop / restart decisions are taken on the device, so the host only
// polls a status word per problem between graph launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/hot.h"
#include "hot_internal.h"
#include "hot_runtime.h"

namespace hot {

void launch_iteration(const LaunchArgs& a, int par, hipStream_t st);
void launch_slab_pass(const LaunchArgs& a, int par, hipStream_t st);
void launch_pair_kernels(const LaunchArgs& a, int par, hipStream_t st);
void launch_setup_mu(const double* mu1, const double* mu2, int m, int n, double* mu1T,
                     double* mu2c, hipStream_t st);
void launch_export(const LaunchArgs& a, int par, int pair, int64_t N, double* xbar,
                   double* zbar, double* sout, hipStream_t st, double* s0out = nullptr);
void launch_export_y(const LaunchArgs& a, int pair, int64_t M3, double* y, hipStream_t st);
void launch_aat_solve(const LaunchArgs& a, int pair, int64_t M, const double* R,
                      hipStream_t st);
void launch_hist_stats_multi(const double* const* ptrs, const int64_t* lens, int count,
                             double* out, hipStream_t st);
void launch_zero(void* p, size_t bytes, hipStream_t st);
void launch_widen(const void* in, void* out, int64_t n, hipStream_t st);
void launch_finalize(const LaunchArgs& a, const SlabItem* items_all, int nitems_all, int npairs,
                     hipStream_t st);
void* static_scratch_init(int device, std::string& err);


}  // namespace hot

using namespace hot;

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------

namespace hot {
// Fold a finished workspace's counters into the context (caller holds ctx->mu).
static void collect_profile(hot_ctx* ctx, Workspace& ws) {
  unsigned long long bytes = 0;
  if (hipMemcpy(&bytes, ws.bytes_ctr, 8, hipMemcpyDeviceToHost) != hipSuccess) return;
  ctx->prof_bytes += (double)bytes;
  ctx->prof_seconds += ws.prof_seconds;
  ctx->prof_launches += (double)ws.prof_launches;
  ctx->iters_launched += (double)ws.iterations_launched;
}
}  // namespace hot

#define HIPCK(expr)                                                                  \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) {                                                          \
      if (ctx) ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);         \
      return HOT_E_DEVICE;                                                           \
    }                                                                                \
  } while (0)

namespace hot {

Workspace::~Workspace() { release(); }

void Workspace::drop_retired() {
  for (auto& g : retired) {
    if (g.second) (void)hipGraphExecDestroy(g.second);
    if (g.first) (void)hipGraphDestroy(g.first);
  }
  retired.clear();
}

void Workspace::release() {
  drop_retired();
  if (stage_ev) (void)hipEventDestroy(stage_ev);
  stage_ev = nullptr;
  stage_pending = false;
  if (stage_h) (void)hipHostFree(stage_h);
  stage_h = nullptr;
  if (quantum_event) (void)hipEventDestroy(quantum_event);
  quantum_event = nullptr;
  if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
  if (graph) (void)hipGraphDestroy(graph);
  graph_exec = nullptr;
  graph = nullptr;
  for (void* p : allocs) (void)hipFree(p);
  allocs.clear();
  if (host_ctl && host_ctl_vec.empty()) (void)hipHostFree(host_ctl);
  host_ctl = nullptr;
  host_ctl_vec.clear();
  if (own_stream && stream) (void)hipStreamDestroy(stream);
  stream = nullptr;
}

// One device buffer: hipMalloc, or the next 256-byte aligned piece of the
// arena.  Past the arena's end nothing is handed out (the pointer is null)
// but arena_used keeps counting, so the caller can report the size needed.
hot_status Workspace::device_buffer(hot_ctx* ctx, void** p, size_t bytes) {
  bytes = std::max<size_t>(bytes, 256);
  if (arena) {
    const size_t off = (arena_used + 255) / 256 * 256;
    arena_used = off + bytes;
    *p = arena_used <= arena_bytes ? (void*)(arena + off) : nullptr;
    return HOT_OK;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    if (ctx) ctx->err = std::string("hipMalloc failed: ") + hipGetErrorString(e);
    return HOT_E_NOMEM;
  }
  allocs.push_back(*p);
  return HOT_OK;
}

hot_status Workspace::alloc_all(hot_ctx* ctx) {
  auto A = [&](void** p, size_t bytes) -> hot_status { return device_buffer(ctx, p, bytes); };
  hot_status st;
  const size_t es = lay.elem_size;
  for (int b = 0; b < 3; ++b)
    if ((st = A(&sb[b], (size_t)lay.state_elems * es)) != HOT_OK) return st;
  if ((st = A((void**)&ab, lay.ab_len * 8)) != HOT_OK) return st;
  for (int q = 0; q < 2; ++q) {
    if ((st = A((void**)&rowsum[q], lay.rs_len * 8)) != HOT_OK) return st;
    if ((st = A((void**)&colpart[q], lay.cp_len * 8)) != HOT_OK) return st;
  }
  if ((st = A((void**)&kitem, lay.items.size() * kKI * 8)) != HOT_OK) return st;
  if ((st = A((void**)&arr, lay.arr_len * 8)) != HOT_OK) return st;
  if ((st = A((void**)&vec, lay.vec_len * 8)) != HOT_OK) return st;
  if ((st = A((void**)&items_d, lay.items.size() * sizeof(SlabItem))) != HOT_OK) return st;
  if ((st = A((void**)&sitems_d, std::max<size_t>(lay.sitems.size(), 1) * sizeof(SmallItem))) != HOT_OK)
    return st;
  const size_t n_it = std::max<size_t>(lay.items.size(), 1) * sizeof(SlabItem);
  const size_t n_si = std::max<size_t>(lay.sitems.size(), 1) * sizeof(SmallItem);
  const size_t n_bl = std::max<size_t>(lay.blocks.size(), 1) * sizeof(PBlock);
  const size_t n_sb = std::max<size_t>(lay.sblocks.size(), 1) * sizeof(PBlock);
  if (lay.geo.size() > 1 && !arena) {  // compacted launch tables (batches only)
    if ((st = A((void**)&items_c, n_it)) != HOT_OK) return st;
    if ((st = A((void**)&sitems_c, n_si)) != HOT_OK) return st;
    if ((st = A((void**)&blocks_c, n_bl)) != HOT_OK) return st;
    if ((st = A((void**)&sblocks_c, n_sb)) != HOT_OK) return st;
    if (hipHostMalloc(&stage_h, n_it + n_si + n_bl + n_sb) != hipSuccess) {
      stage_h = nullptr;
      if (ctx) ctx->err = "hipHostMalloc failed";
      return HOT_E_NOMEM;
    }
  }
  if ((st = A((void**)&blocks_d, lay.blocks.size() * sizeof(PBlock))) != HOT_OK) return st;
  if ((st = A((void**)&sblocks_d, lay.sblocks.size() * sizeof(PBlock))) != HOT_OK) return st;
  if ((st = A((void**)&geo_d, lay.geo.size() * sizeof(PairGeo))) != HOT_OK) return st;
  if ((st = A((void**)&ctl_d, lay.geo.size() * sizeof(PairCtl) * 2)) != HOT_OK) return st;
  if ((st = A((void**)&stats_d, lay.geo.size() * 2 * 8 * 8)) != HOT_OK) return st;
  if ((st = A((void**)&ptrs_d, lay.geo.size() * 2 * (sizeof(void*) + 8))) != HOT_OK) return st;
  if ((st = A((void**)&bytes_ctr, 256)) != HOT_OK) return st;
  if ((st = A((void**)&sync_d, lay.geo.size() * 5 * sizeof(unsigned))) != HOT_OK) return st;
  if (arena) {
    if (arena_used > arena_bytes) {
      if (ctx)
        ctx->err = "problem needs " + std::to_string(arena_used) +
                   " bytes of device scratch, more than the " + std::to_string(arena_bytes) +
                   " the no-alloc entry point holds";
      return HOT_E_INVALID;
    }
    host_ctl_vec.assign(lay.geo.size() * 2, PairCtl());
    host_ctl = host_ctl_vec.data();
  } else if (hipHostMalloc((void**)&host_ctl, lay.geo.size() * sizeof(PairCtl) * 2) !=
             hipSuccess) {
    host_ctl = nullptr;
    if (ctx) ctx->err = "hipHostMalloc failed";
    return HOT_E_NOMEM;
  }
  args.items = items_d;
  args.nitems = (int)lay.items.size();
  args.nbig = (int)lay.nbig;
  args.sitems = sitems_d;
  args.nsitems = (int)lay.sitems.size();
  args.blocks = blocks_d;
  args.nblocks = (int)lay.blocks.size();
  args.sblocks = sblocks_d;
  args.nsblocks = (int)lay.sblocks.size();
  args.geo = geo_d;
  args.ctl[0] = ctl_d;
  args.ctl[1] = ctl_d + lay.geo.size();
  for (int b = 0; b < 3; ++b) args.sb[b] = sb[b];
  args.ab = ab;
  args.rowsum[0] = rowsum[0];
  args.rowsum[1] = rowsum[1];
  args.colpart[0] = colpart[0];
  args.colpart[1] = colpart[1];
  args.kitem = kitem;
  args.arr = arr;
  args.vec = vec;
  args.fp32 = lay.fp32;
  args.maxvpl = lay.maxvpl;
  args.bytes_ctr = bytes_ctr;
  args.sync[0] = sync_d;
  args.sync[1] = sync_d + 2 * lay.geo.size();
  args.lost = sync_d + 4 * lay.geo.size();
  launch_pairs = (int)lay.geo.size();
  return HOT_OK;
}

}  // namespace hot

static hot_status validate_problem(hot_ctx* ctx, const hot_problem* p) {
  if (!p) {
    ctx->err = "null problem";
    return HOT_E_INVALID;
  }
  if (p->m < 1 || p->n < 1 || p->m > kMaxSide || p->n > kMaxSide) {
    ctx->err = "grid sides must be in [1, " + std::to_string(kMaxSide) + "]";
    return HOT_E_INVALID;
  }
  if (!p->mu1 || !p->mu2) {
    ctx->err = "null histogram pointer";
    return HOT_E_INVALID;
  }
  const bool fixed = (p->flags & HOT_FLAG_FIXED_ITERS) != 0;
  if (!fixed && !(p->tol > 0.0) ) {
    ctx->err = "tol must be > 0";
    return HOT_E_INVALID;
  }
  if (p->max_iter < 1 || p->check_every < 1) {
    ctx->err = "max_iter and check_every must be >= 1";
    return HOT_E_INVALID;
  }
  if (p->prec != HOT_FP64 && p->prec != HOT_FP32_STREAM) {
    ctx->err = "unknown precision";
    return HOT_E_INVALID;
  }
  if (!std::isfinite(p->sigma)) {
    ctx->err = "sigma must be finite";
    return HOT_E_INVALID;
  }
  if ((p->flags & HOT_FLAG_ADMM) && !(p->relax <= 0.0 || p->relax < 2.0)) {
    ctx->err = "relax must be in (0, 2)";
    return HOT_E_INVALID;
  }
  return HOT_OK;
}

namespace hot {

hot_status validate_problem_public(hot_ctx* ctx, const hot_problem* p) {
  return validate_problem(ctx, p);
}

// Validate histograms on the device, compute ||b|| and sigma, fill control
// blocks, copy tables and clear the state.  Synchronises `st` once.
hot_status Workspace::setup(hot_ctx* ctx, const hot_problem* probs, int count, hipStream_t st) {
  const size_t np = lay.geo.size();
  escalated_at = 0;
  prof_seconds = 0.0;  // (a cached workspace starts its counts afresh)
  prof_launches = 0;
  iterations_launched = 0;
  restore_tables();  // (no graph is in flight between runs)
  drop_retired();
  std::vector<const double*> ptrs(2 * np);
  std::vector<int64_t> lens(2 * np);
  for (size_t p = 0; p < np; ++p) {
    ptrs[2 * p] = probs[p].mu1;
    ptrs[2 * p + 1] = probs[p].mu2;
    lens[2 * p] = lens[2 * p + 1] = (int64_t)probs[p].m * probs[p].n;
  }
  (void)count;
  const double** pd = (const double**)ptrs_d;
  int64_t* ld = (int64_t*)((char*)ptrs_d + np * 2 * sizeof(void*));
  HIPCK(hipMemcpyAsync(pd, ptrs.data(), np * 2 * sizeof(void*), hipMemcpyHostToDevice, st));
  HIPCK(hipMemcpyAsync(ld, lens.data(), np * 2 * 8, hipMemcpyHostToDevice, st));
  launch_hist_stats_multi(pd, ld, (int)(2 * np), stats_d, st);
  HIPCK(hipGetLastError());
  std::vector<double> stats(np * 2 * 8);
  HIPCK(hipMemcpyAsync(stats.data(), stats_d, stats.size() * 8, hipMemcpyDeviceToHost, st));
  // grid-line positions of problems with non-uniform bins (m + n per pair)
  std::vector<int64_t> pos_at(np, -1);
  int64_t npos = 0;
  for (size_t p = 0; p < np; ++p)
    if (probs[p].coord_row || probs[p].coord_col) {
      pos_at[p] = npos;
      npos += (int64_t)probs[p].m + probs[p].n;
    }
  std::vector<double> pos((size_t)std::max<int64_t>(npos, 1));
  for (size_t p = 0; p < np; ++p) {
    if (pos_at[p] < 0) continue;
    if (probs[p].coord_row)
      HIPCK(hipMemcpyAsync(&pos[pos_at[p]], probs[p].coord_row, (size_t)probs[p].m * 8,
                           hipMemcpyDeviceToHost, st));
    if (probs[p].coord_col)
      HIPCK(hipMemcpyAsync(&pos[pos_at[p] + probs[p].m], probs[p].coord_col,
                           (size_t)probs[p].n * 8, hipMemcpyDeviceToHost, st));
  }
  HIPCK(hipStreamSynchronize(st));
  for (size_t p = 0; p < np; ++p) {
    const double* s1 = &stats[(2 * p) * 8];
    const double* s2 = &stats[(2 * p + 1) * 8];
    // s[0] min, s[1] sum, s[2] non-finite count, s[3] sum of squares, s[4] last entry
    if (s1[2] > 0 || s2[2] > 0) {
      ctx->err = "histogram has non-finite entries (problem " + std::to_string(p) + ")";
      return HOT_E_INVALID;
    }
    if (s1[0] < 0 || s2[0] < 0) {
      ctx->err = "histogram has negative entries (problem " + std::to_string(p) + ")";
      return HOT_E_INVALID;
    }
    const double tot = std::max(s1[1], s2[1]);
    if (!(tot > 0) || std::fabs(s1[1] - s2[1]) > 1e-9 * tot) {
      ctx->err = "histogram totals differ or are zero (problem " + std::to_string(p) + ")";
      return HOT_E_INVALID;
    }
    PairGeo& g = lay.geo[p];
    g.norm_b = std::sqrt(std::max(0.0, s1[3] + s2[3] - s2[4] * s2[4]));
  }
  // cost tables (positions, row sums of the slab cost, their total) and ||c||
  tab_host.assign((size_t)std::max<int64_t>(lay.tab_len, 1), 0.0);
  int coord = 0;
  for (size_t p = 0; p < np; ++p) {
    PairGeo& g = lay.geo[p];
    double sq4[2];
    for (int fam = 0; fam < 2; ++fam) {
      const FamGeo& F = g.f[fam];
      const int L = F.L;
      const double* given = nullptr;
      if (pos_at[p] >= 0 && (fam == 0 ? probs[p].coord_row : probs[p].coord_col))
        given = &pos[pos_at[p] + (fam == 0 ? 0 : g.m)];
      double* X = &tab_host[F.xoff - lay.tab_off];
      double* CR = X + L;
      double cc = 0.0, q4 = 0.0;
      for (int q = 0; q < L; ++q) X[q] = given ? given[q] : (double)q;
      for (int a = 0; a < L; ++a) {
        if (given) {
          double r = 0.0;
          for (int q = 0; q < L; ++q) {
            const double d = X[a] - X[q];
            r += d * d;
            q4 += (d * d) * (d * d);
          }
          CR[a] = r;
        } else {
          CR[a] = cost_rowsum(L, a);  // exact integers
        }
        cc += CR[a];
      }
      X[2 * L] = cc;
      sq4[fam] = given ? q4 : slab_cost_sq(L);
      if (given) {
        coord = 1;
        if (!std::isfinite(cc) || !std::isfinite(q4)) {
          ctx->err = "grid positions must be finite (problem " + std::to_string(p) + ")";
          return HOT_E_INVALID;
        }
      }
    }
    g.norm_c = std::sqrt((double)g.n * sq4[0] + (double)g.m * sq4[1]);
    if (!std::isfinite(g.norm_c)) {
      ctx->err = "cost norm overflows (problem " + std::to_string(p) + ")";
      return HOT_E_INVALID;
    }
  }
  // sigma re-balancing needs x_bar and y_bar of the last restart
  int su = 0;
  for (size_t p = 0; p < np; ++p)
    if ((probs[p].flags & HOT_FLAG_SIGMA_UPDATE) && (probs[p].flags & HOT_FLAG_RESTART) &&
        !(probs[p].flags & (HOT_FLAG_FIXED_ITERS | HOT_FLAG_ADMM)))
      su = 1;
  if (su && !sbx) {
    const size_t xb = (size_t)lay.state_elems * lay.elem_size;
    const size_t yb = (size_t)lay.tab_off * 8;
    void* xbuf = nullptr;
    void* ybuf = nullptr;
    hot_status s1 = device_buffer(ctx, &xbuf, xb);
    if (s1 == HOT_OK) s1 = device_buffer(ctx, &ybuf, yb);
    if (s1 != HOT_OK) return s1;
    if (arena && arena_used > arena_bytes) {
      ctx->err = "problem needs " + std::to_string(arena_used) +
                 " bytes of device scratch (sigma re-balancing included), more than the " +
                 std::to_string(arena_bytes) + " the no-alloc entry point holds";
      return HOT_E_INVALID;
    }
    sbx = xbuf;
    abY = (double*)ybuf;
  }
  const int variant = coord | (su << 1);
  if (graph_exec && graph_variant != variant) {  // captured with other slab kernels
    (void)hipGraphExecDestroy(graph_exec);
    (void)hipGraphDestroy(graph);
    graph_exec = nullptr;
    graph = nullptr;
  }
  args.coord = coord;
  args.su = su;
  args.sbx = su ? sbx : nullptr;
  args.abY = su ? abY : nullptr;
  HIPCK(hipMemcpyAsync(geo_d, lay.geo.data(), np * sizeof(PairGeo), hipMemcpyHostToDevice, st));
  HIPCK(hipMemcpyAsync(items_d, lay.items.data(), lay.items.size() * sizeof(SlabItem),
                       hipMemcpyHostToDevice, st));
  if (!lay.sitems.empty())
    HIPCK(hipMemcpyAsync(sitems_d, lay.sitems.data(), lay.sitems.size() * sizeof(SmallItem),
                         hipMemcpyHostToDevice, st));
  HIPCK(hipMemcpyAsync(blocks_d, lay.blocks.data(), lay.blocks.size() * sizeof(PBlock),
                       hipMemcpyHostToDevice, st));
  HIPCK(hipMemcpyAsync(sblocks_d, lay.sblocks.data(), lay.sblocks.size() * sizeof(PBlock),
                       hipMemcpyHostToDevice, st));
  std::vector<PairCtl> c0(np * 2);
  std::memset(c0.data(), 0, c0.size() * sizeof(PairCtl));
  for (size_t p = 0; p < np; ++p) {
    const hot_problem& pr = probs[p];
    PairCtl& c = c0[p];
    const double nb = lay.geo[p].norm_b, nc = lay.geo[p].norm_c;
    c.sigma = pr.sigma > 0 ? pr.sigma : ((nc > 0 && nb > 0) ? nb / nc : 1.0);
    c.tol = pr.tol;
    c.lam = 0.5;
    c.k = 0;
    c.it = 0;
    c.status = ST_RUNNING;
    c.mode = MODE_INIT;
    c.src = 0;
    c.dst = 1;
    c.anc = -1;
    c.max_iter = pr.max_iter;
    c.T = pr.check_every;
    c.flags = (int32_t)pr.flags;
    // sigma re-balancing acts at restarts only
    if (!(pr.flags & HOT_FLAG_RESTART) || (pr.flags & (HOT_FLAG_FIXED_ITERS | HOT_FLAG_ADMM)))
      c.flags &= ~(int32_t)HOT_FLAG_SIGMA_UPDATE;
    if (ctx->tune.pingpong) c.flags |= 0x100;
    if (ctx->tune.sep_anchor && (pr.flags & HOT_FLAG_FIXED_ITERS)) c.flags |= 0x200;
    c.relax = (pr.flags & HOT_FLAG_ADMM) ? (pr.relax > 0 ? pr.relax : 1.7) : 0.0;
    c.sig_old = c.sigma;
    c0[np + p] = c;
    c0[np + p].mode = MODE_IDLE;
  }
  HIPCK(hipMemcpyAsync(ctl_d, c0.data(), c0.size() * sizeof(PairCtl), hipMemcpyHostToDevice, st));
  for (size_t p = 0; p < np; ++p) {
    const PairGeo& g = lay.geo[p];
    launch_setup_mu(probs[p].mu1, probs[p].mu2, g.m, g.n, arr + arr_mu1T(g), arr + arr_mu2(g),
                    st);
  }
  // zero fills by a kernel (no memset nodes, should a caller capture this)
  launch_zero(sb[0], (size_t)lay.state_elems * lay.elem_size, st);
  if (ctx->tune.sep_anchor) launch_zero(sb[2], (size_t)lay.state_elems * lay.elem_size, st);
  for (int q = 0; q < 2; ++q) {
    launch_zero(rowsum[q], lay.rs_len * 8, st);
    launch_zero(colpart[q], lay.cp_len * 8, st);
  }
  launch_zero(ab, lay.ab_len * 8, st);
  if (args.su) {  // X = 0, Y = 0 before the first restart (the initial point)
    launch_zero(sbx, (size_t)lay.state_elems * lay.elem_size, st);
    launch_zero(abY, (size_t)lay.tab_off * 8, st);
  }
  HIPCK(hipMemcpyAsync(ab + lay.tab_off, tab_host.data(), (size_t)lay.tab_len * 8,
                       hipMemcpyHostToDevice, st));
  launch_zero(kitem, lay.items.size() * kKI * 8, st);
  launch_zero(sync_d, lay.geo.size() * 5 * sizeof(unsigned), st);
  launch_zero(bytes_ctr, 8, st);
  HIPCK(hipGetLastError());
  // the host buffers above are pageable and the copies may still read them
  HIPCK(hipStreamSynchronize(st));
  return HOT_OK;
}

// One problem into slot s of a shared server group: the steps of setup()
// for that problem, on the slot's ranges only (the other slots may hold
// running problems; the stream is idle between their quanta).
hot_status Workspace::setup_slot(hot_ctx* ctx, int s, const hot_problem& pr, const PairGeo& gin,
                                 hipStream_t st) {
  const size_t K = lay.geo.size();
  PairGeo g = gin;
  const int m = g.m, n = g.n;
  const double* ptrs[2] = {pr.mu1, pr.mu2};
  const int64_t lens[2] = {(int64_t)m * n, (int64_t)m * n};
  const double** pd = (const double**)ptrs_d;
  int64_t* ld = (int64_t*)((char*)ptrs_d + K * 2 * sizeof(void*));
  HIPCK(hipMemcpyAsync(pd, ptrs, 2 * sizeof(void*), hipMemcpyHostToDevice, st));
  HIPCK(hipMemcpyAsync(ld, lens, 2 * 8, hipMemcpyHostToDevice, st));
  launch_hist_stats_multi(pd, ld, 2, stats_d, st);
  HIPCK(hipGetLastError());
  double stats[16];
  HIPCK(hipMemcpyAsync(stats, stats_d, sizeof(stats), hipMemcpyDeviceToHost, st));
  std::vector<double> pos;
  if (pr.coord_row || pr.coord_col) {
    pos.assign((size_t)m + n, 0.0);
    if (pr.coord_row)
      HIPCK(hipMemcpyAsync(pos.data(), pr.coord_row, (size_t)m * 8, hipMemcpyDeviceToHost, st));
    if (pr.coord_col)
      HIPCK(hipMemcpyAsync(pos.data() + m, pr.coord_col, (size_t)n * 8, hipMemcpyDeviceToHost, st));
  }
  HIPCK(hipStreamSynchronize(st));
  const double* s1 = stats;
  const double* s2 = stats + 8;
  if (s1[2] > 0 || s2[2] > 0) {
    ctx->err = "histogram has non-finite entries";
    return HOT_E_INVALID;
  }
  if (s1[0] < 0 || s2[0] < 0) {
    ctx->err = "histogram has negative entries";
    return HOT_E_INVALID;
  }
  const double tot = std::max(s1[1], s2[1]);
  if (!(tot > 0) || std::fabs(s1[1] - s2[1]) > 1e-9 * tot) {
    ctx->err = "histogram totals differ or are zero";
    return HOT_E_INVALID;
  }
  g.norm_b = std::sqrt(std::max(0.0, s1[3] + s2[3] - s2[4] * s2[4]));
  // cost tables of both families, as setup() builds them
  std::vector<double> tab[2];
  double sq4[2];
  for (int fam = 0; fam < 2; ++fam) {
    const int L = g.f[fam].L;
    const bool given = fam == 0 ? pr.coord_row != nullptr : pr.coord_col != nullptr;
    tab[fam].assign(2 * (size_t)L + 1, 0.0);
    double* X = tab[fam].data();
    double* CR = X + L;
    double cc = 0.0, q4 = 0.0;
    for (int q = 0; q < L; ++q) X[q] = given ? pos[(fam == 0 ? 0 : m) + q] : (double)q;
    for (int a = 0; a < L; ++a) {
      if (given) {
        double r = 0.0;
        for (int q = 0; q < L; ++q) {
          const double d = X[a] - X[q];
          r += d * d;
          q4 += (d * d) * (d * d);
        }
        CR[a] = r;
      } else {
        CR[a] = cost_rowsum(L, a);
      }
      cc += CR[a];
    }
    X[2 * L] = cc;
    sq4[fam] = given ? q4 : slab_cost_sq(L);
    if (given && (!std::isfinite(cc) || !std::isfinite(q4))) {
      ctx->err = "grid positions must be finite";
      return HOT_E_INVALID;
    }
  }
  g.norm_c = std::sqrt((double)n * sq4[0] + (double)m * sq4[1]);
  if (!std::isfinite(g.norm_c)) {
    ctx->err = "cost norm overflows";
    return HOT_E_INVALID;
  }
  const bool su = (pr.flags & HOT_FLAG_SIGMA_UPDATE) && (pr.flags & HOT_FLAG_RESTART) &&
                  !(pr.flags & (HOT_FLAG_FIXED_ITERS | HOT_FLAG_ADMM));
  if (su && !sbx) {
    void* xbuf = nullptr;
    void* ybuf = nullptr;
    hot_status a = device_buffer(ctx, &xbuf, (size_t)lay.state_elems * lay.elem_size);
    if (a == HOT_OK) a = device_buffer(ctx, &ybuf, (size_t)lay.tab_off * 8);
    if (a != HOT_OK) return a;
    sbx = xbuf;
    abY = (double*)ybuf;
  }
  // control blocks (both parities), as setup() writes them
  PairCtl c;
  std::memset(&c, 0, sizeof(c));
  c.sigma = pr.sigma > 0 ? pr.sigma : ((g.norm_c > 0 && g.norm_b > 0) ? g.norm_b / g.norm_c : 1.0);
  c.tol = pr.tol;
  c.lam = 0.5;
  c.status = ST_RUNNING;
  c.mode = MODE_INIT;
  c.src = 0;
  c.dst = 1;
  c.anc = -1;
  c.max_iter = pr.max_iter;
  c.T = pr.check_every;
  c.flags = (int32_t)pr.flags;
  if (!su) c.flags &= ~(int32_t)HOT_FLAG_SIGMA_UPDATE;
  if (ctx->tune.pingpong) c.flags |= 0x100;
  c.relax = (pr.flags & HOT_FLAG_ADMM) ? (pr.relax > 0 ? pr.relax : 1.7) : 0.0;
  c.sig_old = c.sigma;
  PairCtl idle = c;
  idle.mode = MODE_IDLE;
  const PairCtl cs[2] = {c, idle};
  HIPCK(hipMemcpyAsync(ctl_d + s, &cs[0], sizeof(PairCtl), hipMemcpyHostToDevice, st));
  HIPCK(hipMemcpyAsync(ctl_d + K + s, &cs[1], sizeof(PairCtl), hipMemcpyHostToDevice, st));
  launch_setup_mu(pr.mu1, pr.mu2, m, n, arr + arr_mu1T(g), arr + arr_mu2(g), st);
  // the slot's ranges, zero-filled by a kernel
  const size_t es = lay.elem_size;
  launch_zero((char*)sb[0] + (size_t)s * caps.state * es, (size_t)caps.state * es, st);
  if (ctx->tune.sep_anchor)
    launch_zero((char*)sb[2] + (size_t)s * caps.state * es, (size_t)caps.state * es, st);
  for (int q = 0; q < 2; ++q) {
    launch_zero(rowsum[q] + s * caps.rs, (size_t)caps.rs * 8, st);
    launch_zero(colpart[q] + s * caps.cp, (size_t)caps.cp * 8, st);
  }
  launch_zero(ab + s * caps.ab, (size_t)caps.ab * 8, st);
  if (su) {
    launch_zero((char*)sbx + (size_t)s * caps.state * es, (size_t)caps.state * es, st);
    launch_zero(abY + s * caps.ab, (size_t)caps.ab * 8, st);
  }
  for (int fam = 0; fam < 2; ++fam)
    HIPCK(hipMemcpyAsync(ab + g.f[fam].xoff, tab[fam].data(), tab[fam].size() * 8,
                         hipMemcpyHostToDevice, st));
  launch_zero(kitem + s * caps.items * kKI, (size_t)caps.items * kKI * 8, st);
  launch_zero(sync_d + 2 * s, 2 * sizeof(unsigned), st);
  launch_zero(sync_d + 2 * K + 2 * s, 2 * sizeof(unsigned), st);
  launch_zero(sync_d + 4 * K + s, sizeof(unsigned), st);
  HIPCK(hipMemcpyAsync(geo_d + s, &g, sizeof(PairGeo), hipMemcpyHostToDevice, st));
  HIPCK(hipGetLastError());
  HIPCK(hipStreamSynchronize(st));  // (the host sources above are on this stack)
  lay.geo[s] = g;
  return HOT_OK;
}

hot_status Workspace::init_group(hot_ctx* ctx, hipStream_t st) {
  const size_t K = lay.geo.size();
  HIPCK(hipMemcpyAsync(geo_d, lay.geo.data(), K * sizeof(PairGeo), hipMemcpyHostToDevice, st));
  launch_zero(ctl_d, 2 * K * sizeof(PairCtl), st);
  launch_zero(sync_d, 5 * K * sizeof(unsigned), st);
  HIPCK(hipGetLastError());
  HIPCK(hipStreamSynchronize(st));
  return HOT_OK;
}

// Work tables of the occupied slots of a shared group (the stream is idle).
hot_status Workspace::set_tables(hot_ctx* ctx, const std::vector<SlabItem>& items,
                                 const std::vector<PBlock>& blocks,
                                 const std::vector<PBlock>& sblocks, int coord, int su,
                                 hipStream_t st) {
  if (items.size() > lay.items.size() || blocks.size() > lay.blocks.size() ||
      sblocks.size() > lay.sblocks.size()) {
    ctx->err = "group tables exceed their capacity";
    return HOT_E_INVALID;
  }
  if (!items.empty())
    HIPCK(hipMemcpyAsync(items_d, items.data(), items.size() * sizeof(SlabItem),
                         hipMemcpyHostToDevice, st));
  if (!blocks.empty())
    HIPCK(hipMemcpyAsync(blocks_d, blocks.data(), blocks.size() * sizeof(PBlock),
                         hipMemcpyHostToDevice, st));
  if (!sblocks.empty())
    HIPCK(hipMemcpyAsync(sblocks_d, sblocks.data(), sblocks.size() * sizeof(PBlock),
                         hipMemcpyHostToDevice, st));
  HIPCK(hipStreamSynchronize(st));
  int maxvpl = 1;
  for (const SlabItem& it : items) maxvpl = std::max(maxvpl, (int)lay.geo[it.pair].f[it.fam].vpl);
  args.items = items_d;
  args.nitems = (int)items.size();
  args.nbig = (int)items.size();
  args.sitems = sitems_d;
  args.nsitems = 0;
  args.blocks = blocks_d;
  args.nblocks = (int)blocks.size();
  args.sblocks = sblocks_d;
  args.nsblocks = (int)sblocks.size();
  args.maxvpl = maxvpl;
  args.coord = coord;
  args.su = su;
  args.sbx = su ? sbx : nullptr;
  args.abY = su ? abY : nullptr;
  launch_pairs = (int)lay.geo.size();
  if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
  if (graph) (void)hipGraphDestroy(graph);
  graph_exec = nullptr;
  graph = nullptr;
  return HOT_OK;
}

hot_status Workspace::escalate(hot_ctx* ctx, hipStream_t st) {
  if (!lay.fp32 || arena) return HOT_OK;
  const size_t bytes = (size_t)lay.state_elems * 8;
  void* nb[3] = {nullptr, nullptr, nullptr};
  void* nx = nullptr;
  hot_status s = HOT_OK;
  for (int b = 0; b < 3 && s == HOT_OK; ++b) s = device_buffer(ctx, &nb[b], bytes);
  if (s == HOT_OK && sbx) s = device_buffer(ctx, &nx, bytes);
  if (s != HOT_OK) return s;  // (the new buffers stay in allocs, freed with the workspace)
  for (int b = 0; b < 3; ++b) launch_widen(sb[b], nb[b], lay.state_elems, st);
  if (sbx) launch_widen(sbx, nx, lay.state_elems, st);
  HIPCK(hipGetLastError());
  HIPCK(hipStreamSynchronize(st));
  auto drop = [&](void* p) {
    auto it = std::find(allocs.begin(), allocs.end(), p);
    if (it != allocs.end()) allocs.erase(it);
    (void)hipFree(p);
  };
  for (int b = 0; b < 3; ++b) {
    drop(sb[b]);
    sb[b] = nb[b];
    args.sb[b] = nb[b];
  }
  if (sbx) {
    drop(sbx);
    sbx = nx;
    args.sbx = nx;
  }
  relane_layout(lay, 0, ctx->tune);
  HIPCK(hipMemcpyAsync(geo_d, lay.geo.data(), lay.geo.size() * sizeof(PairGeo),
                       hipMemcpyHostToDevice, st));
  // A new epoch starts at the widened state: the next pass is a restart pass
  // (anchor = max(s - g, g) with the y_bar already solved for s).  Without it
  // the FP64 passes would continue an epoch whose Halpern weight has decayed
  // over the stalled FP32 iterations and whose restart reference sits at the
  // FP32 noise floor.  At a graph boundary the next pass reads ctl[0].
  std::vector<PairCtl> c0(lay.geo.size());
  HIPCK(hipMemcpyAsync(c0.data(), ctl_d, c0.size() * sizeof(PairCtl), hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  for (PairCtl& c : c0) {
    // (src == 2: an epoch starts at this very state already)
    if (c.status != ST_RUNNING || c.mode == MODE_INIT || c.mode == MODE_IDLE || c.src == 2)
      continue;
    c.mode = MODE_RESTART;
    c.sig_old = c.sigma;
    c.k = 0;
    c.it += 1;
    c.restarts += 1;
  }
  HIPCK(hipMemcpyAsync(ctl_d, c0.data(), c0.size() * sizeof(PairCtl), hipMemcpyHostToDevice, st));
  HIPCK(hipStreamSynchronize(st));
  args.fp32 = 0;
  args.maxvpl = lay.maxvpl;
  args.unroll = ctx->tune.unroll_for(lay.key_elems, lay.key_pairs, 0);
  if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
  if (graph) (void)hipGraphDestroy(graph);
  graph_exec = nullptr;
  graph = nullptr;
  return HOT_OK;
}

// Stall of an FP32-stream solve (HOT_FLAG_ESCALATE): the relative KKT at the
// checks has not halved over the last max(1000, k_best / 4) iterations, k_best
// the iteration of the last halving, with at least two restarts done.  (A
// restarted solve in FP64 halves its KKT every few hundred iterations on
// these grids; a premature switch costs at most the FP64 price per pass.)
bool StallWatch::stalled(const PairCtl& c) {
  if (c.kkt > 0.0 && (best == 0.0 || c.kkt < 0.5 * best)) {
    best = c.kkt;
    it_best = c.it;
  }
  return best > 0.0 && c.restarts >= 2 &&
         (int64_t)c.it - it_best > std::max<int64_t>(1000, it_best / 4);
}

static bool use_graphs() {
  const char* e = std::getenv("HOT_NO_GRAPH");
  return !(e && e[0] == '1');
}

// Run graph launches until every problem has stopped.
hot_status Workspace::run(hot_ctx* ctx, hipStream_t st, int64_t max_graphs, StallWatch* watch) {
  const size_t np = lay.geo.size();
  if (profile) return run_profiled(ctx, st, max_graphs, watch);
  const bool graphs = use_graphs();
  if (graphs && !graph_exec) {
    HIPCK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < kGraphIters; ++i) launch_iteration(args, i & 1, st);
    hipError_t e = hipStreamEndCapture(st, &graph);
    if (e != hipSuccess) {
      ctx->err = std::string("graph capture failed: ") + hipGetErrorString(e);
      return HOT_E_DEVICE;
    }
    HIPCK(hipGraphInstantiate(&graph_exec, graph, nullptr, nullptr, 0));
    graph_variant = args.coord | (args.su << 1);
  }
  hipEvent_t ev[2];
  HIPCK(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  HIPCK(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  PairCtl* hc[2] = {host_ctl, host_ctl + np};
  int64_t launched = 0;
  hot_status result = HOT_OK;
  auto launch_one = [&](int slot) -> hipError_t {
    hipError_t e;
    if (graphs) {
      e = hipGraphLaunch(graph_exec, st);
    } else {
      for (int i = 0; i < kGraphIters; ++i) launch_iteration(args, i & 1, st);
      e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(hc[slot], ctl_d, np * sizeof(PairCtl), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    return hipEventRecord(ev[slot], st);
  };
  hipError_t e = launch_one(0);
  launched = 1;
  int cur = 0;
  while (e == hipSuccess) {
    // keep one graph in flight while the previous one's status is read
    if (launched < max_graphs) {
      if (launched == nan_after) e = poison_state(st);
      if (e != hipSuccess) break;
      e = launch_one(cur ^ 1);
      if (e != hipSuccess) break;
      ++launched;
    }
    iterations_launched = launched * kGraphIters;
    e = hipEventSynchronize(ev[cur]);
    if (e != hipSuccess) break;
    bool all_done = true;
    for (size_t p = 0; p < np; ++p)
      if (hc[cur][p].status == ST_RUNNING) all_done = false;
    if (all_done || launched >= max_graphs) {
      if (launched > 1 && !all_done) {
        // last launched graph: wait for it too
        e = hipEventSynchronize(ev[cur ^ 1]);
      }
      break;
    }
    if (watch && lay.fp32 && np == 1 && watch->stalled(hc[cur][0])) {
      // drain the graph in flight, widen the state, restart the pipeline
      // (at a graph boundary the latest control blocks are ctl[0])
      e = hipStreamSynchronize(st);
      if (e == hipSuccess) e = hipMemcpy(hc[0], ctl_d, np * sizeof(PairCtl), hipMemcpyDeviceToHost);
      if (e != hipSuccess) break;
      if (hc[0][0].status != ST_RUNNING) break;
      const hot_status es = escalate(ctx, st);
      if (es != HOT_OK) {
        result = es;
        break;
      }
      escalated_at = hc[0][0].it;
      if (graphs) {
        const hot_status gs = ensure_graph(ctx, st);
        if (gs != HOT_OK) {
          result = gs;
          break;
        }
      }
      e = launch_one(0);
      ++launched;
      cur = 0;
      continue;
    }
    cur ^= 1;
  }
  if (e != hipSuccess && result == HOT_OK) {
    ctx->err = std::string("iteration launch failed: ") + hipGetErrorString(e);
    result = HOT_E_DEVICE;
  }
  (void)hipStreamSynchronize(st);
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (result == HOT_OK) {
    // the final control blocks: after whole graphs the latest copy is ctl[0]
    e = finalize(st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipMemcpy(host_ctl, ctl_d, np * sizeof(PairCtl), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      ctx->err = std::string("status copy failed: ") + hipGetErrorString(e);
      result = HOT_E_DEVICE;
    }
  }
  return result;
}

// Failure-path test hook: a NaN into the first flow element of every state
// buffer (whichever the next pass reads), ordered on the stream between two
// graphs.  Only contexts created with HOT_TEST_NAN_AFTER set ever call it.
hipError_t Workspace::poison_state(hipStream_t st) {
  static const double nan64 = std::nan("");
  static const float nan32 = std::nanf("");
  const void* src = lay.fp32 ? (const void*)&nan32 : (const void*)&nan64;
  const int64_t off = std::min(lay.geo[0].f[0].soff, lay.geo[0].f[1].soff);
  for (int b = 0; b < 3; ++b) {
    hipError_t e = hipMemcpyAsync((char*)sb[b] + off * lay.elem_size, src, lay.elem_size,
                                  hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// No-alloc run: direct launches of kGraphIters iterations on st, then the
// control blocks are copied back and st is synchronised; no graph, event or
// pinned buffer.  Same kernels in the same order as run().
hot_status Workspace::run_direct(hot_ctx* ctx, hipStream_t st, int64_t max_graphs) {
  const size_t np = lay.geo.size();
  for (int64_t g = 0; g < max_graphs; ++g) {
    for (int i = 0; i < kGraphIters; ++i) launch_iteration(args, i & 1, st);
    HIPCK(hipGetLastError());
    iterations_launched += kGraphIters;
    HIPCK(hipMemcpyAsync(host_ctl, ctl_d, np * sizeof(PairCtl), hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    bool all_done = true;
    for (size_t p = 0; p < np; ++p)
      if (host_ctl[p].status == ST_RUNNING) all_done = false;
    if (all_done) break;
  }
  HIPCK(finalize(st));
  HIPCK(hipMemcpyAsync(host_ctl, ctl_d, np * sizeof(PairCtl), hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  return HOT_OK;
}

hipError_t Workspace::finalize(hipStream_t st) {
  if (group)  // the occupied slots' items (a free slot's geometry covers no item)
    launch_finalize(args, args.items, args.nitems, (int)lay.geo.size(), st);
  else
    launch_finalize(args, items_d, (int)lay.items.size(), (int)lay.geo.size(), st);
  return hipGetLastError();
}

// Profiling run: direct launches, a hipEvent pair around every slab pass on
// the workspace stream, no pipelining.  Same kernels and iteration order as
// the graph path.
hot_status Workspace::run_profiled(hot_ctx* ctx, hipStream_t st, int64_t max_graphs,
                                   StallWatch* watch) {
  const size_t np = lay.geo.size();
  std::vector<hipEvent_t> evs(2 * kGraphIters);
  for (auto& e : evs) HIPCK(hipEventCreate(&e));
  hot_status result = HOT_OK;
  bool esc_next = false;  // widen one graph after the stall, as run() does
  for (int64_t g = 0; g < max_graphs; ++g) {
    for (int i = 0; i < kGraphIters; ++i) {
      HIPCK(hipEventRecord(evs[2 * i], st));
      launch_slab_pass(args, i & 1, st);
      HIPCK(hipEventRecord(evs[2 * i + 1], st));
      launch_pair_kernels(args, i & 1, st);
    }
    HIPCK(hipGetLastError());
    HIPCK(hipMemcpyAsync(host_ctl, ctl_d, np * sizeof(PairCtl), hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    for (int i = 0; i < kGraphIters; ++i) {
      float ms = 0.f;
      HIPCK(hipEventElapsedTime(&ms, evs[2 * i], evs[2 * i + 1]));
      prof_seconds += ms * 1e-3;
      ++prof_launches;
    }
    iterations_launched += kGraphIters;
    bool all_done = true;
    for (size_t p = 0; p < np; ++p)
      if (host_ctl[p].status == ST_RUNNING) all_done = false;
    if (all_done) break;
    if (esc_next) {
      esc_next = false;
      result = escalate(ctx, st);
      if (result != HOT_OK) break;
      escalated_at = host_ctl[0].it;
    } else if (watch && lay.fp32 && np == 1 && watch->stalled(host_ctl[0])) {
      esc_next = true;
    }
  }
  for (auto& e : evs) (void)hipEventDestroy(e);
  HIPCK(finalize(st));
  HIPCK(hipMemcpyAsync(host_ctl, ctl_d, np * sizeof(PairCtl), hipMemcpyDeviceToHost, st));
  HIPCK(hipStreamSynchronize(st));
  return result;
}

// Full launch tables (every problem of the workspace); retires a graph
// captured with compacted ones.
void Workspace::restore_tables() {
  const bool compacted = args.items != items_d;
  args.items = items_d;
  args.nitems = (int)lay.items.size();
  args.nbig = (int)lay.nbig;
  args.sitems = sitems_d;
  args.nsitems = (int)lay.sitems.size();
  args.blocks = blocks_d;
  args.nblocks = (int)lay.blocks.size();
  args.sblocks = sblocks_d;
  args.nsblocks = (int)lay.sblocks.size();
  launch_pairs = (int)lay.geo.size();
  if (compacted && graph_exec) {
    retired.push_back({graph, graph_exec});
    graph = nullptr;
    graph_exec = nullptr;
  }
}

// Between graphs: when at most half of the problems the current tables
// cover are still running, launch only those from now on (their results do
// not depend on which other problems share a launch).  The new tables are
// uploaded on the workspace's stream, so graphs still in flight finish
// with the old ones first; the graph is re-captured with the new tables.
hot_status Workspace::compact(hot_ctx* ctx, const PairCtl* hc) {
  if (!stage_h) return HOT_OK;
  const size_t np = lay.geo.size();
  std::vector<char> act(np, 0);
  int active = 0;
  for (size_t p = 0; p < np; ++p)
    if (hc[p].status == ST_RUNNING) {
      act[p] = 1;
      ++active;
    }
  if (active == 0 || 2 * active > launch_pairs) return HOT_OK;
  // the previous compaction's uploads read stage_h asynchronously, queued
  // behind graphs that may still run: wait for them before rewriting it
  if (stage_pending) {
    HIPCK(hipEventSynchronize(stage_ev));
    stage_pending = false;
  }
  if (!stage_ev) HIPCK(hipEventCreateWithFlags(&stage_ev, hipEventDisableTiming));
  SlabItem* it = (SlabItem*)stage_h;
  SmallItem* si = (SmallItem*)((char*)stage_h + std::max<size_t>(lay.items.size(), 1) * sizeof(SlabItem));
  PBlock* bl = (PBlock*)((char*)si + std::max<size_t>(lay.sitems.size(), 1) * sizeof(SmallItem));
  PBlock* sb = bl + std::max<size_t>(lay.blocks.size(), 1);
  int nit = 0, nbig = 0, nsi = 0, nbl = 0, nsb = 0;
  for (const SlabItem& x : lay.items)  // block plain-update items first, as in the layout
    if (act[x.pair] && !x.small) it[nit++] = x;
  nbig = nit;
  for (const SlabItem& x : lay.items)
    if (act[x.pair] && x.small) it[nit++] = x;
  for (const SmallItem& x : lay.sitems)
    if (act[x.pair]) si[nsi++] = x;
  for (const PBlock& x : lay.blocks)
    if (act[x.pair]) bl[nbl++] = x;
  for (const PBlock& x : lay.sblocks)
    if (act[x.pair]) sb[nsb++] = x;
  HIPCK(hipMemcpyAsync(items_c, it, (size_t)std::max(nit, 1) * sizeof(SlabItem),
                       hipMemcpyHostToDevice, stream));
  if (nsi > 0)
    HIPCK(hipMemcpyAsync(sitems_c, si, (size_t)nsi * sizeof(SmallItem), hipMemcpyHostToDevice,
                         stream));
  HIPCK(hipMemcpyAsync(blocks_c, bl, (size_t)nbl * sizeof(PBlock), hipMemcpyHostToDevice, stream));
  HIPCK(hipMemcpyAsync(sblocks_c, sb, (size_t)nsb * sizeof(PBlock), hipMemcpyHostToDevice, stream));
  HIPCK(hipEventRecord(stage_ev, stream));
  stage_pending = true;
  if (graph_exec) retired.push_back({graph, graph_exec});
  graph = nullptr;
  graph_exec = nullptr;
  args.items = items_c;
  args.nitems = nit;
  args.nbig = nbig;
  args.sitems = sitems_c;
  args.nsitems = nsi;
  args.blocks = blocks_c;
  args.nblocks = nbl;
  args.sblocks = sblocks_c;
  args.nsblocks = nsb;
  launch_pairs = active;
  return ensure_graph(ctx, stream);
}

hot_status Workspace::ensure_graph(hot_ctx* ctx, hipStream_t st) {
  if (graph_exec) return HOT_OK;
  HIPCK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  for (int i = 0; i < kGraphIters; ++i) launch_iteration(args, i & 1, st);
  hipError_t e = hipStreamEndCapture(st, &graph);
  if (e != hipSuccess) {
    if (ctx) ctx->err = std::string("graph capture failed: ") + hipGetErrorString(e);
    return HOT_E_DEVICE;
  }
  HIPCK(hipGraphInstantiate(&graph_exec, graph, nullptr, nullptr, 0));
  graph_variant = args.coord | (args.su << 1);
  return HOT_OK;
}

hipError_t Workspace::launch_quantum(hipStream_t st) {
  hipError_t e;
  if (!quantum_event) {
    e = hipEventCreateWithFlags(&quantum_event, hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  e = hipGraphLaunch(graph_exec, st);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(host_ctl, ctl_d, lay.geo.size() * sizeof(PairCtl), hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  return hipEventRecord(quantum_event, st);
}

static hot_status status_of(int32_t s) {
  switch (s) {
    case ST_CONVERGED:
    case ST_FIXED_DONE:
      return HOT_OK;
    case ST_MAXITER:
      return HOT_E_NOT_CONVERGED;
    case ST_NUMERIC:
      return HOT_E_NUMERIC;
    case ST_SYNC_LOST:
      return HOT_E_DEVICE;
    default:
      return HOT_E_NOT_CONVERGED;
  }
}

void Workspace::fill_result(int p, hot_result* r, double seconds) const {
  const PairCtl& c = host_ctl[p];
  std::memset(r, 0, sizeof(*r));
  r->primal_obj = c.pobj;
  r->dual_obj = c.dobj;
  r->kkt = c.kkt;
  r->res_primal = c.res_p;
  r->res_dual = c.res_d;
  r->res_comp = c.res_c;
  r->sigma = c.sigma;
  r->seconds = seconds;
  r->kkt_abs = c.kkt_abs;
  r->iters = c.it;
  r->restarts = c.restarts;
  r->status = (int32_t)status_of(c.status);
  r->feaserr = c.feaserr;
  r->escalated_at = escalated_at;
}

}  // namespace hot


struct hot_batch {
  hot_ctx* ctx = nullptr;
  GroupedBatch gb;
  std::string key;  // workspace-cache key of its shapes and grouping
  std::thread th;
  hot_status status = HOT_OK;
  double seconds = 0;
  int count = 0;
};

extern "C" {

const char* hot_status_string(hot_status s) {
  switch (s) {
    case HOT_OK: return "ok";
    case HOT_E_INVALID: return "invalid argument";
    case HOT_E_NOMEM: return "out of device memory";
    case HOT_E_DEVICE: return "device error";
    case HOT_E_NOT_CONVERGED: return "not converged";
    case HOT_E_BUSY: return "busy";
    case HOT_E_CANCELLED: return "cancelled";
    case HOT_E_NUMERIC: return "non-finite value in iteration";
  }
  return "unknown status";
}

hot_status hot_ctx_create(int device, hot_ctx** out) {
  if (!out) return HOT_E_INVALID;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= device || device < 0) {
    (void)hipGetLastError();
    return HOT_E_DEVICE;
  }
  if (hipSetDevice(device) != hipSuccess) return HOT_E_DEVICE;
  hot_ctx* c = new hot_ctx();
  c->device = device;
  const char* e = std::getenv("HOT_ITEM_ELEMS");
  if (e) c->tune.item_elems = std::max<int64_t>(1024, std::atoll(e));
  e = std::getenv("HOT_MIN_ITEMS");
  if (e) c->tune.min_items = std::max<int64_t>(1, std::atoll(e));
  e = std::getenv("HOT_SMALL_SIDE");
  if (e) c->tune.small_side = std::max(0, std::atoi(e));
  e = std::getenv("HOT_REDUCE_GROUP");
  if (e) c->tune.reduce_group = std::max(0, std::min(16, std::atoi(e)));
  e = std::getenv("HOT_ROW_GROUP");
  if (e) c->tune.row_group = std::max(0, std::min(16, std::atoi(e)));
  e = std::getenv("HOT_SOLVE_PRE");
  if (e) c->tune.solve_pre = std::atoi(e) != 0;
  e = std::getenv("HOT_FUSE");
  if (e) c->tune.fuse = std::atoi(e) != 0;
  e = std::getenv("HOT_FUSE_PAIR");
  if (e) c->tune.fuse_pair = std::atoi(e) != 0;
  e = std::getenv("HOT_BATCH_GROUPS");
  if (e) c->tune.batch_groups = std::max(1, std::min(4, std::atoi(e)));
  e = std::getenv("HOT_VPL_TARGET");
  if (e) c->tune.vec_per_lane = std::max(1, std::min(8, std::atoi(e)));
  e = std::getenv("HOT_NT_STORE");
  if (e) c->tune.nt_store = std::atoi(e) != 0;
  e = std::getenv("HOT_PINGPONG");
  if (e) c->tune.pingpong = std::atoi(e) != 0;
  e = std::getenv("HOT_UNROLL");
  if (e) c->tune.unroll = std::atoi(e) >= 2 ? 2 : 1;
  e = std::getenv("HOT_TEST_NAN_AFTER");
  if (e) c->nan_after = std::max(1, std::atoi(e));
  // the no-alloc entry point's scratch array: its address on this device
  c->scratch = static_scratch_init(device, c->scratch_err);
  *out = c;
  return HOT_OK;
}

void hot_ctx_destroy(hot_ctx* ctx) { delete ctx; }

const char* hot_ctx_last_error(const hot_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

hot_status hot_ctx_set_profiling(hot_ctx* ctx, int on) {
  if (!ctx) return HOT_E_INVALID;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->profiling = on != 0;
  ctx->prof_seconds = ctx->prof_launches = ctx->prof_bytes = ctx->iters_launched = 0;
  return HOT_OK;
}

hot_status hot_ctx_profile_read(hot_ctx* ctx, double* out) {
  if (!ctx || !out) return HOT_E_INVALID;
  std::lock_guard<std::mutex> lk(ctx->mu);
  out[0] = ctx->prof_launches;
  out[1] = ctx->prof_seconds;
  out[2] = ctx->prof_bytes;
  out[3] = ctx->iters_launched;
  return HOT_OK;
}

size_t hot_footprint_bytes(int32_t m, int32_t n, int32_t prec, uint32_t flags) {
  Layout lay;
  std::string err;
  if (prec != HOT_FP64 && prec != HOT_FP32_STREAM) return 0;
  if (!build_layout({{m, n}}, prec == HOT_FP32_STREAM, default_tuning(), lay, err)) return 0;
  return lay.bytes(flags);
}

size_t hot_ctx_footprint_bytes(hot_ctx* ctx, int32_t m, int32_t n, int32_t prec, uint32_t flags) {
  Layout lay;
  std::string err;
  if (!ctx || (prec != HOT_FP64 && prec != HOT_FP32_STREAM)) return 0;
  if (!build_layout({{m, n}}, prec == HOT_FP32_STREAM, ctx->tune, lay, err)) return 0;
  return lay.bytes(flags);
}

int64_t hot_plan_capacity(int32_t m, int32_t n) {
  if (m < 1 || n < 1) return 0;
  const int64_t M = (int64_t)m * n;
  return M * (m + n - 1) + 2 * M - 1;
}

}  // extern "C"

namespace hot {

hot_status make_workspace(hot_ctx* ctx, const hot_problem* probs, int count,
                          std::shared_ptr<Workspace>& out, int64_t key_elems, int key_pairs) {
  if (count < 1) {
    ctx->err = "count must be >= 1";
    return HOT_E_INVALID;
  }
  std::vector<std::pair<int, int>> shapes;
  int prec = probs[0].prec;
  for (int p = 0; p < count; ++p) {
    hot_status s = validate_problem(ctx, &probs[p]);
    if (s != HOT_OK) return s;
    if (probs[p].prec != prec) {
      ctx->err = "all problems of a batch must use the same precision";
      return HOT_E_INVALID;
    }
    shapes.push_back({probs[p].m, probs[p].n});
  }
  auto ws = std::make_shared<Workspace>();
  std::string err;
  if (!build_layout(shapes, prec == HOT_FP32_STREAM, ctx->tune, ws->lay, err, key_elems,
                    key_pairs)) {
    ctx->err = err;
    return HOT_E_INVALID;
  }
  ws->device = ctx->device;
  ws->profile = ctx->profiling;
  ws->nan_after = ctx->nan_after;
  hot_status s = ws->alloc_all(ctx);
  {
    int64_t total = 0;
    for (int p = 0; p < count; ++p)
      total += (int64_t)probs[p].m * probs[p].m * probs[p].n + (int64_t)probs[p].m * probs[p].n * probs[p].n;
    if (key_elems >= 0) total = key_elems;
    ws->args.unroll = ctx->tune.unroll_for(total, key_pairs >= 0 ? key_pairs : count,
                                           prec == HOT_FP32_STREAM);
  }
  ws->args.nt_store = ctx->tune.nt_store;
  ws->args.fuse = ctx->tune.fuse;
  ws->args.solve_pre = ctx->tune.solve_pre;
  ws->args.fuse_pair = ctx->tune.fuse_pair;
  // the algorithmic byte count is kept only when the passes are timed
  ws->args.bytes_ctr = ws->profile ? ws->bytes_ctr : nullptr;
  if (s != HOT_OK) return s;
  if (hipStreamCreateWithFlags(&ws->stream, hipStreamNonBlocking) != hipSuccess) {
    ctx->err = "stream creation failed";
    return HOT_E_DEVICE;
  }
  ws->own_stream = true;
  out = ws;
  return HOT_OK;
}

hot_status make_groups(hot_ctx* ctx, const hot_problem* probs, int count, int groups,
                       GroupedBatch& gb) {
  gb = GroupedBatch();
  if (count < 1) {
    ctx->err = "count must be >= 1";
    return HOT_E_INVALID;
  }
  const int G = std::max(1, std::min(groups, count));
  auto elems = [&](int p) {
    return (int64_t)probs[p].m * probs[p].m * probs[p].n +
           (int64_t)probs[p].m * probs[p].n * probs[p].n;
  };
  int64_t total = 0;
  for (int p = 0; p < count; ++p) total += std::max<int64_t>(0, elems(p));
  // largest first onto the lightest group, then each group in input order
  std::vector<int> order(count);
  for (int p = 0; p < count; ++p) order[p] = p;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return elems(a) > elems(b); });
  std::vector<int64_t> load(G, 0);
  std::vector<std::vector<int>> members(G);
  for (int p : order) {
    const int g = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    members[g].push_back(p);
    load[g] += elems(p);
  }
  gb.where.assign(count, {0, 0});
  for (int g = 0; g < G; ++g) {
    std::sort(members[g].begin(), members[g].end());
    std::vector<hot_problem> sub;
    for (size_t q = 0; q < members[g].size(); ++q) {
      sub.push_back(probs[members[g][q]]);
      gb.where[members[g][q]] = {g, (int)q};
    }
    std::shared_ptr<Workspace> ws;
    // every group is laid out with the launch shape of the whole batch
    const hot_status s = make_workspace(ctx, sub.data(), (int)sub.size(), ws, total, count);
    if (s != HOT_OK) return s;
    gb.wss.push_back(ws);
  }
  return HOT_OK;
}

// at most this many cached entries / bytes per context
constexpr size_t kWsCacheEntries = 8;
constexpr size_t kWsCacheBytes = size_t(8) << 30;

std::string ws_cache_key(const hot_problem* probs, int count, int groups) {
  std::string k = std::to_string(groups) + "/" + std::to_string(probs[0].prec);
  for (int p = 0; p < count; ++p)
    k += "/" + std::to_string(probs[p].m) + "x" + std::to_string(probs[p].n);
  return k;
}

bool ws_cache_take(hot_ctx* ctx, const std::string& key, GroupedBatch& gb) {
  if (ctx->profiling || ctx->nan_after >= 0) return false;
  for (auto it = ctx->ws_cache.begin(); it != ctx->ws_cache.end(); ++it)
    if (it->key == key) {
      gb = std::move(it->gb);
      ctx->ws_cache_bytes -= it->bytes;
      ctx->ws_cache.erase(it);
      return true;
    }
  return false;
}

void ws_cache_put(hot_ctx* ctx, const std::string& key, GroupedBatch&& gb) {
  // (timed runs and failure-path tests build their own workspaces)
  if (ctx->profiling || ctx->nan_after >= 0) return;
  size_t bytes = 0;
  for (const auto& ws : gb.wss) {
    if (ws->profile || ws->arena) return;
    bytes += ws->lay.bytes(ws->sbx ? HOT_FLAG_SIGMA_UPDATE : 0);
  }
  if (bytes > kWsCacheBytes) return;
  hot_ctx::CachedWs e;
  e.key = key;
  e.gb = std::move(gb);
  e.bytes = bytes;
  ctx->ws_cache.push_front(std::move(e));
  ctx->ws_cache_bytes += bytes;
  while (ctx->ws_cache.size() > kWsCacheEntries || ctx->ws_cache_bytes > kWsCacheBytes) {
    ctx->ws_cache_bytes -= ctx->ws_cache.back().bytes;
    ctx->ws_cache.pop_back();
  }
}

void ws_cache_clear(hot_ctx* ctx) {
  ctx->ws_cache.clear();
  ctx->ws_cache_bytes = 0;
}

// Iterate several workspaces (disjoint problems) concurrently, each on its
// own stream with two captured graphs in flight, until all have stopped.
hot_status run_concurrent(hot_ctx* ctx, const std::vector<std::shared_ptr<Workspace>>& wss,
                          int64_t max_graphs) {
  if (wss.size() == 1 || !use_graphs() || wss[0]->profile) {
    for (const auto& ws : wss) {
      const hot_status s = ws->run(ctx, ws->stream, max_graphs);
      if (s != HOT_OK) return s;
    }
    return HOT_OK;
  }
  struct St {
    Workspace* ws;
    hipEvent_t ev[2];
    PairCtl* hc[2];
    int64_t launched;
    int cur;
    bool done;
  };
  std::vector<St> sts;
  hot_status result = HOT_OK;
  for (const auto& w : wss) {
    St t;
    t.ws = w.get();
    t.ev[0] = t.ev[1] = nullptr;
    const size_t np = w->lay.geo.size();
    t.hc[0] = w->host_ctl;
    t.hc[1] = w->host_ctl + np;
    t.launched = 0;
    t.cur = 0;
    t.done = false;
    sts.push_back(t);
  }
  auto launch_one = [&](St& t, int slot) -> hipError_t {
    hipError_t e = hipGraphLaunch(t.ws->graph_exec, t.ws->stream);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(t.hc[slot], t.ws->ctl_d, t.ws->lay.geo.size() * sizeof(PairCtl),
                       hipMemcpyDeviceToHost, t.ws->stream);
    if (e != hipSuccess) return e;
    ++t.launched;
    t.ws->iterations_launched = t.launched * kGraphIters;
    return hipEventRecord(t.ev[slot], t.ws->stream);
  };
  hipError_t e = hipSuccess;
  for (St& t : sts) {
    if ((result = t.ws->ensure_graph(ctx, t.ws->stream)) != HOT_OK) break;
    for (int q = 0; q < 2 && e == hipSuccess; ++q)
      e = hipEventCreateWithFlags(&t.ev[q], hipEventDisableTiming);
    if (e == hipSuccess) e = launch_one(t, 0);
    if (e == hipSuccess && t.launched < max_graphs) e = launch_one(t, 1);
    if (e != hipSuccess) break;
  }
  bool busy = result == HOT_OK && e == hipSuccess;
  while (busy) {
    busy = false;
    for (St& t : sts) {
      if (t.done) continue;
      // graphs k (slot cur) and k+1 (slot cur^1) are queued; wait for k
      if ((e = hipEventSynchronize(t.ev[t.cur])) != hipSuccess) break;
      bool running = false;
      for (size_t p = 0; p < t.ws->lay.geo.size(); ++p)
        if (t.hc[t.cur][p].status == ST_RUNNING) running = true;
      if (!running || t.launched >= max_graphs) {
        t.done = true;
        continue;
      }
      if ((result = t.ws->compact(ctx, t.hc[t.cur])) != HOT_OK) break;
      if ((e = launch_one(t, t.cur)) != hipSuccess) break;  // graph k+2 reuses slot cur
      t.cur ^= 1;
      busy = true;
    }
    if (e != hipSuccess || result != HOT_OK) break;
  }
  if (result == HOT_OK && e != hipSuccess) {
    ctx->err = std::string("iteration launch failed: ") + hipGetErrorString(e);
    result = HOT_E_DEVICE;
  }
  for (St& t : sts) {
    (void)hipStreamSynchronize(t.ws->stream);
    t.ws->drop_retired();
    for (int q = 0; q < 2; ++q)
      if (t.ev[q]) (void)hipEventDestroy(t.ev[q]);
    if (result == HOT_OK) {
      // after whole graphs the latest control blocks are ctl[0]
      e = t.ws->finalize(t.ws->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(t.ws->stream);
      if (e == hipSuccess)
        e = hipMemcpy(t.ws->host_ctl, t.ws->ctl_d, t.ws->lay.geo.size() * sizeof(PairCtl),
                      hipMemcpyDeviceToHost);
      if (e != hipSuccess) {
        ctx->err = std::string("status copy failed: ") + hipGetErrorString(e);
        result = HOT_E_DEVICE;
      }
    }
  }
  return result;
}

}  // namespace hot

extern "C" {

hot_status hot_solve(hot_ctx* ctx, const hot_problem* prob, hot_stream_t stream,
                     hot_solution** sol_out, hot_result* res) {
  if (!ctx || !res) return HOT_E_INVALID;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->err.clear();
  if (sol_out) *sol_out = nullptr;
  if (hipSetDevice(ctx->device) != hipSuccess) return HOT_E_DEVICE;
  const auto t0 = std::chrono::steady_clock::now();
  std::shared_ptr<Workspace> ws;
  hot_status s = validate_problem(ctx, prob);
  if (s != HOT_OK) return s;
  const std::string key = ws_cache_key(prob, 1, 1);
  GroupedBatch cached;
  if (ws_cache_take(ctx, key, cached)) {
    ws = cached.wss[0];
  } else {
    s = make_workspace(ctx, prob, 1, ws);
    if (s != HOT_OK) return s;
  }
  hipStream_t st = ws->stream;
  // order after the caller's stream
  hipEvent_t ev;
  HIPCK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  HIPCK(hipEventRecord(ev, (hipStream_t)stream));
  HIPCK(hipStreamWaitEvent(st, ev, 0));
  (void)hipEventDestroy(ev);
  s = ws->setup(ctx, prob, 1, st);
  if (s != HOT_OK) return s;
  const int64_t max_graphs = (int64_t)prob->max_iter * 2 / kGraphIters + 8;
  StallWatch watch;
  const bool esc = (prob->flags & HOT_FLAG_ESCALATE) && prob->prec == HOT_FP32_STREAM &&
                   !(prob->flags & HOT_FLAG_FIXED_ITERS) && prob->tol > 0;
  s = ws->run(ctx, st, max_graphs, esc ? &watch : nullptr);
  if (s != HOT_OK) return s;
  collect_profile(ctx, *ws);
  const double secs =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  ws->fill_result(0, res, secs);
  if (!sol_out && ws->lay.fp32 == (prob->prec == HOT_FP32_STREAM ? 1 : 0)) {
    // kept for the next solve of this shape (not a widened one)
    GroupedBatch keep;
    keep.wss.push_back(ws);
    keep.where.push_back({0, 0});
    ws_cache_put(ctx, key, std::move(keep));
  }
  if (sol_out) {
    hot_solution* so = new hot_solution();
    so->ws = ws;
    so->pair = 0;
    so->m = prob->m;
    so->n = prob->n;
    so->prec = prob->prec;
    *sol_out = so;
  }
  return (hot_status)res->status;
}

void hot_solution_free(hot_solution* sol) { delete sol; }

hot_status hot_solution_export(hot_ctx* ctx, const hot_solution* sol, hot_stream_t stream,
                               double* xbar, double* ybar, double* zbar, double* s) {
  if (!ctx || !sol) return HOT_E_INVALID;
  std::lock_guard<std::mutex> lk(ctx->mu);
  const int64_t m = sol->m, n = sol->n;
  const int64_t N = m * m * n + m * n * n, M = m * n;
  hipStream_t st = (hipStream_t)stream;
  if (xbar || zbar || s) launch_export(sol->ws->args, 0, sol->pair, N, xbar, zbar, s, st);
  if (ybar) launch_export_y(sol->ws->args, sol->pair, 3 * M - 1, ybar, st);
  HIPCK(hipGetLastError());
  HIPCK(hipStreamSynchronize(st));
  return HOT_OK;
}

hot_status hot_solution_anchor(hot_ctx* ctx, const hot_solution* sol, hot_stream_t stream,
                               double* s0, double* info) {
  if (!ctx || !sol) return HOT_E_INVALID;
  std::lock_guard<std::mutex> lk(ctx->mu);
  const int64_t m = sol->m, n = sol->n;
  const int64_t N = m * m * n + m * n * n;
  hipStream_t st = (hipStream_t)stream;
  if (s0) launch_export(sol->ws->args, 0, sol->pair, N, nullptr, nullptr, nullptr, st, s0);
  HIPCK(hipGetLastError());
  HIPCK(hipStreamSynchronize(st));
  if (info) {
    // the control block the solve ended with (the last copy is ctl[0])
    const PairCtl& c = sol->ws->host_ctl[sol->pair];
    info[0] = (double)c.k;
    info[1] = c.lam;
    info[2] = c.sigma;
    info[3] = c.anc < 0 ? 0.0 : (c.anc == c.src ? 1.0 : 2.0);
  }
  return HOT_OK;
}

hot_status hot_aat_solve(hot_ctx* ctx, int32_t m, int32_t n, const double* R, double* y,
                         hot_stream_t stream) {
  if (!ctx || !R || !y) return HOT_E_INVALID;
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (m < 1 || n < 1 || m > kMaxSide || n > kMaxSide) {
    ctx->err = "grid sides out of range";
    return HOT_E_INVALID;
  }
  auto ws = std::make_shared<Workspace>();
  std::string err;
  if (!build_layout({{m, n}}, 0, ctx->tune, ws->lay, err)) {
    ctx->err = err;
    return HOT_E_INVALID;
  }
  hot_status s = ws->alloc_all(ctx);
  if (s != HOT_OK) return s;
  ws->args.solve_pre = ctx->tune.solve_pre;
  hipStream_t st = (hipStream_t)stream;
  HIPCK(hipMemcpyAsync(ws->geo_d, ws->lay.geo.data(), sizeof(PairGeo), hipMemcpyHostToDevice, st));
  HIPCK(hipMemcpyAsync(ws->blocks_d, ws->lay.blocks.data(), ws->lay.blocks.size() * sizeof(PBlock),
                       hipMemcpyHostToDevice, st));
  HIPCK(hipMemcpyAsync(ws->sblocks_d, ws->lay.sblocks.data(),
                       ws->lay.sblocks.size() * sizeof(PBlock), hipMemcpyHostToDevice, st));
  launch_aat_solve(ws->args, 0, (int64_t)m * n, R, st);
  launch_export_y(ws->args, 0, 3 * (int64_t)m * n - 1, y, st);
  HIPCK(hipGetLastError());
  HIPCK(hipStreamSynchronize(st));
  return HOT_OK;
}

hot_status hot_batch_submit(hot_ctx* ctx, const hot_problem* probs, int32_t count,
                            hot_stream_t stream, hot_batch** out) {
  if (!ctx || !probs || !out || count < 1) return HOT_E_INVALID;
  *out = nullptr;
  GroupedBatch gb;
  std::string key;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->err.clear();
    if (hipSetDevice(ctx->device) != hipSuccess) return HOT_E_DEVICE;
    // timed (profiling) solves run the batch as one launch per pass, so each
    // timed slab pass is the whole batch's; otherwise concurrent groups
    const int groups = ctx->profiling ? 1 : ctx->tune.batch_groups;
    key = ws_cache_key(probs, count, groups);
    hot_status s = HOT_OK;
    if (ws_cache_take(ctx, key, gb)) {  // same shapes: validate the problems only
      for (int p = 0; p < count && s == HOT_OK; ++p) {
        s = validate_problem(ctx, &probs[p]);
        if (s == HOT_OK && probs[p].prec != probs[0].prec) {
          ctx->err = "all problems of a batch must use the same precision";
          s = HOT_E_INVALID;
        }
      }
    } else {
      s = make_groups(ctx, probs, count, groups, gb);
    }
    if (s != HOT_OK) return s;
    // order every group after the caller's stream
    hipEvent_t ev;
    HIPCK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIPCK(hipEventRecord(ev, (hipStream_t)stream));
    for (const auto& ws : gb.wss) HIPCK(hipStreamWaitEvent(ws->stream, ev, 0));
    (void)hipEventDestroy(ev);
    std::vector<std::vector<hot_problem>> sub(gb.wss.size());
    for (int p = 0; p < count; ++p) sub[gb.where[p].first].push_back(probs[p]);
    for (size_t g = 0; g < gb.wss.size(); ++g) {
      s = gb.wss[g]->setup(ctx, sub[g].data(), (int)sub[g].size(), gb.wss[g]->stream);
      if (s != HOT_OK) return s;
    }
  }
  int64_t max_it = 1;
  for (int p = 0; p < count; ++p) max_it = std::max<int64_t>(max_it, probs[p].max_iter);
  hot_batch* b = new hot_batch();
  b->ctx = ctx;
  b->gb = std::move(gb);
  b->count = count;
  b->key = key;
  const int64_t max_graphs = max_it * 2 / kGraphIters + 8;
  const int dev = ctx->device;
  b->th = std::thread([b, max_graphs, dev]() {
    (void)hipSetDevice(dev);
    const auto t0 = std::chrono::steady_clock::now();
    hot_ctx tmp;  // private error sink for the worker thread
    b->status = run_concurrent(&tmp, b->gb.wss, max_graphs);
    {
      std::lock_guard<std::mutex> lk(b->ctx->mu);
      if (b->status != HOT_OK) b->ctx->err = tmp.err;
      else
        for (const auto& ws : b->gb.wss) collect_profile(b->ctx, *ws);
    }
    b->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  });
  *out = b;
  return HOT_OK;
}

hot_status hot_batch_wait(hot_batch* b, hot_result* results) {
  if (!b) return HOT_E_INVALID;
  if (b->th.joinable()) b->th.join();
  hot_status s = b->status;
  if (s == HOT_OK && results)
    for (int p = 0; p < b->count; ++p)
      b->gb.wss[b->gb.where[p].first]->fill_result(b->gb.where[p].second, &results[p], b->seconds);
  if (s == HOT_OK) {  // kept for the next batch of these shapes
    std::lock_guard<std::mutex> lk(b->ctx->mu);
    ws_cache_put(b->ctx, b->key, std::move(b->gb));
  }
  delete b;
  return s;
}

}  // extern "C"
