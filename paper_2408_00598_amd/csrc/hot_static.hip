// hot_solve_noalloc: a solve that allocates no memory, for callers that cannot
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  Every device buffer of the solve (flow state, sums, dual
// vectors, launch tables, control blocks) is carved out of one file-scope
// device array of kScratchBytes; the iteration is launched directly on the
// caller's stream (no graph, no event, no pinned host buffer) and the control
// blocks are read back into host memory between quanta.  The kernels, their
// launch shapes and their order are those of hot_solve, so the results are
// the same bit for bit.
//
// Each device the library runs on holds its own copy of the array until the
// process ends.  Its address on a device is taken once, with that device
// current, when the first context on it is created (hipGetSymbolAddress);
// host code uses that address only, never the array's name.  All calls on one
// device share the array: calls that overlap on a device (two contexts on the
// same device used from two threads) race and must be serialised by the
// caller; calls on one context are serialised by its mutex.
#include <hip/hip_runtime.h>

#include <chrono>
#include <mutex>
#include <string>

#include "../../include/hot.h"
#include "hot_internal.h"
#include "hot_runtime.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};
std::string g_scratch_err[kMaxDevices];

}  // namespace

namespace hot {

void launch_export(const LaunchArgs& a, int par, int pair, int64_t N, double* xbar,
                   double* zbar, double* sout, hipStream_t st, double* s0out = nullptr);
void launch_export_y(const LaunchArgs& a, int pair, int64_t M3, double* y, hipStream_t st);
hot_status validate_problem_public(hot_ctx* ctx, const hot_problem* p);

// Address of the scratch array on `device` (the caller has made it current);
// taken once per device, null with `err` set if that failed.
void* static_scratch_init(int device, std::string& err) {
  if (device < 0 || device >= kMaxDevices) {
    err = "device index beyond the no-alloc entry point's table";
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_done[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      g_scratch_err[device] = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    }
    g_scratch_ptr[device] = p;
    g_scratch_done[device] = true;
  }
  err = g_scratch_err[device];
  return g_scratch_ptr[device];
}

}  // namespace hot

using namespace hot;

#define HIPCK_NA(expr)                                                     \
  do {                                                                     \
    hipError_t e_ = (expr);                                                \
    if (e_ != hipSuccess) {                                                \
      ctx->err = std::string(#expr) + ": " + hipGetErrorString(e_);        \
      return HOT_E_DEVICE;                                                 \
    }                                                                      \
  } while (0)

extern "C" {

size_t hot_noalloc_capacity(void) { return kScratchBytes; }

hot_status hot_solve_noalloc(hot_ctx* ctx, const hot_problem* prob, hot_stream_t stream,
                             double* xbar, double* ybar, hot_result* res) {
  if (!ctx || !res) return HOT_E_INVALID;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->err.clear();
  if (!ctx->scratch) {
    ctx->err = "no-alloc scratch unavailable: " + ctx->scratch_err;
    return HOT_E_DEVICE;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return HOT_E_DEVICE;
  const auto t0 = std::chrono::steady_clock::now();
  hot_status s = validate_problem_public(ctx, prob);
  if (s != HOT_OK) return s;
  // the layout hot_solve would use (same tuning), carved out of the array
  Workspace ws;
  std::string err;
  if (!build_layout({{prob->m, prob->n}}, prob->prec == HOT_FP32_STREAM, ctx->tune, ws.lay,
                    err)) {
    ctx->err = err;
    return HOT_E_INVALID;
  }
  ws.device = ctx->device;
  ws.arena = (char*)ctx->scratch;
  ws.arena_bytes = kScratchBytes;
  if ((s = ws.alloc_all(ctx)) != HOT_OK) return s;
  {
    const int64_t total = (int64_t)prob->m * prob->m * prob->n + (int64_t)prob->m * prob->n * prob->n;
    ws.args.unroll = ctx->tune.unroll_for(total, 1, prob->prec == HOT_FP32_STREAM);
  }
  ws.args.nt_store = ctx->tune.nt_store;
  ws.args.fuse = ctx->tune.fuse;
  ws.args.solve_pre = ctx->tune.solve_pre;
  ws.args.bytes_ctr = nullptr;
  hipStream_t st = (hipStream_t)stream;
  ws.stream = st;
  ws.own_stream = false;
  if ((s = ws.setup(ctx, prob, 1, st)) != HOT_OK) return s;
  const int64_t max_graphs = (int64_t)prob->max_iter * 2 / kGraphIters + 8;
  if ((s = ws.run_direct(ctx, st, max_graphs)) != HOT_OK) return s;
  // after whole quanta the latest control blocks are ctl[0]
  const int64_t m = prob->m, n = prob->n;
  if (xbar) launch_export(ws.args, 0, 0, m * m * n + m * n * n, xbar, nullptr, nullptr, st);
  if (ybar) launch_export_y(ws.args, 0, 3 * m * n - 1, ybar, st);
  HIPCK_NA(hipGetLastError());
  HIPCK_NA(hipMemcpyAsync(ws.host_ctl, ws.ctl_d, sizeof(PairCtl), hipMemcpyDeviceToHost, st));
  HIPCK_NA(hipStreamSynchronize(st));
  const double secs =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  ws.fill_result(0, res, secs);
  return (hot_status)res->status;
}

}  // extern "C"
