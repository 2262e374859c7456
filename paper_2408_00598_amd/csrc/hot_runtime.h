// Host-side runtime structures of libhot (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/hot.h"
#include "hot_internal.h"

namespace hot {

// Iterations captured per graph launch (even: control blocks alternate parity).
constexpr int kGraphIters = 20;

struct Tuning {
  int64_t item_elems;   // largest target of elements per slab-pass workgroup
  int64_t min_items;    // aim for at least this many slab-pass workgroups per launch
  int unroll;           // rows loaded ahead per wave (1 or 2)
  int vec_per_lane;     // target 16-byte vectors per lane per slab row (2 or 4)
  int nt_store;         // non-temporal stores of the new state
  int pingpong;         // never update the state in place (read one buffer, write the other)
  int sep_anchor;       // autotuner runs: stream a zero anchor from its own buffer, as
                        // every pass after the first restart does
  int small_side;       // families with slab side <= this run plain-update passes
                        // wave-per-slab (whole slab per wave, no block barriers)
  int batch_groups;     // concurrent groups (streams) a batch is split into
  int fuse;             // default for one slab kernel for every pass
  int row_group;        // > 0: slabs per solve wave and slots per reduce block (else by launch size)
  int reduce_group;     // > 0: slots per reduce block (overrides row_group for the reduce)
  int solve_pre;        // 1: the solve issues its decision-free loads before the decision, 0: after
  int fuse_pair;        // 1: reduce and solve in one launch (k_pair_fused)
  // autotuned launch shapes, keyed by (precision, floor(log2) of the
  // launch's flow elements, floor(log2) of its pair count): one large pair
  // and a batch of small ones of the same total get separate entries
  struct Choice {
    int64_t item_elems;
    int unroll;
    int vec_per_lane;
  };
  typedef std::tuple<int, int, int> Key;
  std::map<Key, Choice> table;
  // elements per slab-pass workgroup for a launch of `npairs` problems over
  // `elems` flow elements
  int64_t item_elems_for(int64_t elems, int npairs, int fp32) const;
  int unroll_for(int64_t elems, int npairs, int fp32) const;
  int vec_per_lane_for(int64_t elems, int npairs, int fp32) const;
};
Tuning default_tuning();
int size_class(int64_t v);  // floor(log2(v)) for v >= 1
// ||c||^2 of one slab's cost on the uniform grid: sum_{p,q} (p-q)^4 (exact)
double slab_cost_sq(int L);
inline Tuning::Key tune_key(int fp32, int64_t elems, int npairs) {
  return Tuning::Key{fp32, size_class(elems), size_class(npairs)};
}

struct LaunchArgs {
  const SlabItem* items = nullptr;
  int nitems = 0;
  int nbig = 0;                       // block items whose plain passes use the block kernel
  const SmallItem* sitems = nullptr;  // wave-per-slab items
  int nsitems = 0;
  const PBlock* blocks = nullptr;   // reduce blocks
  int nblocks = 0;
  const PBlock* sblocks = nullptr;  // solve blocks
  int nsblocks = 0;
  const PairGeo* geo = nullptr;
  PairCtl* ctl[2] = {nullptr, nullptr};
  void* sb[3] = {nullptr, nullptr, nullptr};
  double* ab = nullptr;
  double* rowsum[2] = {nullptr, nullptr};
  double* colpart[2] = {nullptr, nullptr};
  double* kitem = nullptr;
  double* arr = nullptr;
  double* vec = nullptr;
  int fp32 = 0;
  int maxvpl = 1;
  int unroll = 1;  // rows loaded ahead per wave in the plain update pass
  int nt_store = 0;   // non-temporal stores of the new state
  int coord = 0;      // some pair has non-uniform bins: slab passes read positions
  int su = 0;         // some pair re-balances sigma at restarts
  int fuse = 0;       // one slab kernel for plain, check and restart passes
  int solve_pre = 1;  // the solve issues its decision-free loads before the decision
  int fuse_pair = 0;  // reduce and solve in one launch (k_pair_fused)
  unsigned* sync[2] = {nullptr, nullptr};  // per pair (reduce count, solve count), by parity
  unsigned* lost = nullptr;                // per pair: a fused wait ran out
  void* sbx = nullptr;      // x_bar of the last restart (sigma re-balancing), else null
  double* abY = nullptr;    // alpha / beta of the last restart (sigma re-balancing)
  unsigned long long* bytes_ctr = nullptr;  // algorithmic stream bytes of slab passes
};

struct Layout {
  int fp32 = 0;
  int elem_size = 8;
  std::vector<PairGeo> geo;
  std::vector<SlabItem> items;      // block items; the first nbig are not small
  int64_t nbig = 0;
  std::vector<SmallItem> sitems;    // wave-per-slab items
  std::vector<PBlock> blocks;
  std::vector<PBlock> sblocks;
  int64_t state_elems = 0, ab_len = 0, rs_len = 0, cp_len = 0, arr_len = 0, vec_len = 0;
  int64_t tab_off = 0, tab_len = 0;  // cost tables of every family, inside ab
  int maxvpl = 1;
  int64_t key_elems = 0;  // launch totals the shape was looked up under
  int key_pairs = 0;
  size_t bytes(uint32_t flags = 0) const;  // device bytes; flags: HOT_FLAG_* of the problems
};

// key_elems / key_pairs >= 0: look the launch shape up under these totals
// (a group of a larger batch uses the batch's entry)
bool build_layout(const std::vector<std::pair<int, int>>& shapes, int fp32, const Tuning& tune,
                  Layout& lay, std::string& err, int64_t key_elems = -1, int key_pairs = -1);
void relane_layout(Layout& lay, int fp32, const Tuning& tune);

// Slots of a shared server group: every slot holds one problem at fixed
// bases in the group's arrays, with the geometry and work tables its own
// single-problem layout gives it (so its kernels and reduction order are
// those of a solve alone).  A slot's capacities are the array lengths and
// table sizes of the single-problem layout of the group's largest shape.
struct SlotCaps {
  int64_t state = 0, ab = 0, rs = 0, cp = 0, arr = 0, vec = 0;
  int64_t items = 0, blocks = 0, sblocks = 0;
};
SlotCaps slot_caps(const Layout& one);
bool slot_fits(const Layout& one, const SlotCaps& c);
// the single problem of `one` placed in slot s: its geometry with every
// offset moved to the slot's bases, and its work-table entries
void place_in_slot(const Layout& one, int s, const SlotCaps& c, PairGeo& g,
                   std::vector<SlabItem>& items, std::vector<PBlock>& blocks,
                   std::vector<PBlock>& sblocks);
// arrays and tables of a group of K slots (geometry zero until slots fill)
void group_layout(const SlotCaps& c, int K, int fp32, Layout& lay);

// Tracks the best relative KKT of a solve for HOT_FLAG_ESCALATE.
struct StallWatch {
  double best = 0.0;
  int64_t it_best = 0;
  bool stalled(const PairCtl& c);
};

struct Workspace {
  int device = 0;
  Layout lay;
  LaunchArgs args;
  std::vector<void*> allocs;
  void* sb[3] = {nullptr, nullptr, nullptr};
  double* ab = nullptr;
  double* rowsum[2] = {nullptr, nullptr};
  double* colpart[2] = {nullptr, nullptr};
  double* kitem = nullptr;
  double* arr = nullptr;
  double* vec = nullptr;
  SlabItem* items_d = nullptr;
  SmallItem* sitems_d = nullptr;
  PBlock* blocks_d = nullptr;
  PBlock* sblocks_d = nullptr;
  PairGeo* geo_d = nullptr;
  PairCtl* ctl_d = nullptr;
  double* stats_d = nullptr;
  void* ptrs_d = nullptr;
  PairCtl* host_ctl = nullptr;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  unsigned long long* bytes_ctr = nullptr;
  unsigned* sync_d = nullptr;    // counters of the fused reduce + solve (5 per problem)
  std::vector<double> tab_host;  // cost tables uploaded by setup
  // launch tables restricted to the problems still running (a batch whose
  // problems have mostly stopped launches only the rest): device copies,
  // pinned host staging, problems the current tables cover, retired graphs
  SlabItem* items_c = nullptr;
  SmallItem* sitems_c = nullptr;
  PBlock* blocks_c = nullptr;
  PBlock* sblocks_c = nullptr;
  void* stage_h = nullptr;
  hipEvent_t stage_ev = nullptr;  // recorded after the last upload from stage_h
  bool stage_pending = false;
  int launch_pairs = 0;
  std::vector<std::pair<hipGraph_t, hipGraphExec_t>> retired;
  hot_status compact(hot_ctx* ctx, const PairCtl* hc);
  void restore_tables();
  void drop_retired();
  int graph_variant = 0;         // slab kernel variant the graph was captured with
  void* sbx = nullptr;           // sigma re-balancing buffers, allocated on first use
  double* abY = nullptr;
  // profiling (events around every slab pass; direct launches)
  bool profile = false;
  double prof_seconds = 0.0;
  int64_t prof_launches = 0;
  int64_t iterations_launched = 0;

  // no-alloc solves: every device buffer is carved out of a caller-given
  // arena (256-byte aligned) instead of hipMalloc, and the control blocks are
  // read back into host_ctl_vec (no pinned allocation)
  char* arena = nullptr;
  size_t arena_bytes = 0, arena_used = 0;
  std::vector<PairCtl> host_ctl_vec;
  // test hook (HOT_TEST_NAN_AFTER): after this many graphs, write a NaN into
  // the first flow element of every state buffer; < 0 off
  int64_t nan_after = -1;

  ~Workspace();
  void release();
  hot_status device_buffer(hot_ctx* ctx, void** p, size_t bytes);
  hot_status alloc_all(hot_ctx* ctx);
  hot_status setup(hot_ctx* ctx, const hot_problem* probs, int count, hipStream_t st);
  // shared server groups: set up problem `pr` in slot s (geometry g from
  // place_in_slot; the stream is idle), and install the work tables of the
  // occupied slots (re-captured into the graph on the next ensure_graph)
  bool group = false;
  SlotCaps caps;
  hot_status setup_slot(hot_ctx* ctx, int s, const hot_problem& pr, const PairGeo& g,
                        hipStream_t st);
  // a new group: every slot's geometry zero (covering no item), control
  // blocks and fused-launch counters cleared, before any slot is used
  hot_status init_group(hot_ctx* ctx, hipStream_t st);
  hot_status set_tables(hot_ctx* ctx, const std::vector<SlabItem>& items,
                        const std::vector<PBlock>& blocks, const std::vector<PBlock>& sblocks,
                        int coord, int su, hipStream_t st);
  hot_status run(hot_ctx* ctx, hipStream_t st, int64_t max_graphs,
                 StallWatch* watch = nullptr);
  // direct launches on st, a stream synchronisation per quantum, no graph,
  // event or pinned buffer (the no-alloc entry point)
  hot_status run_direct(hot_ctx* ctx, hipStream_t st, int64_t max_graphs);
  // Non-blocking pieces of run() for the server: capture the graph once,
  // launch one graph (kGraphIters iterations) + status copy + event.
  hot_status ensure_graph(hot_ctx* ctx, hipStream_t st);
  hipError_t launch_quantum(hipStream_t st);
  hipError_t poison_state(hipStream_t st);
  // FP32 -> FP64 streams in place (the stream is idle): the state buffers are
  // widened exactly, the lanes re-derived, the graph re-captured
  hot_status escalate(hot_ctx* ctx, hipStream_t st);
  int32_t escalated_at = 0;  // iteration count at the widening, 0 if none
  // after the last graph: the feasibility error of every problem's final
  // iterate into ctl[0] (on st; copy the control blocks after it)
  hipError_t finalize(hipStream_t st);
  hipEvent_t quantum_event = nullptr;
  hot_status run_profiled(hot_ctx* ctx, hipStream_t st, int64_t max_graphs,
                          StallWatch* watch = nullptr);
  void fill_result(int p, hot_result* r, double seconds) const;
};

hot_status make_workspace(hot_ctx* ctx, const hot_problem* probs, int count,
                          std::shared_ptr<Workspace>& out, int64_t key_elems = -1,
                          int key_pairs = -1);

// A batch split into groups of problems (balanced by flow elements), one
// workspace and stream each, iterated concurrently so that one group's
// latency-bound pair kernels overlap another group's streaming slab pass.
struct GroupedBatch {
  std::vector<std::shared_ptr<Workspace>> wss;
  std::vector<std::pair<int, int>> where;  // problem -> (group, index in group)
};
hot_status make_groups(hot_ctx* ctx, const hot_problem* probs, int count, int groups,
                       GroupedBatch& gb);
hot_status run_concurrent(hot_ctx* ctx, const std::vector<std::shared_ptr<Workspace>>& wss,
                          int64_t max_graphs);

// Workspace cache of a context (caller holds ctx->mu): the key of a call,
// take a matching entry, keep a finished one, drop all.
std::string ws_cache_key(const hot_problem* probs, int count, int groups);
bool ws_cache_take(hot_ctx* ctx, const std::string& key, GroupedBatch& gb);
void ws_cache_put(hot_ctx* ctx, const std::string& key, GroupedBatch&& gb);
void ws_cache_clear(hot_ctx* ctx);

}  // namespace hot

struct hot_ctx {
  int device = 0;
  std::mutex mu;
  std::string err;
  hot::Tuning tune = hot::default_tuning();
  int64_t nan_after = -1;  // HOT_TEST_NAN_AFTER (failure-path tests only)
  // device address of this device's no-alloc scratch array (null if its
  // set-up failed; scratch_err says why)
  void* scratch = nullptr;
  std::string scratch_err;
  // measurement counters (hot_ctx_profile_read)
  bool profiling = false;
  double prof_seconds = 0, prof_launches = 0, prof_bytes = 0, iters_launched = 0;
  // plan-recovery scratch: grows to the largest recovery seen, kept until the
  // context is destroyed; rec_mu is held for the whole of a recovery
  std::mutex rec_mu;
  void* rec_buf = nullptr;
  size_t rec_bytes = 0;
  // Workspaces of finished solves and batches, kept for the next call with
  // the same shapes, precision and grouping (most recent first; a few
  // entries and a byte cap; cleared when the launch-shape tuning changes).
  // A reused workspace is set up afresh (control blocks, state, tables);
  // only its allocation and captured graph are saved.
  struct CachedWs {
    std::string key;
    hot::GroupedBatch gb;
    size_t bytes = 0;
  };
  std::list<CachedWs> ws_cache;
  size_t ws_cache_bytes = 0;
  ~hot_ctx() {
    if (rec_buf) (void)hipFree(rec_buf);
  }
};

struct hot_solution {
  std::shared_ptr<hot::Workspace> ws;
  int pair = 0;
  int32_t m = 0, n = 0;
  int prec = 0;
};
