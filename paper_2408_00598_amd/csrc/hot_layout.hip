// Host-side layout of libhot's device buffers (no device code): the launch
// shape of the slab pass (tuned or by rule), the offsets of every per-problem
// array, and the work tables of the slab pass, the pair reduce and the pair
// solve.  Kept apart from the runtime so that the host logic also builds with
// a plain C++ compiler (the sanitizer test builds it with g++).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "hot_internal.h"
#include "hot_runtime.h"

namespace hot {

static int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}
static int ilog2(int v) {
  int r = 0;
  while ((1 << r) < v) ++r;
  return r;
}
static int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// ||c||^2 of the reduced model: n copies of the m x m slab cost and m copies
// of the n x n slab cost, each sum_{p,q} (p-q)^4.
double slab_cost_sq(int L) {
  unsigned __int128 s = 0;
  for (int d = 1; d < L; ++d) {
    unsigned __int128 d4 = (unsigned __int128)d * d * d * d;
    s += 2 * (unsigned __int128)(L - d) * d4;
  }
  return (double)s;
}

int size_class(int64_t v) {
  int c = 0;
  while ((int64_t(1) << (c + 1)) <= v) ++c;
  return c;
}

int64_t Tuning::item_elems_for(int64_t elems, int npairs, int fp32) const {  // launch totals
  auto it = table.find(tune_key(fp32, elems, npairs));
  if (it != table.end()) return it->second.item_elems;
  return std::max<int64_t>(2048, std::min<int64_t>(item_elems, elems / std::max<int64_t>(1, min_items)));
}

int Tuning::unroll_for(int64_t elems, int npairs, int fp32) const {
  auto it = table.find(tune_key(fp32, elems, npairs));
  return it != table.end() ? it->second.unroll : unroll;
}

int Tuning::vec_per_lane_for(int64_t elems, int npairs, int fp32) const {
  auto it = table.find(tune_key(fp32, elems, npairs));
  return it != table.end() ? it->second.vec_per_lane : vec_per_lane;
}

Tuning default_tuning() {
  Tuning t;
  // (what the autotuner picked on every FP32 workload it was run on: items
  // of at most 8192 elements, two 16-byte vectors per lane)
  t.item_elems = 8192;
  t.min_items = 2048;
  t.unroll = 1;
  t.vec_per_lane = 2;
  t.nt_store = 1;
  t.pingpong = 1;
  t.sep_anchor = 0;
  t.small_side = 48;
  t.batch_groups = 2;
  t.fuse = 1;
  t.row_group = 0;
  t.reduce_group = 0;
  t.solve_pre = 1;
  t.fuse_pair = 0;
  return t;
}

size_t Layout::bytes(uint32_t flags) const {
  // sigma re-balancing keeps x_bar and (alpha, beta) of the last restart
  const size_t su = (flags & HOT_FLAG_SIGMA_UPDATE)
                        ? (size_t)state_elems * elem_size + (size_t)tab_off * 8 + 512
                        : 0;
  // widening FP32 streams to FP64 allocates FP64 state buffers (3, and x_bar
  // with sigma re-balancing) while the FP32 ones still exist
  const size_t esc = (fp32 && (flags & HOT_FLAG_ESCALATE))
                         ? (size_t)state_elems * 8 * ((flags & HOT_FLAG_SIGMA_UPDATE) ? 4 : 3)
                         : 0;
  return su + esc + (size_t)state_elems * elem_size * 3 + (size_t)ab_len * 8 + (size_t)rs_len * 8 * 2 +
         (size_t)cp_len * 8 * 2 + (size_t)items.size() * (kKI * 8 + sizeof(SlabItem)) +
         sitems.size() * sizeof(SmallItem) +
         (size_t)arr_len * 8 + (size_t)vec_len * 8 + geo.size() * sizeof(PairGeo) +
         (blocks.size() + sblocks.size()) * sizeof(PBlock) + geo.size() * sizeof(PairCtl) * 2 +
         geo.size() * 5 * sizeof(unsigned) + 4096;
}

bool build_layout(const std::vector<std::pair<int, int>>& shapes, int fp32, const Tuning& tune,
                  Layout& lay, std::string& err, int64_t key_elems, int key_pairs) {
  lay = Layout();
  lay.fp32 = fp32;
  lay.elem_size = fp32 ? 4 : 8;
  const int W = fp32 ? 4 : 2;
  int64_t total = 0;
  for (const auto& sh : shapes) {
    const int m = sh.first, n = sh.second;
    if (m < 1 || n < 1 || m > kMaxSide || n > kMaxSide) {
      err = "grid sides must be in [1, " + std::to_string(kMaxSide) + "]";
      return false;
    }
    total += (int64_t)m * m * n + (int64_t)m * n * n;
  }
  // workgroup size of the slab pass: enough workgroups to fill the chip,
  // never more than item_elems elements each (or the autotuned size for
  // this total)
  const int npairs = key_pairs >= 0 ? key_pairs : (int)shapes.size();
  if (key_elems >= 0) total = key_elems;
  lay.key_elems = total;
  lay.key_pairs = npairs;
  const int64_t item_elems = tune.item_elems_for(total, npairs, fp32);
  int64_t soff = 0, aboff = 0, rsoff = 0, cpoff = 0, moff = 0, voff = 0, taboff = 0;
  int maxvpl = 1;
  // a launch with many row blocks gives each solve wave four slabs and each
  // reduce block four slots, so that fewer blocks repeat the per-pair
  // prologue (256-pair batch: +2% from the solve, +0.5% from the reduce); a
  // few pairs keep one per block for parallelism (128 x 128 alone: -4% with
  // four)
  int64_t rows4 = 0;
  for (const auto& sh : shapes) rows4 += (sh.first + sh.second + 3) / 4;
  // the wave-per-slab pass costs a launch of its own each iteration: worth it
  // only for launches with many small slabs (256-pair batch: ~8,000; a lone
  // 32 x 32 pair, 64 slabs, is 13% faster without it)
  int64_t small_slabs = 0;
  for (const auto& sh : shapes) {
    if (sh.first <= tune.small_side) small_slabs += sh.second;   // F1: n slabs of side m
    if (sh.second <= tune.small_side) small_slabs += sh.first;   // F2: m slabs of side n
  }
  const int small_side = small_slabs >= kMinSmallSlabs ? tune.small_side : 0;
  const int row_group = tune.row_group > 0 ? tune.row_group : (rows4 > 2048 ? 4 : 1);
  for (size_t p = 0; p < shapes.size(); ++p) {
    const int m = shapes[p].first, n = shapes[p].second;
    PairGeo g;
    std::memset(&g, 0, sizeof(g));
    g.m = m;
    g.n = n;
    g.item0 = (int32_t)lay.items.size();
    for (int fam = 0; fam < 2; ++fam) {
      FamGeo& F = g.f[fam];
      F.L = fam == 0 ? m : n;
      F.nslab = fam == 0 ? n : m;
      F.P = (int32_t)round_up(F.L, W);
      const int Q = F.P / W;
      // about two 16-byte vectors per lane per row: short DPP trees for the
      // row sums, few column accumulators per lane
      const int vt = tune.vec_per_lane_for(total, npairs, fp32);
      const int LR = std::min(64, next_pow2((Q + vt - 1) / vt));
      const int vpl = (Q + LR - 1) / LR;
      F.lrs = ilog2(LR);
      F.vpl = vpl;
      maxvpl = std::max(maxvpl, vpl);
      const int step = 8 * (64 / LR);  // rows one workgroup covers per (two-row) step
      const bool small = F.L <= small_side;  // whole slab per wave
      int rows = (int)std::max<int64_t>(1, item_elems / F.P);
      rows = (int)round_up(rows, step);
      if (rows >= F.L || small) rows = F.L;
      F.rpc = rows;
      F.nchunk = (F.L + rows - 1) / rows;
      soff = round_up(soff, 64);
      F.soff = soff;
      soff += (int64_t)F.nslab * F.L * F.P;
      F.aboff = aboff;
      aboff += (int64_t)F.nslab * 2 * F.L;
      F.sumoff = aboff;
      aboff += (int64_t)F.nslab * 2;
      F.xoff = taboff;  // relative to the table region, which follows all pairs
      taboff += 2 * (int64_t)F.L + 1;
      F.rsoff = rsoff;
      rsoff += (int64_t)F.nslab * F.L;
      F.cpoff = cpoff;
      cpoff += (int64_t)F.nslab * F.nchunk * F.L;
      for (int s = 0; s < F.nslab; ++s)
        for (int c = 0; c < F.nchunk; ++c)
          lay.items.push_back(SlabItem{(int32_t)p, fam, s, c, (int32_t)lay.items.size(),
                                       small ? 1 : 0, 0, 0});
      if (small)
        for (int s = 0; s < F.nslab; s += 4)
          lay.sitems.push_back(SmallItem{(int32_t)p, fam, s, std::min(4, F.nslab - s)});
    }
    g.nitem = (int32_t)lay.items.size() - g.item0;
    // reduce row blocks: rows j = 4b..4b+3 of F1 (row j alone when F1 is
    // wide), then the rows k of F2 likewise
    g.f[0].wide = m >= kWideSide ? 1 : 0;
    g.f[1].wide = n >= kWideSide ? 1 : 0;
    g.nb1 = g.f[0].wide ? n : (n + 3) / 4;
    g.nblk = g.nb1 + (g.f[1].wide ? m : (m + 3) / 4);
    g.ns1 = (m + 63) / 64;              // reduce strips over the columns k of rs1
    g.ns2 = (n + 63) / 64;              // reduce strips over the columns j of rs2
    // solve row blocks: slabs 4 spw b .. 4 spw (b + 1) - 1 (the result does
    // not depend on spw)
    g.spw = row_group;
    g.nsblk = (m + n + 4 * g.spw - 1) / (4 * g.spw);
    g.ntj = (n + 31) / 32;              // solve tiles
    g.ntk = (m + 31) / 32;
    g.ipb = (g.nitem + g.nblk - 1) / g.nblk;
    g.blk0 = (int32_t)lay.blocks.size();
    // (the grouping of slots into blocks does not change the result; two
    // slots per reduce block measured best on the 256-pair batch: 133.9
    // solves/s against 133.2 with four and 132.2 with one)
    g.rq = tune.reduce_group > 0 ? tune.reduce_group : (row_group > 1 ? 2 : 1);
    const int rq1 = g.f[0].wide ? 1 : g.rq, rq2 = g.f[1].wide ? 1 : g.rq;
    for (int b = 0; b < (g.nb1 + rq1 - 1) / rq1; ++b)
      lay.blocks.push_back(PBlock{(int32_t)p, b, 0, 0});
    for (int b = 0; b < (g.nblk - g.nb1 + rq2 - 1) / rq2; ++b)
      lay.blocks.push_back(PBlock{(int32_t)p, b, 3, 0});
    for (int b = 0; b < g.ns1; ++b) lay.blocks.push_back(PBlock{(int32_t)p, b, 1, 0});
    for (int b = 0; b < g.ns2; ++b) lay.blocks.push_back(PBlock{(int32_t)p, b, 2, 0});
    g.sblk0 = (int32_t)lay.sblocks.size();
    for (int b = 0; b < g.nsblk; ++b) lay.sblocks.push_back(PBlock{(int32_t)p, b, 0, 0});
    for (int b = 0; b < g.ntj * g.ntk; ++b) lay.sblocks.push_back(PBlock{(int32_t)p, b, 1, 0});
    g.moff = moff;
    moff += 5 * (int64_t)m * n;
    g.voff = voff;
    voff += vec_size(g);
    g.norm_c = std::sqrt((double)n * slab_cost_sq(m) + (double)m * slab_cost_sq(n));
    lay.geo.push_back(g);
  }
  // launch order: items of the block plain-update pass first (the check /
  // restart kernel runs over all of them); kslot keeps each pair's KKT
  // partial slots contiguous
  std::stable_partition(lay.items.begin(), lay.items.end(),
                        [](const SlabItem& it) { return it.small == 0; });
  lay.nbig = 0;
  for (const SlabItem& it : lay.items) lay.nbig += it.small == 0;
  lay.state_elems = round_up(std::max<int64_t>(soff, 64), 64);
  for (PairGeo& g : lay.geo)
    for (int fam = 0; fam < 2; ++fam) g.f[fam].xoff += aboff;
  lay.tab_off = aboff;
  lay.tab_len = taboff;
  lay.ab_len = aboff + taboff;
  lay.rs_len = std::max<int64_t>(rsoff, 1);
  lay.cp_len = std::max<int64_t>(cpoff, 1);
  lay.arr_len = std::max<int64_t>(moff, 1);
  lay.vec_len = std::max<int64_t>(voff, 1);
  lay.maxvpl = maxvpl;
  return true;
}

SlotCaps slot_caps(const Layout& one) {
  SlotCaps c;
  c.state = round_up(one.state_elems, 64);
  c.ab = round_up(one.ab_len, 64);
  c.rs = round_up(one.rs_len, 64);
  c.cp = round_up(one.cp_len, 64);
  c.arr = round_up(one.arr_len, 64);
  c.vec = round_up(one.vec_len, 64);
  c.items = round_up((int64_t)one.items.size(), 8);  // (kitem ranges stay 64-byte aligned)
  c.blocks = (int64_t)one.blocks.size();
  c.sblocks = (int64_t)one.sblocks.size();
  return c;
}

bool slot_fits(const Layout& one, const SlotCaps& c) {
  return one.geo.size() == 1 && one.sitems.empty() && one.state_elems <= c.state &&
         one.ab_len <= c.ab && one.rs_len <= c.rs && one.cp_len <= c.cp && one.arr_len <= c.arr &&
         one.vec_len <= c.vec && (int64_t)one.items.size() <= c.items &&
         (int64_t)one.blocks.size() <= c.blocks && (int64_t)one.sblocks.size() <= c.sblocks;
}

void place_in_slot(const Layout& one, int s, const SlotCaps& c, PairGeo& g,
                   std::vector<SlabItem>& items, std::vector<PBlock>& blocks,
                   std::vector<PBlock>& sblocks) {
  g = one.geo[0];
  g.item0 += (int32_t)(s * c.items);
  g.blk0 += (int32_t)(s * c.blocks);
  g.sblk0 += (int32_t)(s * c.sblocks);
  for (int fam = 0; fam < 2; ++fam) {
    FamGeo& F = g.f[fam];
    F.soff += s * c.state;
    F.aboff += s * c.ab;
    F.sumoff += s * c.ab;
    F.xoff += s * c.ab;
    F.rsoff += s * c.rs;
    F.cpoff += s * c.cp;
  }
  g.moff += s * c.arr;
  g.voff += s * c.vec;
  items = one.items;
  for (SlabItem& it : items) {
    it.pair = s;
    it.kslot += (int32_t)(s * c.items);
  }
  blocks = one.blocks;
  for (PBlock& b : blocks) b.pair = s;
  sblocks = one.sblocks;
  for (PBlock& b : sblocks) b.pair = s;
}

void group_layout(const SlotCaps& c, int K, int fp32, Layout& lay) {
  lay = Layout();
  lay.fp32 = fp32;
  lay.elem_size = fp32 ? 4 : 8;
  PairGeo zero;
  std::memset(&zero, 0, sizeof(zero));
  lay.geo.assign(K, zero);
  lay.items.assign(K * c.items, SlabItem{0, 0, 0, 0, 0, 0, 0, 0});
  lay.nbig = (int64_t)lay.items.size();
  lay.blocks.assign(K * c.blocks, PBlock{0, 0, 0, 0});
  lay.sblocks.assign(K * c.sblocks, PBlock{0, 0, 0, 0});
  lay.state_elems = K * c.state;
  lay.ab_len = K * c.ab;
  lay.tab_off = lay.ab_len;  // (sigma re-balancing keeps a copy of all of it)
  lay.tab_len = 0;
  lay.rs_len = K * c.rs;
  lay.cp_len = K * c.cp;
  lay.arr_len = K * c.arr;
  lay.vec_len = K * c.vec;
  lay.maxvpl = 1;
}

// Lanes of every family for streams of another precision on the same pitches,
// offsets and row chunks: when a solve's FP32 state is widened to FP64 in
// place, the elements per 16-byte vector change and the buffer geometry does
// not (an FP32 pitch is a multiple of 4 elements, so also of 2).
void relane_layout(Layout& lay, int fp32, const Tuning& tune) {
  const int W = fp32 ? 4 : 2;
  int maxvpl = 1;
  for (PairGeo& g : lay.geo)
    for (int fam = 0; fam < 2; ++fam) {
      FamGeo& F = g.f[fam];
      const int Q = F.P / W;
      const int vt = tune.vec_per_lane_for(lay.key_elems, lay.key_pairs, fp32);
      const int LR = std::min(64, next_pow2((Q + vt - 1) / vt));
      F.lrs = ilog2(LR);
      F.vpl = (Q + LR - 1) / LR;
      maxvpl = std::max(maxvpl, F.vpl);
    }
  lay.fp32 = fp32;
  lay.elem_size = fp32 ? 4 : 8;
  lay.maxvpl = maxvpl;
}

}  // namespace hot
