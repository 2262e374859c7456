// Host-side check of libhot's buffer layout (build_layout), built with
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_sanitizers.py.
// For many shapes, batches and launch tunings it verifies that every slab's
// rows are covered by exactly one slab-pass item, that the per-problem
// ranges of every device array lie inside the array and do not overlap, and
// that the reduce and solve tables cover each problem's rows.  Exits 1 on
// the first violation (the sanitizers abort on memory or UB errors).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <utility>
#include <vector>

#include "hot_internal.h"
#include "hot_runtime.h"

using namespace hot;

static int fails = 0;
#define CHECK(c, ...)                                     \
  do {                                                    \
    if (!(c)) {                                           \
      std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      std::fprintf(stderr, __VA_ARGS__);                  \
      std::fprintf(stderr, "\n");                         \
      ++fails;                                            \
      return;                                             \
    }                                                     \
  } while (0)

struct Range {
  int64_t lo, hi;
};

static bool disjoint(std::vector<Range> v) {
  std::sort(v.begin(), v.end(), [](const Range& a, const Range& b) { return a.lo < b.lo; });
  for (size_t q = 1; q < v.size(); ++q)
    if (v[q].lo < v[q - 1].hi) return false;
  return true;
}

static void check(const std::vector<std::pair<int, int>>& shapes, int fp32, const Tuning& tune) {
  Layout lay;
  std::string err;
  CHECK(build_layout(shapes, fp32, tune, lay, err), "build_layout failed: %s", err.c_str());
  CHECK(lay.geo.size() == shapes.size(), "pair count");
  CHECK(lay.bytes(0) > 0 && lay.bytes(HOT_FLAG_SIGMA_UPDATE) > lay.bytes(0), "bytes");
  std::vector<Range> st, abr, rs, cp, mr, vr;
  for (size_t p = 0; p < lay.geo.size(); ++p) {
    const PairGeo& g = lay.geo[p];
    CHECK(g.m == shapes[p].first && g.n == shapes[p].second, "shape");
    mr.push_back({g.moff, g.moff + 5 * (int64_t)g.m * g.n});
    vr.push_back({g.voff, g.voff + vec_size(g)});
    for (int fam = 0; fam < 2; ++fam) {
      const FamGeo& F = g.f[fam];
      CHECK(F.L == (fam == 0 ? g.m : g.n) && F.nslab == (fam == 0 ? g.n : g.m), "family sides");
      CHECK(F.P >= F.L && F.P % (fp32 ? 4 : 2) == 0 && F.soff % 64 == 0, "pitch / alignment");
      CHECK(F.rpc >= 1 && F.nchunk == (F.L + F.rpc - 1) / F.rpc, "chunks");
      CHECK(F.vpl >= 1 && F.vpl <= lay.maxvpl && (1 << F.lrs) <= 64, "lanes");
      st.push_back({F.soff, F.soff + (int64_t)F.nslab * F.L * F.P});
      abr.push_back({F.aboff, F.aboff + (int64_t)F.nslab * 2 * F.L});
      abr.push_back({F.sumoff, F.sumoff + (int64_t)F.nslab * 2});
      abr.push_back({F.xoff, F.xoff + 2 * (int64_t)F.L + 1});
      rs.push_back({F.rsoff, F.rsoff + (int64_t)F.nslab * F.L});
      cp.push_back({F.cpoff, F.cpoff + (int64_t)F.nslab * F.nchunk * F.L});
    }
  }
  for (const auto* v : {&st, &abr, &rs, &cp, &mr, &vr}) CHECK(disjoint(*v), "overlapping ranges");
  for (const Range& r : st) CHECK(r.lo >= 0 && r.hi <= lay.state_elems, "state range");
  for (const Range& r : abr) CHECK(r.lo >= 0 && r.hi <= lay.ab_len, "alpha/beta range");
  for (const Range& r : rs) CHECK(r.lo >= 0 && r.hi <= lay.rs_len, "row-sum range");
  for (const Range& r : cp) CHECK(r.lo >= 0 && r.hi <= lay.cp_len, "column-partial range");
  for (const Range& r : mr) CHECK(r.lo >= 0 && r.hi <= lay.arr_len, "M-array range");
  for (const Range& r : vr) CHECK(r.lo >= 0 && r.hi <= lay.vec_len, "vector range");
  // slab-pass items: every (pair, family, slab, chunk) exactly once; kslots a
  // permutation; the first nbig items are the non-small ones
  std::vector<std::vector<int>> seen(lay.geo.size());
  for (size_t p = 0; p < lay.geo.size(); ++p) {
    const PairGeo& g = lay.geo[p];
    CHECK(g.item0 >= 0 && g.nitem >= 0 && g.item0 + g.nitem <= (int)lay.items.size(), "item range");
    seen[p].assign(g.nitem, 0);
  }
  std::vector<int> slot(lay.items.size(), 0);
  for (size_t q = 0; q < lay.items.size(); ++q) {
    const SlabItem& it = lay.items[q];
    CHECK(it.pair >= 0 && it.pair < (int)lay.geo.size(), "item pair");
    const PairGeo& g = lay.geo[it.pair];
    const FamGeo& F = g.f[it.fam];
    CHECK(it.slab >= 0 && it.slab < F.nslab && it.chunk >= 0 && it.chunk < F.nchunk, "item index");
    CHECK(it.kslot >= g.item0 && it.kslot < g.item0 + g.nitem, "kslot range");
    CHECK(++slot[it.kslot] == 1, "kslot repeated");
    const int local = (it.fam == 0 ? 0 : g.f[0].nslab * g.f[0].nchunk) + it.slab * F.nchunk + it.chunk;
    CHECK(local < g.nitem && ++seen[it.pair][local] == 1, "item repeated");
    CHECK((q < (size_t)lay.nbig) == (it.small == 0), "block items first");
  }
  for (size_t p = 0; p < lay.geo.size(); ++p)
    for (int v : seen[p]) CHECK(v == 1, "slab chunk not covered");
  // wave-per-slab items cover exactly the small slabs
  for (const SmallItem& si : lay.sitems) {
    const FamGeo& F = lay.geo[si.pair].f[si.fam];
    CHECK(si.slab0 >= 0 && si.nslab >= 1 && si.nslab <= 4 && si.slab0 + si.nslab <= F.nslab,
          "small item");
    CHECK(F.nchunk == 1, "small slab in one chunk");
  }
  // reduce and solve tables: per pair, the counts the kernels assume
  std::vector<int> nred(lay.geo.size(), 0), nsol(lay.geo.size(), 0);
  for (const PBlock& b : lay.blocks) {
    CHECK(b.pair >= 0 && b.pair < (int)lay.geo.size() && b.kind >= 0 && b.kind <= 3, "reduce block");
    ++nred[b.pair];
  }
  for (const PBlock& b : lay.sblocks) {
    CHECK(b.pair >= 0 && b.pair < (int)lay.geo.size() && (b.kind == 0 || b.kind == 1), "solve block");
    ++nsol[b.pair];
  }
  for (size_t p = 0; p < lay.geo.size(); ++p) {
    const PairGeo& g = lay.geo[p];
    CHECK(g.nsblk * 4 * g.spw >= g.m + g.n && nsol[p] == g.nsblk + g.ntj * g.ntk, "solve blocks");
    CHECK(g.ntj * 32 >= g.n && g.ntk * 32 >= g.m, "solve tiles");
    CHECK(nred[p] >= g.ns1 + g.ns2 + 1, "reduce blocks");
    // the fused reduce + solve waits for exactly these counts
    CHECK(nred[p] == reduce_blocks_of(g) && nsol[p] == solve_blocks_of(g), "fused counts");
  }
}

// A shared server group: problems placed in slots of the class's capacity
// keep their own geometry, lie inside their slot's ranges and never overlap
// another slot.
static void check_group(int side, int fp32, const Tuning& tune) {
  Layout cap, grp;
  std::string err;
  CHECK(build_layout({{side, side}}, fp32, tune, cap, err), "class layout");
  const SlotCaps c = slot_caps(cap);
  const int K = 5;
  group_layout(c, K, fp32, grp);
  CHECK(grp.state_elems == K * c.state && grp.ab_len == K * c.ab &&
            (int64_t)grp.items.size() == K * c.items,
        "group capacities");
  CHECK(c.state % 64 == 0 && c.ab % 64 == 0 && c.items % 8 == 0, "slot alignment");
  // a slot not yet used covers no item (the finalize pass visits every slot)
  for (const PairGeo& z : grp.geo) CHECK(z.item0 == 0 && z.nitem == 0, "empty slot geometry");
  const std::pair<int, int> shapes[] = {{side, side}, {side / 2 + 1, side}, {side, 3},
                                        {1, 1}, {side - 1, side / 3 + 1}};
  std::vector<Range> st, abr, rs, cp, mr, vr, it;
  int placed = 0;
  for (int s = 0; s < K; ++s) {
    Layout one;
    CHECK(build_layout({shapes[s]}, fp32, tune, one, err), "slot layout");
    if (!slot_fits(one, c)) continue;  // (runs alone instead)
    PairGeo g;
    std::vector<SlabItem> items;
    std::vector<PBlock> blocks, sblocks;
    place_in_slot(one, s, c, g, items, blocks, sblocks);
    ++placed;
    const PairGeo& g0 = one.geo[0];
    CHECK(g.m == g0.m && g.n == g0.n && g.nitem == g0.nitem && g.nblk == g0.nblk &&
              reduce_blocks_of(g) == (int)blocks.size() && solve_blocks_of(g) == (int)sblocks.size(),
          "slot geometry");
    for (const SlabItem& x : items)
      CHECK(x.pair == s && x.kslot >= g.item0 && x.kslot < g.item0 + g.nitem &&
                x.kslot < (s + 1) * c.items,
            "slot item");
    for (const PBlock& b : blocks) CHECK(b.pair == s, "slot reduce block");
    for (const PBlock& b : sblocks) CHECK(b.pair == s, "slot solve block");
    it.push_back({g.item0, g.item0 + g.nitem});
    mr.push_back({g.moff, g.moff + 5 * (int64_t)g.m * g.n});
    vr.push_back({g.voff, g.voff + vec_size(g)});
    for (int fam = 0; fam < 2; ++fam) {
      const FamGeo& F = g.f[fam];
      const FamGeo& F0 = g0.f[fam];
      CHECK(F.L == F0.L && F.P == F0.P && F.rpc == F0.rpc && F.nchunk == F0.nchunk &&
                F.vpl == F0.vpl && F.lrs == F0.lrs && F.soff % 64 == 0,
            "slot family geometry");
      st.push_back({F.soff, F.soff + (int64_t)F.nslab * F.L * F.P});
      abr.push_back({F.aboff, F.aboff + (int64_t)F.nslab * 2 * F.L});
      abr.push_back({F.sumoff, F.sumoff + (int64_t)F.nslab * 2});
      abr.push_back({F.xoff, F.xoff + 2 * (int64_t)F.L + 1});
      rs.push_back({F.rsoff, F.rsoff + (int64_t)F.nslab * F.L});
      cp.push_back({F.cpoff, F.cpoff + (int64_t)F.nslab * F.nchunk * F.L});
      CHECK(F.soff >= s * c.state && F.soff + (int64_t)F.nslab * F.L * F.P <= (s + 1) * c.state,
            "slot state range");
      CHECK(F.xoff + 2 * (int64_t)F.L + 1 <= (s + 1) * c.ab && F.aboff >= s * c.ab,
            "slot alpha/beta range");
      CHECK(F.cpoff + (int64_t)F.nslab * F.nchunk * F.L <= (s + 1) * c.cp, "slot partial range");
    }
  }
  CHECK(placed >= 4, "only %d of %d shapes fit a slot of side %d", placed, K, side);
  for (const auto* v : {&st, &abr, &rs, &cp, &mr, &vr, &it}) CHECK(disjoint(*v), "slots overlap");
  for (const Range& r : st) CHECK(r.hi <= grp.state_elems, "group state range");
  for (const Range& r : mr) CHECK(r.hi <= grp.arr_len, "group M-array range");
  for (const Range& r : vr) CHECK(r.hi <= grp.vec_len, "group vector range");
}

int main() {
  std::vector<std::pair<int, int>> sides = {{1, 1},   {1, 2},   {2, 1},    {3, 17},   {17, 3},
                                            {32, 32}, {48, 48}, {65, 33},  {100, 3},  {128, 128},
                                            {255, 257}, {256, 256}, {512, 512}, {1024, 48},
                                            {48, 1024}, {1024, 1024}};
  for (int fp32 = 0; fp32 < 2; ++fp32)
    for (int variant = 0; variant < 4; ++variant) {
      Tuning t = default_tuning();
      if (variant == 1) { t.item_elems = 2048; t.unroll = 2; t.vec_per_lane = 2; }
      if (variant == 2) { t.item_elems = 131072; t.vec_per_lane = 8; t.small_side = 0; }
      if (variant == 3) { t.row_group = 4; t.reduce_group = 3; }
      for (const auto& s : sides) check({s}, fp32, t);
      // a batch of mixed sides (the wave-per-slab and row-group rules switch on)
      std::vector<std::pair<int, int>> batch;
      for (int q = 0; q < 300; ++q) {
        const int a = 8 + (q * 37) % 121, b = 8 + (q * 53) % 121;
        batch.push_back({a, q % 3 == 0 ? b : a});
      }
      check(batch, fp32, t);
      check({{1, 1}, {1024, 1}, {1, 1024}, {7, 7}}, fp32, t);
    }
  for (int fp32 = 0; fp32 < 2; ++fp32)
    for (int side : {32, 48, 64, 96, 128, 192, 256}) check_group(side, fp32, default_tuning());
  // invalid sides are refused, not laid out
  Layout lay;
  std::string err;
  if (build_layout({{0, 5}}, 0, default_tuning(), lay, err) ||
      build_layout({{5, 1025}}, 1, default_tuning(), lay, err)) {
    std::fprintf(stderr, "FAIL: invalid sides accepted\n");
    ++fails;
  }
  std::printf("layout checks: %d failures\n", fails);
  return fails ? 1 : 0;
}
