// api.hip -- host side of the C ABI declared in include/slh.h.
//
// Validation, the device key table, the per-context working memory and the
// launch sequence of one batch: prelude -> FORS and TREE -> WOTS, per
// parameter set, in chunks that fit the context's memory budget.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/slh.h"
#include "kernels.hpp"

using namespace slh;

namespace {

thread_local std::string g_free_err;  // errors of the context-free calls

struct Sizes {
  uint32_t n, h, d, hp, a, k, len, m, sig;
};
bool sizes_of(uint32_t param, Sizes* s) {
  switch (param) {
    case SLH_SHA2_128F: *s = {16, 66, 22, 3, 6, 33, 35, 34, uint32_t(P<1>::sig_bytes)}; return true;
    case SLH_SHA2_192F: *s = {24, 66, 22, 3, 8, 33, 51, 42, uint32_t(P<2>::sig_bytes)}; return true;
    case SLH_SHA2_256F: *s = {32, 68, 17, 4, 9, 35, 67, 49, uint32_t(P<3>::sig_bytes)}; return true;
    case SLH_SHA2_128S: *s = {16, 63, 7, 9, 12, 14, 35, 30, uint32_t(P<4>::sig_bytes)}; return true;
    case SLH_SHA2_192S: *s = {24, 63, 7, 9, 14, 17, 51, 39, uint32_t(P<5>::sig_bytes)}; return true;
    case SLH_SHA2_256S: *s = {32, 64, 8, 8, 14, 22, 67, 47, uint32_t(P<6>::sig_bytes)}; return true;
    case SLH_SHAKE_128F: *s = {16, 66, 22, 3, 6, 33, 35, 34, uint32_t(P<7>::sig_bytes)}; return true;
    case SLH_SHAKE_192F: *s = {24, 66, 22, 3, 8, 33, 51, 42, uint32_t(P<8>::sig_bytes)}; return true;
    case SLH_SHAKE_256F: *s = {32, 68, 17, 4, 9, 35, 67, 49, uint32_t(P<9>::sig_bytes)}; return true;
    case SLH_SHAKE_128S: *s = {16, 63, 7, 9, 12, 14, 35, 30, uint32_t(P<10>::sig_bytes)}; return true;
    case SLH_SHAKE_192S: *s = {24, 63, 7, 9, 14, 17, 51, 39, uint32_t(P<11>::sig_bytes)}; return true;
    case SLH_SHAKE_256S: *s = {32, 64, 8, 8, 14, 22, 67, 47, uint32_t(P<12>::sig_bytes)}; return true;
    default: return false;
  }
}

constexpr int kSets = 12;  // parameter sets 1..12 (slh.h SLH_SHA2_*, SLH_SHAKE_*)
// SHA2 set with the same shape (n, h, d, a, k): ids 7..12 are the SHAKE
// counterparts of ids 1..6.
constexpr uint32_t shape_of(uint32_t param) { return (param - 1) % 6 + 1; }
constexpr int kBranches = 3;  // branch streams per context
constexpr size_t kAlign = 256;
size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

void be_words(const uint8_t* b, int nbytes, uint32_t* w) {
  for (int i = 0; i < nbytes / 4; i++)
    w[i] = (uint32_t(b[4 * i]) << 24) | (uint32_t(b[4 * i + 1]) << 16) | (uint32_t(b[4 * i + 2]) << 8) |
           uint32_t(b[4 * i + 3]);
}

DevKey make_devkey(uint32_t param, uint32_t n, const uint8_t* sk_seed, const uint8_t* sk_prf,
                   const uint8_t* pk_seed, const uint8_t* pk_root) {
  DevKey K;
  std::memset(&K, 0, sizeof K);
  K.param = param;
  K.n = n;
  be_words(sk_seed, n, K.sk_seed);
  be_words(sk_prf, n, K.sk_prf);
  be_words(pk_seed, n, K.pk_seed);
  if (pk_root) be_words(pk_root, n, K.pk_root);
  return K;
}

}  // namespace

// Knobs of one parameter set (see slh_tuning in slh.h).
struct Tuning {
  uint32_t fg = 0;          // FORS trees per workgroup (0 = default of the set)
  uint32_t wgs_per_cu = 0;  // fused mode: persistent workgroups per CU (0 = occupancy limit)
  uint32_t keep = 1;        // keep signing-leaf chain values for the WOTS gather
  uint32_t split = 0;       // split_max_blocks (0 = 1.5 x the CU count)
};

struct GraphKey {
  size_t n[kSets + 1];
  const void* msgs;
  void* sigs;
  uint8_t* ws[kSets + 1];
  size_t ws_bytes[kSets + 1];
  uint32_t fg[kSets + 1], wpc[kSets + 1], keep[kSets + 1];
  bool operator==(const GraphKey& o) const { return std::memcmp(this, &o, sizeof o) == 0; }
};

struct slh_ctx {
  int device = 0;
  int cus = 0;
  uint64_t budget = 0;
  std::string err;
  DevKey* keys = nullptr;
  uint32_t nkeys = 0, cap = 0;
  std::vector<uint32_t> key_param;
  uint8_t* ws[kSets + 1] = {};  // working memory per parameter set
  size_t ws_bytes[kSets + 1] = {};
  Tuning tune[kSets + 1];
  DevItem* staging = nullptr;  // pinned host copy of the items of a call
  size_t staging_cap = 0;
  uint8_t* vbuf = nullptr;     // device copy of a verify batch's items
  size_t vbuf_bytes = 0;
  VerifyItem* vstage = nullptr;  // pinned host copy of a verify batch's items
  size_t vstage_cap = 0;
  hipEvent_t done = nullptr;   // end of the last call's GPU work
  bool pending = false;
  hipStream_t cap_stream = nullptr;          // stream graphs are captured on
  // concurrent branches of a mixed fused batch: the g-th parameter set with
  // work runs on branch[g % kBranches].  A few streams per context, not one
  // per set: a process has only a few hardware queues, and more streams
  // make the busy ones of different contexts (server lanes) share queues.
  hipStream_t branch[kBranches] = {};
  hipEvent_t fork = nullptr, join[kBranches] = {};
  std::vector<std::pair<GraphKey, hipGraphExec_t>> graphs;
  // optional per-phase timing: event pairs around every kernel launch
  bool profile = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct Mark { int phase; size_t a, b; uint64_t units; };
  std::vector<Mark> marks;
  double phase_ms[SLH_NPHASES] = {0};
  uint64_t phase_launches[SLH_NPHASES] = {0};
  uint64_t phase_units[SLH_NPHASES] = {0};
  unsigned long long* dstats = nullptr;  // device: trees, distinct trees (dedup mode)
  uint8_t* cache = nullptr;              // device: cached upper-layer trees of keys
  size_t cache_bytes = 0, cache_used = 0;
  std::vector<uint32_t> key_cached;      // per key slot: cached layers
  uint8_t* xbuf = nullptr;               // device: encoded messages of slh_sign_batch_ext
  size_t xbuf_bytes = 0;
  ExtJob* xjobs = nullptr;               // pinned host copy of their encode jobs
  size_t xjobs_cap = 0;
};

namespace {

int fail(slh_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg; else g_free_err = msg;
  return code;
}
int hip_fail(slh_ctx* c, hipError_t e, const char* what) {
  return fail(c, SLH_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
#define HIPCHK(c, x)                                   \
  do {                                                 \
    hipError_t e_ = (x);                               \
    if (e_ != hipSuccess) return hip_fail((c), e_, #x); \
  } while (0)

// Timing of one launch: an event before and after it on the same stream.
struct PhaseTimer {
  slh_ctx* c;
  hipStream_t s;
  int phase;
  uint64_t units;
  size_t a = 0;
  bool on;
  PhaseTimer(slh_ctx* c_, hipStream_t s_, int phase_, uint64_t units_, bool allowed)
      : c(c_), s(s_), phase(phase_), units(units_), on(c_->profile && allowed) {
    if (on) a = take();
  }
  size_t take() {
    if (c->ev_used == c->ev_pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) { on = false; return 0; }
      c->ev_pool.push_back(e);
    }
    const size_t i = c->ev_used++;
    (void)hipEventRecord(c->ev_pool[i], s);
    return i;
  }
  ~PhaseTimer() {
    if (!on) return;
    const size_t b = take();
    if (on) c->marks.push_back({phase, a, b, units});
  }
};

void drop_graphs(slh_ctx* c) {
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.second);
  c->graphs.clear();
}

// FORS trees per workgroup that have a compiled variant, per parameter set.
// Small sets: FORS units of 2^12 leaves, one or two per workgroup.
bool fg_ok(uint32_t param, uint32_t fg) {
  param = shape_of(param);
  if (param >= 4) return fg == 1 || fg == 2;
  if (param == 3) return fg == 2 || fg == 4 || fg == 8;
  return fg == 4 || fg == 8 || fg == 16;
}
uint32_t fg_default(uint32_t param) {
  param = shape_of(param);
  return param >= 4 ? 1u : (param == 3 ? 4u : 8u);
}

// The fused persistent kernel, dedup and the key cache cover the sets whose
// XMSS and FORS trees fit one unit (the fast sets).
template <int ID>
constexpr bool whole_trees() { return P<ID>::tree_units == 1 && P<ID>::fors_units == 1; }

// Call f(std::integral_constant<int, FG>) for the compiled FORS group size fg.
template <int FG>
using FgC = std::integral_constant<int, FG>;
template <int ID, typename F>
void with_fg(uint32_t fg, F&& f) {
  constexpr uint32_t S = shape_of(ID);
  if constexpr (S >= 4) {
    if (fg == 2) f(FgC<2>{}); else f(FgC<1>{});
  } else if constexpr (S == 3) {
    if (fg == 2) f(FgC<2>{}); else if (fg == 8) f(FgC<8>{}); else f(FgC<4>{});
  } else {
    if (fg == 4) f(FgC<4>{}); else if (fg == 16) f(FgC<16>{}); else f(FgC<8>{});
  }
}

// Call f(std::integral_constant<int, ID>) for parameter set `param` (1..12).
template <typename F>
auto with_set(uint32_t param, F&& f) {
  switch (param) {
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 3: return f(std::integral_constant<int, 3>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 5: return f(std::integral_constant<int, 5>{});
    case 6: return f(std::integral_constant<int, 6>{});
    case 7: return f(std::integral_constant<int, 7>{});
    case 8: return f(std::integral_constant<int, 8>{});
    case 9: return f(std::integral_constant<int, 9>{});
    case 10: return f(std::integral_constant<int, 10>{});
    case 11: return f(std::integral_constant<int, 11>{});
    default: return f(std::integral_constant<int, 12>{});
  }
}

template <int ID, int FG>
int occupancy_of() {
  static int occ = -1;
  if (occ < 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&k_fused<ID, FG>),
                                                     kTreeThreads, 0) != hipSuccess || nb < 1)
      nb = 1;
    occ = nb;
  }
  return occ;
}
template <int ID>
int occupancy(uint32_t fg) {
  if constexpr (!whole_trees<ID>()) {
    return 1;
  } else if constexpr (shape_of(ID) == 3) {
    return fg == 2 ? occupancy_of<ID, 2>() : fg == 8 ? occupancy_of<ID, 8>() : occupancy_of<ID, 4>();
  } else {
    return fg == 4 ? occupancy_of<ID, 4>() : fg == 16 ? occupancy_of<ID, 16>() : occupancy_of<ID, 8>();
  }
}

// Working-memory plan of one chunk of `n` messages of parameter set ID.
// TREE blocks of one plain launch at most (the staging is reused by the
// launches of a chunk when the small sets need more blocks than this).
constexpr uint32_t kMaxTreeBlocks = 32768;

template <int ID>
struct Plan {
  using Q = P<ID>;
  static constexpr uint32_t TPB = kLeavesPerBlock >> Q::unit_hp;  // trees (or units) per TREE block
  size_t n = 0;
  bool fused = false, dedup = false, keep = true;
  uint32_t parts = 0;  // > 0: TREE blocks' chains split over this many workgroups (small batches)
  uint32_t fg = 8, grid = 0, ntb = 0, nfg = 0, table = 0;
  size_t o_recs = 0, o_items = 0, o_stage = 0, o_spill = 0, o_roots = 0, o_queue = 0;
  size_t o_table = 0, o_rep = 0, o_ulist = 0, o_lown = 0, o_nodes = 0, o_troots = 0, o_uroots = 0, total = 0;
  static constexpr size_t stage_per_block = size_t(Q::len) * kLeavesPerBlock * Q::NW * 4;
  Plan(size_t n_, uint32_t mode, const Tuning& t, int cus)
      : n(n_),
        fused(whole_trees<ID>() && (mode & SLH_MODE_FUSED) != 0),
        dedup(whole_trees<ID>() && (mode & SLH_MODE_DEDUP) != 0),
        keep(t.keep != 0) {
    fg = t.fg ? t.fg : fg_default(ID);
    const size_t trees = n * Q::d;
    ntb = uint32_t((trees * Q::tree_units + TPB - 1) / TPB);
    nfg = uint32_t((n * Q::k * Q::fors_units + fg - 1) / fg);
    // With few TREE blocks the batch cannot fill the chip and its time is
    // one block's chain latency: split each block's chains over up to len
    // one-wave workgroups, about 8 waves per CU in all (the per-phase path;
    // the same bytes in every mode).  Measured on MI355X, the split wins up
    // to about 1.4 blocks per CU, ties to 2 and loses above.
    const uint32_t split_max =
        t.split == SLH_SPLIT_NEVER ? 0u : (t.split ? t.split : 3u * uint32_t(cus) / 2u);
    if (ntb <= split_max) {
      parts = std::max<uint32_t>(1u, std::min<uint32_t>(Q::len, 8u * uint32_t(cus) / std::max(1u, ntb)));
      fused = false;
    }
    if (fused) {
      const uint32_t per_cu = t.wgs_per_cu ? t.wgs_per_cu : uint32_t(occupancy<ID>(fg));
      grid = std::min<uint32_t>(per_cu * uint32_t(cus), ntb + nfg);
    } else {
      grid = std::min(ntb, kMaxTreeBlocks);
    }
    o_recs = 0;
    o_items = o_recs + up(n * sizeof(WorkRec));
    o_stage = o_items + up(n * sizeof(DevItem));
    // the fused kernel double-buffers its staging per workgroup
    o_spill = o_stage + up(size_t(grid) * stage_per_block * (fused ? 2 : 1));
    o_roots = o_spill + (keep ? up(n * Q::d * Q::len * 16 * Q::NW * 4) : 0);
    o_troots = o_roots + up(n * Q::k * Q::fors_units * Q::NW * 4);  // unit roots
    o_uroots = o_troots + (Q::fors_units > 1 ? up(n * Q::k * Q::NW * 4) : 0);  // tree roots
    o_queue = o_uroots + (Q::tree_units > 1 ? up(trees * Q::tree_units * Q::NW * 4) : 0);
    // dedup: hash table (>= 2 slots per tree), representative per tree, list
    // of representatives (its count is the word after the work counter), the
    // owner of every leaf of every tree, and every node of every tree
    o_table = o_queue + kAlign;
    if (dedup) {
      table = 2;
      while (table < 2 * trees) table <<= 1;
      o_rep = o_table + up(size_t(table) * sizeof(DedupSlot));
      o_ulist = o_rep + up(trees * 4);
      o_lown = o_ulist + up(trees * 4);
      o_nodes = o_lown + up(trees * Q::leaves * 4);
      total = o_nodes + up(trees * TreeNodes<ID>::count * Q::NW * 4);
    } else {
      total = o_table;
    }
  }
};

// Make sure parameter set p has `bytes` of working memory (waits for pending
// work and drops captured graphs before replacing the buffer).
int ensure_ws(slh_ctx* c, int p, size_t bytes) {
  if (c->ws_bytes[p] >= bytes) return SLH_OK;
  if (c->pending) HIPCHK(c, hipEventSynchronize(c->done));
  drop_graphs(c);
  if (c->ws[p]) HIPCHK(c, hipFree(c->ws[p]));
  c->ws[p] = nullptr;
  c->ws_bytes[p] = 0;
  hipError_t e = hipMalloc(&c->ws[p], bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, SLH_ENOMEM, "hipMalloc of working memory failed");
  }
  c->ws_bytes[p] = bytes;
  return SLH_OK;
}

// Working-memory share of one parameter set: the budget split evenly over
// the sets the context holds keys of.
uint64_t budget_share(const slh_ctx* c) {
  int sets = 0;
  for (int p = 1; p <= kSets; p++)
    sets += std::find(c->key_param.begin(), c->key_param.end(), uint32_t(p)) != c->key_param.end() ? 1 : 0;
  return c->budget / uint64_t(sets ? sets : 1);
}

template <int ID, int FG>
void launch_fors(slh_ctx* c, const Plan<ID>& pl, uint8_t* sigs, WorkRec* recs, uint32_t* roots, hipStream_t s) {
  hipLaunchKernelGGL((k_fors<ID, FG>), dim3(pl.nfg), dim3(kForsThreads), 0, s, c->keys, recs,
                     uint32_t(pl.n * P<ID>::k * P<ID>::fors_units), sigs, roots);
}
// Dedup buffers of a chunk (all null without dedup).
struct DedupBufs {
  DedupSlot* table = nullptr;
  uint32_t* rep = nullptr;
  uint32_t* ulist = nullptr;
  uint32_t* ucount = nullptr;
  uint32_t* lown = nullptr;
  uint32_t* nodes = nullptr;
};

template <int ID, int FG>
void launch_fused(slh_ctx* c, const Plan<ID>& pl, uint8_t* sigs, WorkRec* recs, uint32_t* stage, uint32_t* spill,
                  uint32_t* roots, uint32_t* queue, const DedupBufs& db, hipStream_t s) {
  hipLaunchKernelGGL((k_fused<ID, FG>), dim3(pl.grid), dim3(kTreeThreads), 0, s, c->keys, recs, uint32_t(pl.n),
                     sigs, stage, spill, roots, queue, pl.ntb, pl.nfg, db.ulist, db.ucount, db.lown, db.nodes);
}

// Enqueue one chunk on stream s.  `timing` is false while a graph is captured.
template <int ID>
int launch_chunk(slh_ctx* c, const Plan<ID>& pl, const DevItem* h_items, const uint8_t* msgs, uint8_t* sigs,
                 hipStream_t s, bool timing) {
  using Q = P<ID>;
  uint8_t* base = c->ws[ID];
  WorkRec* recs = reinterpret_cast<WorkRec*>(base + pl.o_recs);
  DevItem* items = reinterpret_cast<DevItem*>(base + pl.o_items);
  uint32_t* stage = reinterpret_cast<uint32_t*>(base + pl.o_stage);
  uint32_t* spill = pl.keep ? reinterpret_cast<uint32_t*>(base + pl.o_spill) : nullptr;
  uint32_t* roots = reinterpret_cast<uint32_t*>(base + pl.o_roots);
  uint32_t* queue = reinterpret_cast<uint32_t*>(base + pl.o_queue);
  DedupBufs db;
  if (pl.dedup) {
    db.table = reinterpret_cast<DedupSlot*>(base + pl.o_table);
    db.rep = reinterpret_cast<uint32_t*>(base + pl.o_rep);
    db.ulist = reinterpret_cast<uint32_t*>(base + pl.o_ulist);
    db.ucount = queue + 1;
    db.lown = reinterpret_cast<uint32_t*>(base + pl.o_lown);
    db.nodes = reinterpret_cast<uint32_t*>(base + pl.o_nodes);
  }
  HIPCHK(c, hipMemcpyAsync(items, h_items, pl.n * sizeof(DevItem), hipMemcpyHostToDevice, s));
  const uint32_t n = uint32_t(pl.n);
  const uint32_t trees = n * Q::d;
  {
    PhaseTimer t(c, s, SLH_PHASE_PRELUDE, n, timing);
    hipLaunchKernelGGL((k_prelude<ID>), dim3((n + 63) / 64), dim3(64), 0, s, c->keys, items, n, msgs, sigs, recs,
                       pl.fused ? queue : nullptr);
    if constexpr (whole_trees<ID>()) {
      if (pl.dedup) {
      const uint32_t nlown = trees * Q::leaves;
      hipLaunchKernelGGL(k_dedup_init, dim3((std::max(pl.table, nlown) + 255) / 256), dim3(256), 0, s, db.table,
                         pl.table, db.lown, nlown, db.ucount);
      hipLaunchKernelGGL((k_dedup_insert<ID>), dim3((trees + 255) / 256), dim3(256), 0, s, c->keys, recs, n,
                         db.table, pl.table, db.rep);
      hipLaunchKernelGGL((k_dedup_resolve<ID>), dim3((trees + 255) / 256), dim3(256), 0, s, recs, n, db.table,
                         db.rep, db.ulist, db.ucount, db.lown);
      hipLaunchKernelGGL(k_dedup_stats, dim3(1), dim3(64), 0, s, trees, db.ucount, c->dstats);
      }
    }
  }
  if constexpr (whole_trees<ID>()) {
    if (pl.fused) {
      PhaseTimer t(c, s, SLH_PHASE_FUSED, n, timing);
      with_fg<ID>(pl.fg, [&](auto fgc) {
        launch_fused<ID, decltype(fgc)::value>(c, pl, sigs, recs, stage, spill, roots, queue, db, s);
      });
    }
  }
  if (!pl.fused) {
    {
      PhaseTimer t(c, s, SLH_PHASE_FORS, n, timing);
      with_fg<ID>(pl.fg, [&](auto fgc) { launch_fors<ID, decltype(fgc)::value>(c, pl, sigs, recs, roots, s); });
      if constexpr (Q::fors_units > 1) {
        const uint32_t nft = n * Q::k;
        hipLaunchKernelGGL((k_fors_top<ID>), dim3((nft + 63) / 64), dim3(64), 0, s, c->keys, recs, nft, sigs, roots,
                           reinterpret_cast<uint32_t*>(base + pl.o_troots));
      }
    }
    {
      PhaseTimer t(c, s, SLH_PHASE_TREE, n, timing);
      uint32_t* uroots = Q::tree_units > 1 ? reinterpret_cast<uint32_t*>(base + pl.o_uroots) : nullptr;
      const uint32_t units = trees * Q::tree_units;
      // at most kMaxTreeBlocks blocks per launch, reusing the staging
      for (uint32_t b0 = 0; b0 < pl.ntb; b0 += kMaxTreeBlocks) {
        const uint32_t nb = std::min(kMaxTreeBlocks, pl.ntb - b0), first = b0 * Plan<ID>::TPB;
        const uint32_t nu = std::min(units - first, nb * Plan<ID>::TPB);
        if (pl.parts) {
          hipLaunchKernelGGL((k_tree_chains<ID, kSignTrees>), dim3(nb, pl.parts), dim3(64), 0, s, c->keys, recs, nu,
                             sigs, stage, spill, 0u, nullptr, db.ulist, db.ucount, db.lown, first, uroots);
          hipLaunchKernelGGL((k_tree_finish<ID, kSignTrees>), dim3(nb), dim3(64), 0, s, c->keys, recs, nu, sigs,
                             stage, spill, 0u, nullptr, db.ulist, db.ucount, db.lown, db.nodes, first, uroots);
        } else
          hipLaunchKernelGGL((k_tree<ID, kSignTrees>), dim3(nb), dim3(kTreeThreads), 0, s, c->keys, recs, nu, sigs,
                             stage, spill, 0u, nullptr, db.ulist, db.ucount, db.lown, db.nodes, first, uroots);
      }
      if constexpr (Q::tree_units > 1)
        hipLaunchKernelGGL((k_tree_top<ID, kSignTrees>), dim3((trees + 63) / 64), dim3(64), 0, s, c->keys, recs,
                           trees, sigs, 0u, nullptr, 0u, uroots);
    }
  }
  {
    PhaseTimer t(c, s, SLH_PHASE_WOTS, n, timing);
    if constexpr (whole_trees<ID>()) {
      if (pl.dedup)
        hipLaunchKernelGGL((k_dedup_scatter<ID>), dim3((trees + 255) / 256), dim3(256), 0, s, c->keys, recs, n,
                           sigs, db.rep, db.nodes, c->cache);
    }
    const uint32_t* troots =
        Q::fors_units > 1 ? reinterpret_cast<const uint32_t*>(base + pl.o_troots) : roots;  // tree roots
    hipLaunchKernelGGL((k_fors_pk<ID>), dim3((n + 63) / 64), dim3(64), 0, s, c->keys, recs, n, troots);
    const uint32_t nw = n * Q::d * Q::len;
    if (pl.keep && pl.dedup) {
      if constexpr (whole_trees<ID>())
        hipLaunchKernelGGL((k_wots_dedup<ID>), dim3((nw + 255) / 256), dim3(256), 0, s, c->keys, recs, n, sigs,
                           spill, db.rep, db.lown);
    } else if (pl.keep)
      hipLaunchKernelGGL((k_wots<ID>), dim3((nw + 255) / 256), dim3(256), 0, s, recs, n, sigs, spill);
    else
      hipLaunchKernelGGL((k_wots_recompute<ID>), dim3((nw + 255) / 256), dim3(256), 0, s, c->keys, recs, n, sigs);
  }
  HIPCHK(c, hipGetLastError());
  return SLH_OK;
}

// Messages per chunk for parameter set ID within `budget` bytes.
template <int ID>
size_t chunk_size(slh_ctx* c, size_t count, uint32_t mode, uint64_t budget) {
  const Tuning& t = c->tune[ID];
  const Plan<ID> one(1, mode, t, c->cus), big(1024, mode, t, c->cus);
  const size_t per = (big.total - one.total) / 1023 + 1;
  const size_t fixed = one.total > per ? one.total - per : 0;
  size_t chunk = budget > fixed ? (budget - fixed) / per : 1;
  chunk = std::max<size_t>(1, std::min(chunk, count));
  // the dedup table is rounded up to a power of two: shrink until it fits
  while (chunk > 1 && Plan<ID>(chunk, mode, t, c->cus).total > budget) chunk -= chunk / 64 + 1;
  return chunk;
}

template <int ID>
int prepare_group(slh_ctx* c, size_t count, uint32_t mode, uint64_t budget, size_t* chunk) {
  *chunk = chunk_size<ID>(c, count, mode, budget);
  const Plan<ID> pl(*chunk, mode, c->tune[ID], c->cus);
  return ensure_ws(c, ID, pl.total);
}

template <int ID>
int enqueue_group(slh_ctx* c, const DevItem* h_items, size_t count, size_t chunk, const uint8_t* msgs,
                  uint8_t* sigs, hipStream_t s, uint32_t mode, bool timing) {
  for (size_t off = 0; off < count; off += chunk) {
    const size_t cnt = std::min(chunk, count - off);
    const Plan<ID> pl(cnt, mode, c->tune[ID], c->cus);
    const int rc = launch_chunk<ID>(c, pl, h_items + off, msgs, sigs, s, timing);
    if (rc) return rc;
  }
  return SLH_OK;
}

int enqueue_all(slh_ctx* c, const size_t* per, const size_t* start, const size_t* chunk, const uint8_t* msgs,
                uint8_t* sigs, hipStream_t s, uint32_t mode, bool timing) {
  int groups = 0;
  for (int p = 1; p <= kSets; p++) groups += per[p] ? 1 : 0;
  const bool branches = (mode & SLH_MODE_FUSED) && groups > 1;
  if (branches) HIPCHK(c, hipEventRecord(c->fork, s));
  int g = 0;
  for (int p = 1; p <= kSets; p++) {
    if (!per[p]) continue;
    hipStream_t b = s;
    const int br = g++ % kBranches;
    if (branches) {
      b = c->branch[br];
      HIPCHK(c, hipStreamWaitEvent(b, c->fork, 0));
    }
    const int rc = with_set(uint32_t(p), [&](auto id) {
      return enqueue_group<decltype(id)::value>(c, c->staging + start[p], per[p], chunk[p], msgs, sigs, b, mode,
                                                timing);
    });
    if (rc) return rc;
    if (branches) {
      HIPCHK(c, hipEventRecord(c->join[br], b));
      HIPCHK(c, hipStreamWaitEvent(s, c->join[br], 0));
    }
  }
  return SLH_OK;
}

}  // namespace

namespace {
template <int ID>
int keygen_impl(const uint8_t* seed, uint8_t* pk, uint8_t* sk) {
  using Q = P<ID>;
  const uint32_t n = Q::n;
  DevKey hk = make_devkey(ID, n, seed, seed + n, seed + 2 * n, nullptr);
  DevKey* dk = nullptr;
  uint32_t* stage = nullptr;
  uint32_t* root = nullptr;
  uint32_t* uroots = nullptr;
  constexpr uint32_t UT = Q::tree_units;  // TREE blocks of the top tree (1 for the fast sets)
  const size_t stage_bytes = size_t(UT) * Q::len * kLeavesPerBlock * Q::NW * 4;
  hipError_t e = hipMalloc(&dk, sizeof(DevKey));
  if (e == hipSuccess) e = hipMalloc(&stage, stage_bytes);
  if (e == hipSuccess) e = hipMalloc(&root, 32);
  if (e == hipSuccess) e = hipMalloc(&uroots, size_t(UT) * Q::NW * 4);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    if (dk) (void)hipFree(dk);
    if (stage) (void)hipFree(stage);
    if (root) (void)hipFree(root);
    if (uroots) (void)hipFree(uroots);
    return fail(nullptr, SLH_ENOMEM, "keygen device allocation failed");
  }
  uint32_t hroot[8] = {0};
  e = hipMemcpy(dk, &hk, sizeof hk, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_key_midstates, dim3(1), dim3(64), 0, 0, dk, 0u, 1u);
    // one tree: its chains split over len one-wave workgroups per unit
    hipLaunchKernelGGL((k_tree_chains<ID, kKeygenTree>), dim3(UT, Q::len), dim3(64), 0, 0, dk, nullptr, UT, nullptr,
                       stage, nullptr, 0u, root, nullptr, nullptr, nullptr, 0u, uroots);
    hipLaunchKernelGGL((k_tree_finish<ID, kKeygenTree>), dim3(UT), dim3(64), 0, 0, dk, nullptr, UT, nullptr, stage,
                       nullptr, 0u, root, nullptr, nullptr, nullptr, nullptr, 0u, uroots);
    if constexpr (UT > 1)
      hipLaunchKernelGGL((k_tree_top<ID, kKeygenTree>), dim3(1), dim3(64), 0, 0, dk, nullptr, 1u, nullptr, 0u, root,
                         0u, uroots);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(hroot, root, Q::n, hipMemcpyDeviceToHost);
  (void)hipFree(dk);
  (void)hipFree(stage);
  (void)hipFree(root);
  (void)hipFree(uroots);
  if (e != hipSuccess) return hip_fail(nullptr, e, "keygen");
  std::memcpy(sk, seed, 3 * n);
  for (uint32_t i = 0; i < n / 4; i++) {
    for (int b = 0; b < 4; b++) {
      const uint8_t byte = uint8_t(hroot[i] >> (24 - 8 * b));
      sk[3 * n + 4 * i + b] = byte;
      pk[n + 4 * i + b] = byte;
    }
  }
  std::memcpy(pk, seed + 2 * n, n);
  return SLH_OK;
}

// Most cached layers per parameter set: at most 2^16 trees per key.
// (the small sets' trees are built in units; they are not cached)
uint32_t max_cache_layers(uint32_t param) {
  param = shape_of(param);
  return param >= 4 ? 0u : (param == 3 ? 4u : 6u);
}

// Build the cached upper layers of keys [first, first + count) (all of set ID).
template <int ID>
int cache_impl(slh_ctx* c, uint32_t first, uint32_t count, uint32_t layers) {
  using Q = P<ID>;
  const uint64_t per = CacheShape<ID>::trees(layers);
  const uint64_t per_bytes = per * TreeNodes<ID>::count * Q::NW * 4;
  const uint64_t need = per_bytes * count;
  if (uint64_t(count) * per >= (1ull << 31)) return fail(c, SLH_EINVAL, "too many cached trees in one call");
  if (c->pending) HIPCHK(c, hipEventSynchronize(c->done));
  if (c->cache_used + need > c->cache_bytes) {
    // grow: the captured graphs hold the old address
    const size_t nb = std::max<size_t>(c->cache_used + need, c->cache_bytes * 2);
    uint8_t* nc = nullptr;
    if (hipMalloc(&nc, nb) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, SLH_ENOMEM, "hipMalloc of the tree cache failed");
    }
    if (c->cache_used) HIPCHK(c, hipMemcpy(nc, c->cache, c->cache_used, hipMemcpyDeviceToDevice));
    if (c->cache) HIPCHK(c, hipFree(c->cache));
    c->cache = nc;
    c->cache_bytes = nb;
    drop_graphs(c);
  }
  const uint64_t off0 = c->cache_used;
  hipLaunchKernelGGL(k_set_cache, dim3((count + 63) / 64), dim3(64), 0, 0, c->keys, first, count, layers, off0,
                     per_bytes);
  HIPCHK(c, hipGetLastError());
  // all trees of the range, in launches of at most 1024 TREE blocks
  constexpr uint32_t TPB = kLeavesPerBlock / Q::leaves;
  constexpr uint32_t kMaxBlocks = 1024;
  const size_t stage_bytes = size_t(kMaxBlocks) * Q::len * kLeavesPerBlock * Q::NW * 4;
  uint32_t* stage = nullptr;
  if (hipMalloc(&stage, stage_bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, SLH_ENOMEM, "hipMalloc of cache staging failed");
  }
  const uint32_t total = uint32_t(count * per);
  uint32_t* nodes = reinterpret_cast<uint32_t*>(c->cache + off0);
  hipError_t e = hipSuccess;
  for (uint32_t t0 = 0; t0 < total && e == hipSuccess; t0 += kMaxBlocks * TPB) {
    const uint32_t n = std::min<uint32_t>(kMaxBlocks * TPB, total - t0);
    hipLaunchKernelGGL((k_tree<ID, kCacheTrees>), dim3((n + TPB - 1) / TPB), dim3(kTreeThreads), 0, 0, c->keys,
                       nullptr, n, nullptr, stage, nullptr, first, nullptr, nullptr, nullptr, nullptr, nodes, t0,
                       nullptr);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  (void)hipFree(stage);
  if (e != hipSuccess) return hip_fail(c, e, "tree cache build");
  c->cache_used += need;
  for (uint32_t i = 0; i < count; i++) c->key_cached[first + i] = layers;
  return SLH_OK;
}

template <int ID>
int verify_impl(const uint8_t* msg, size_t msg_len, const uint8_t* sig, const uint8_t* pk) {
  using Q = P<ID>;
  const size_t mbytes = std::max<size_t>(msg_len, 1);
  const size_t total = up(sizeof(VerifyItem)) + up(mbytes) + up(Q::sig_bytes) + up(2 * Q::n) + up(sizeof(int));
  uint8_t* buf = nullptr;
  hipError_t e = hipMalloc(&buf, total);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(nullptr, SLH_ENOMEM, "verify device allocation failed");
  }
  VerifyItem it{0, msg_len, 0, 0, 0};
  uint8_t* d_items = buf;
  uint8_t* d_msg = d_items + up(sizeof(VerifyItem));
  uint8_t* d_sig = d_msg + up(mbytes);
  uint8_t* d_pk = d_sig + up(Q::sig_bytes);
  int* d_res = reinterpret_cast<int*>(d_pk + up(2 * Q::n));
  int res = -1;
  e = hipMemcpy(d_items, &it, sizeof it, hipMemcpyHostToDevice);
  if (e == hipSuccess && msg_len) e = hipMemcpy(d_msg, msg, msg_len, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_sig, sig, Q::sig_bytes, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_pk, pk, 2 * Q::n, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    hipLaunchKernelGGL((k_verify<ID, kVerifyGroupWide>), dim3(1), dim3(kVerifyThreads), 0, 0,
                       reinterpret_cast<const VerifyItem*>(d_items), 1u, d_msg, d_sig, d_pk, d_res);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(&res, d_res, sizeof res, hipMemcpyDeviceToHost);
  (void)hipFree(buf);
  if (e != hipSuccess) return hip_fail(nullptr, e, "verify");
  return res;
}
}  // namespace

extern "C" {

int slh_params(uint32_t param, slh_sizes* out) {
  Sizes s;
  if (!out || !sizes_of(param, &s)) return fail(nullptr, SLH_EINVAL, "unknown parameter set");
  out->n = s.n; out->h = s.h; out->d = s.d; out->hp = s.hp; out->a = s.a; out->k = s.k;
  out->len = s.len; out->m = s.m;
  out->seed_bytes = 3 * s.n; out->pk_bytes = 2 * s.n; out->sk_bytes = 4 * s.n; out->sig_bytes = s.sig;
  return SLH_OK;
}

int slh_ctx_create(int device, uint64_t hbm_budget, slh_ctx** out) {
  if (!out) return fail(nullptr, SLH_EINVAL, "null output pointer");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDeviceCount");
  if (device < 0 || device >= ndev) return fail(nullptr, SLH_EINVAL, "no such device");
  slh_ctx* c = new slh_ctx();
  c->device = device;
  c->budget = hbm_budget ? hbm_budget : (uint64_t(8) << 30);
  e = hipSetDevice(device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipMalloc(&c->dstats, 2 * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMemset(c->dstats, 0, 2 * sizeof(unsigned long long));
  // all streams at the default priority
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
  for (int b = 0; b < kBranches && e == hipSuccess; b++) {
    e = hipStreamCreateWithFlags(&c->branch[b], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->join[b], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    slh_ctx_destroy(c);
    return hip_fail(nullptr, e, "context set-up");
  }
  for (int p = 1; p <= kSets; p++) c->tune[p].fg = fg_default(uint32_t(p));
  *out = c;
  return SLH_OK;
}

int slh_ctx_destroy(slh_ctx* c) {
  if (!c) return SLH_OK;
  (void)hipSetDevice(c->device);
  if (c->pending) (void)hipEventSynchronize(c->done);
  (void)hipDeviceSynchronize();
  drop_graphs(c);
  for (int p = 0; p <= kSets; p++)
    if (c->ws[p]) (void)hipFree(c->ws[p]);
  for (int b = 0; b < kBranches; b++) {
    if (c->branch[b]) (void)hipStreamDestroy(c->branch[b]);
    if (c->join[b]) (void)hipEventDestroy(c->join[b]);
  }
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->keys) (void)hipFree(c->keys);
  if (c->dstats) (void)hipFree(c->dstats);
  if (c->cache) (void)hipFree(c->cache);
  if (c->xbuf) (void)hipFree(c->xbuf);
  if (c->xjobs) (void)hipHostFree(c->xjobs);
  if (c->staging) (void)hipHostFree(c->staging);
  if (c->vbuf) (void)hipFree(c->vbuf);
  if (c->vstage) (void)hipHostFree(c->vstage);
  if (c->done) (void)hipEventDestroy(c->done);
  if (c->fork) (void)hipEventDestroy(c->fork);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  delete c;
  return SLH_OK;
}

const char* slh_last_error(const slh_ctx* c) { return c ? c->err.c_str() : g_free_err.c_str(); }

int slh_ctx_profile(slh_ctx* c, int enable) {
  if (!c) return fail(nullptr, SLH_EINVAL, "null context");
  c->profile = enable != 0;
  return SLH_OK;
}

int slh_ctx_phase_times(slh_ctx* c, double* ms, uint64_t* launches, uint64_t* messages, int reset) {
  if (!c || !ms || !launches || !messages) return fail(c, SLH_EINVAL, "null argument");
  HIPCHK(c, hipSetDevice(c->device));
  for (const auto& m : c->marks) {
    HIPCHK(c, hipEventSynchronize(c->ev_pool[m.b]));
    float t = 0.f;
    HIPCHK(c, hipEventElapsedTime(&t, c->ev_pool[m.a], c->ev_pool[m.b]));
    c->phase_ms[m.phase] += t;
    c->phase_launches[m.phase] += 1;
    c->phase_units[m.phase] += m.units;
  }
  c->marks.clear();
  c->ev_used = 0;
  for (int i = 0; i < SLH_NPHASES; i++) {
    ms[i] = c->phase_ms[i];
    launches[i] = c->phase_launches[i];
    messages[i] = c->phase_units[i];
    if (reset) { c->phase_ms[i] = 0; c->phase_launches[i] = 0; c->phase_units[i] = 0; }
  }
  return SLH_OK;
}

int slh_ctx_dedup_stats(slh_ctx* c, uint64_t* trees, uint64_t* distinct, int reset) {
  if (!c || !trees || !distinct) return fail(c, SLH_EINVAL, "null argument");
  HIPCHK(c, hipSetDevice(c->device));
  if (c->pending) HIPCHK(c, hipEventSynchronize(c->done));
  unsigned long long h[2] = {0, 0};
  HIPCHK(c, hipMemcpy(h, c->dstats, sizeof h, hipMemcpyDeviceToHost));
  *trees = h[0];
  *distinct = h[1];
  if (reset) HIPCHK(c, hipMemset(c->dstats, 0, sizeof h));
  return SLH_OK;
}

int slh_ctx_reserve(slh_ctx* c, uint32_t count, uint32_t mode) {
  if (!c) return fail(nullptr, SLH_EINVAL, "null context");
  if (mode & ~(SLH_MODE_FUSED | SLH_MODE_GRAPH | SLH_MODE_DEDUP)) return fail(c, SLH_EINVAL, "unknown mode");
  if (count == 0) return SLH_OK;
  HIPCHK(c, hipSetDevice(c->device));
  if (c->pending) HIPCHK(c, hipEventSynchronize(c->done));
  if (c->staging_cap < count) {
    drop_graphs(c);
    if (c->staging) HIPCHK(c, hipHostFree(c->staging));
    c->staging = nullptr;
    c->staging_cap = 0;
    if (hipHostMalloc(&c->staging, size_t(count) * sizeof(DevItem)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, SLH_ENOMEM, "pinned staging allocation failed");
    }
    c->staging_cap = count;
  }
  const uint64_t share = budget_share(c);
  size_t chunk = 0;
  int rc = SLH_OK;
  for (int p = 1; p <= kSets && !rc; p++) {
    if (std::find(c->key_param.begin(), c->key_param.end(), uint32_t(p)) == c->key_param.end()) continue;
    rc = with_set(uint32_t(p), [&](auto id) {
      return prepare_group<decltype(id)::value>(c, count, mode, share, &chunk);
    });
  }
  return rc;
}

int slh_ctx_cache_keys(slh_ctx* c, uint32_t first_slot, uint32_t count, uint32_t layers) {
  if (!c) return fail(nullptr, SLH_EINVAL, "null context");
  if (count == 0 || uint64_t(first_slot) + count > c->nkeys) return fail(c, SLH_EINVAL, "key range outside the table");
  const uint32_t param = c->key_param[first_slot];
  if (max_cache_layers(param) == 0) return fail(c, SLH_EINVAL, "the small parameter sets have no tree cache");
  if (layers == 0 || layers > max_cache_layers(param))
    return fail(c, SLH_EINVAL, "cached layers must be 1.." + std::to_string(max_cache_layers(param)));
  for (uint32_t i = first_slot; i < first_slot + count; i++) {
    if (c->key_param[i] != param) return fail(c, SLH_EINVAL, "keys of different parameter sets");
    if (c->key_cached[i]) return fail(c, SLH_EINVAL, "key " + std::to_string(i) + " is cached already");
  }
  HIPCHK(c, hipSetDevice(c->device));
  switch (param) {
    case 1: return cache_impl<1>(c, first_slot, count, layers);
    case 2: return cache_impl<2>(c, first_slot, count, layers);
    case 3: return cache_impl<3>(c, first_slot, count, layers);
    case 7: return cache_impl<7>(c, first_slot, count, layers);
    case 8: return cache_impl<8>(c, first_slot, count, layers);
    default: return cache_impl<9>(c, first_slot, count, layers);  // the small sets were rejected above
  }
}

int slh_ctx_add_keys(slh_ctx* c, uint32_t param, const uint8_t* sks, uint32_t count, uint32_t* first_slot) {
  Sizes s;
  if (!c) return fail(nullptr, SLH_EINVAL, "null context");
  if (!sizes_of(param, &s)) return fail(c, SLH_EINVAL, "unknown parameter set");
  if (!sks || !first_slot || count == 0) return fail(c, SLH_EINVAL, "null keys, null slot or zero count");
  if (uint64_t(c->nkeys) + count > (1u << 24)) return fail(c, SLH_EINVAL, "too many keys");
  HIPCHK(c, hipSetDevice(c->device));
  if (c->pending) HIPCHK(c, hipEventSynchronize(c->done));
  // captured graphs hold the key table's address (which a reallocation
  // below frees) and working-memory chunks sized for the sets that had keys
  drop_graphs(c);
  if (c->nkeys + count > c->cap) {
    uint32_t ncap = std::max<uint32_t>(64, c->cap);
    while (ncap < c->nkeys + count) ncap *= 2;
    DevKey* nk = nullptr;
    if (hipMalloc(&nk, size_t(ncap) * sizeof(DevKey)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, SLH_ENOMEM, "hipMalloc of the key table failed");
    }
    if (c->keys) {
      HIPCHK(c, hipMemcpy(nk, c->keys, size_t(c->nkeys) * sizeof(DevKey), hipMemcpyDeviceToDevice));
      HIPCHK(c, hipFree(c->keys));
    }
    c->keys = nk;
    c->cap = ncap;
  }
  std::vector<DevKey> hk(count);
  const uint32_t n = s.n;
  for (uint32_t i = 0; i < count; i++) {
    const uint8_t* k = sks + size_t(i) * 4 * n;
    hk[i] = make_devkey(param, n, k, k + n, k + 2 * n, k + 3 * n);
  }
  HIPCHK(c, hipMemcpy(c->keys + c->nkeys, hk.data(), count * sizeof(DevKey), hipMemcpyHostToDevice));
  hipLaunchKernelGGL(k_key_midstates, dim3((count + 63) / 64), dim3(64), 0, 0, c->keys, c->nkeys, count);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipDeviceSynchronize());
  *first_slot = c->nkeys;
  c->nkeys += count;
  c->key_param.resize(c->nkeys, param);
  c->key_cached.resize(c->nkeys, 0);
  return SLH_OK;
}

}  // extern "C"

namespace {
// slh_sign_batch with an optional opt_rand location per item (rnd[i] =
// kNoRnd: deterministic).
int sign_impl(slh_ctx* c, const slh_item* items, const uint64_t* rnd, uint32_t count, const uint8_t* msgs,
              uint64_t msgs_bytes, uint8_t* sigs, uint64_t sigs_bytes, uint32_t mode, void* stream) {
  if (!c) return fail(nullptr, SLH_EINVAL, "null context");
  if (count == 0) return SLH_OK;
  if (!items || !sigs) return fail(c, SLH_EINVAL, "null items or signature buffer");
  if (mode & ~(SLH_MODE_FUSED | SLH_MODE_GRAPH | SLH_MODE_DEDUP)) return fail(c, SLH_EINVAL, "unknown mode");
  if (reinterpret_cast<uintptr_t>(sigs) % 16) return fail(c, SLH_EINVAL, "signature buffer not 16-byte aligned");
  // validation, and grouping by parameter set
  std::vector<std::pair<uint64_t, uint64_t>> ranges;
  ranges.reserve(count);
  size_t per[kSets + 1] = {};
  for (uint32_t i = 0; i < count; i++) {
    const slh_item& it = items[i];
    Sizes s;
    if (!sizes_of(it.param, &s)) return fail(c, SLH_EINVAL, "item " + std::to_string(i) + ": unknown parameter set");
    if (it.key_slot >= c->nkeys || c->key_param[it.key_slot] != it.param)
      return fail(c, SLH_EINVAL, "item " + std::to_string(i) + ": key slot missing or of another parameter set");
    if (it.msg_len > msgs_bytes || it.msg_off > msgs_bytes - it.msg_len)
      return fail(c, SLH_EINVAL, "item " + std::to_string(i) + ": message outside the message buffer");
    if (it.msg_len && !msgs) return fail(c, SLH_EINVAL, "null message buffer");
    if (it.sig_off % 16) return fail(c, SLH_EINVAL, "item " + std::to_string(i) + ": signature offset not 16-byte aligned");
    if (s.sig > sigs_bytes || it.sig_off > sigs_bytes - s.sig)
      return fail(c, SLH_EINVAL, "item " + std::to_string(i) + ": signature outside the signature buffer");
    ranges.emplace_back(it.sig_off, it.sig_off + s.sig);
    per[it.param]++;
  }
  std::sort(ranges.begin(), ranges.end());
  for (size_t i = 1; i < ranges.size(); i++)
    if (ranges[i].first < ranges[i - 1].second) return fail(c, SLH_EINVAL, "signature ranges overlap");
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool graph = (mode & SLH_MODE_GRAPH) != 0;
  // the pinned staging copy of the items may still be read by the previous call
  if (c->pending) HIPCHK(c, hipEventSynchronize(c->done));
  if (c->staging_cap < count) {
    drop_graphs(c);
    if (c->staging) HIPCHK(c, hipHostFree(c->staging));
    c->staging = nullptr;
    c->staging_cap = 0;
    if (hipHostMalloc(&c->staging, size_t(count) * sizeof(DevItem)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, SLH_ENOMEM, "pinned staging allocation failed");
    }
    c->staging_cap = count;
  }
  size_t start[kSets + 1] = {}, fill[kSets + 1] = {};
  for (int p = 2; p <= kSets; p++) start[p] = start[p - 1] + per[p - 1];
  for (uint32_t i = 0; i < count; i++) {
    const slh_item& it = items[i];
    DevItem& d = c->staging[start[it.param] + fill[it.param]++];
    d.param = it.param; d.key_slot = it.key_slot; d.msg_off = it.msg_off; d.msg_len = it.msg_len;
    d.sig_off = it.sig_off;
    d.rnd_off = rnd ? rnd[i] : kNoRnd;
  }
  // working memory: the budget is shared by the parameter sets the context
  // holds keys of, so that each set's share does not depend on the mix
  const uint64_t share = budget_share(c);
  size_t chunk[kSets + 1] = {};
  int rc = SLH_OK;
  for (int p = 1; p <= kSets && !rc; p++)
    if (per[p])
      rc = with_set(uint32_t(p), [&](auto id) {
        return prepare_group<decltype(id)::value>(c, per[p], mode, share, &chunk[p]);
      });
  if (rc) return rc;
  if (!graph) {
    rc = enqueue_all(c, per, start, chunk, msgs, sigs, s, mode, true);
    if (rc) return rc;
  } else {
    GraphKey key;
    std::memset(&key, 0, sizeof key);
    for (int p = 1; p <= kSets; p++) {
      key.n[p] = per[p];
      key.ws[p] = c->ws[p];
      key.ws_bytes[p] = c->ws_bytes[p];
      key.fg[p] = c->tune[p].fg;
      key.wpc[p] = c->tune[p].wgs_per_cu;
      key.keep[p] = c->tune[p].keep;
    }
    key.n[0] = mode & (SLH_MODE_FUSED | SLH_MODE_DEDUP);
    key.msgs = msgs;
    key.sigs = sigs;
    hipGraphExec_t exec = nullptr;
    for (auto& g : c->graphs)
      if (g.first == key) exec = g.second;
    if (!exec) {
      HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
      rc = enqueue_all(c, per, start, chunk, msgs, sigs, c->cap_stream, mode, false);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
      if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
      e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
      if (c->graphs.size() >= 8) {
        (void)hipGraphExecDestroy(c->graphs.front().second);
        c->graphs.erase(c->graphs.begin());
      }
      c->graphs.emplace_back(key, exec);
    }
    HIPCHK(c, hipGraphLaunch(exec, s));
  }
  HIPCHK(c, hipEventRecord(c->done, s));
  c->pending = true;
  return SLH_OK;
}

// One request of the external interface, as the encoder needs it.
struct ExtReq {
  uint32_t param, prehash, ctx_len;
  uint64_t msg_off, msg_len, ctx_off, rnd_off;
};

// Validate external requests and lay out the encode buffer: the job table,
// then per request opt_rand (if given) and M' (FIPS 205 Algorithms 22-25),
// each 16-byte aligned.  *total: bytes of the buffer.
int plan_ext(slh_ctx* c, const std::vector<ExtReq>& reqs, const uint8_t* msgs, uint64_t msgs_bytes,
             std::vector<ExtJob>* jobs, uint64_t* total) {
  const size_t count = reqs.size();
  jobs->assign(count, ExtJob{});
  uint64_t cur = up(uint64_t(count) * sizeof(ExtJob));
  auto a16 = [](uint64_t x) { return (x + 15) / 16 * 16; };
  for (size_t i = 0; i < count; i++) {
    const ExtReq& r = reqs[i];
    Sizes sz;
    const std::string at = "item " + std::to_string(i) + ": ";
    if (!sizes_of(r.param, &sz)) return fail(c, SLH_EINVAL, at + "unknown parameter set");
    if (r.msg_len > msgs_bytes || r.msg_off > msgs_bytes - r.msg_len)
      return fail(c, SLH_EINVAL, at + "message outside the message buffer");
    if (r.ctx_len > 255) return fail(c, SLH_EINVAL, at + "context string longer than 255 bytes");
    if (r.ctx_len > msgs_bytes || r.ctx_off > msgs_bytes - r.ctx_len)
      return fail(c, SLH_EINVAL, at + "context string outside the message buffer");
    if (r.prehash > SLH_PREHASH_SHA512) return fail(c, SLH_EINVAL, at + "unknown pre-hash");
    if (r.rnd_off != SLH_RND_NONE && (sz.n > msgs_bytes || r.rnd_off > msgs_bytes - sz.n))
      return fail(c, SLH_EINVAL, at + "opt_rand outside the message buffer");
    if (!msgs && (r.msg_len || r.ctx_len || r.rnd_off != SLH_RND_NONE))
      return fail(c, SLH_EINVAL, "null message buffer");
    ExtJob& J = (*jobs)[i];
    J.msg_off = r.msg_off;
    J.msg_len = r.msg_len;
    J.ctx_off = r.ctx_off;
    J.ctx_len = r.ctx_len;
    J.prehash = r.prehash;
    J.n = sz.n;
    J.rnd_in = r.rnd_off == SLH_RND_NONE ? kNoRnd : r.rnd_off;
    if (J.rnd_in != kNoRnd) {
      J.rnd_out = cur;
      cur = a16(cur + sz.n);
    }
    const uint64_t body =
        r.prehash == SLH_PREHASH_NONE ? r.msg_len : 11 + (r.prehash == SLH_PREHASH_SHA256 ? 32 : 64);
    J.out_off = cur;
    J.out_len = 2 + r.ctx_len + body;
    cur = a16(cur + J.out_len);
  }
  *total = cur;
  return SLH_OK;
}

// Encode the planned messages into the context's encode buffer on `stream`.
int launch_encode(slh_ctx* c, const std::vector<ExtJob>& jobs, uint64_t total, const uint8_t* msgs, void* stream) {
  const size_t count = jobs.size();
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // the encode buffer and its pinned job table may still be read by the last call
  if (c->pending) HIPCHK(c, hipEventSynchronize(c->done));
  if (c->xbuf_bytes < total) {
    drop_graphs(c);
    if (c->xbuf) HIPCHK(c, hipFree(c->xbuf));
    c->xbuf = nullptr;
    c->xbuf_bytes = 0;
    if (hipMalloc(&c->xbuf, total) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, SLH_ENOMEM, "hipMalloc of the encode buffer failed");
    }
    c->xbuf_bytes = total;
  }
  if (c->xjobs_cap < count) {
    if (c->xjobs) HIPCHK(c, hipHostFree(c->xjobs));
    c->xjobs = nullptr;
    c->xjobs_cap = 0;
    if (hipHostMalloc(&c->xjobs, count * sizeof(ExtJob)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, SLH_ENOMEM, "pinned job table allocation failed");
    }
    c->xjobs_cap = count;
  }
  std::memcpy(c->xjobs, jobs.data(), count * sizeof(ExtJob));
  HIPCHK(c, hipMemcpyAsync(c->xbuf, c->xjobs, count * sizeof(ExtJob), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_encode_ext, dim3(uint32_t(count)), dim3(kEncodeThreads), 0, s,
                     reinterpret_cast<const ExtJob*>(c->xbuf), msgs, c->xbuf);
  HIPCHK(c, hipGetLastError());
  return SLH_OK;
}

}  // namespace

extern "C" {

int slh_sign_batch(slh_ctx* c, const slh_item* items, uint32_t count, const uint8_t* msgs, uint64_t msgs_bytes,
                   uint8_t* sigs, uint64_t sigs_bytes, uint32_t mode, void* stream) {
  return sign_impl(c, items, nullptr, count, msgs, msgs_bytes, sigs, sigs_bytes, mode, stream);
}

int slh_sign_batch_ext(slh_ctx* c, const slh_item_ext* items, uint32_t count, const uint8_t* msgs,
                       uint64_t msgs_bytes, uint8_t* sigs, uint64_t sigs_bytes, uint32_t mode, void* stream) {
  if (!c) return fail(nullptr, SLH_EINVAL, "null context");
  if (count == 0) return SLH_OK;
  if (!items || !sigs) return fail(c, SLH_EINVAL, "null items or signature buffer");
  std::vector<ExtReq> reqs(count);
  for (uint32_t i = 0; i < count; i++) {
    const slh_item_ext& it = items[i];
    reqs[i] = ExtReq{it.param, it.prehash, it.ctx_len, it.msg_off, it.msg_len, it.ctx_off, it.rnd_off};
  }
  std::vector<ExtJob> jobs;
  uint64_t total = 0;
  int rc = plan_ext(c, reqs, msgs, msgs_bytes, &jobs, &total);
  if (rc) return rc;
  std::vector<slh_item> inner(count);
  std::vector<uint64_t> rnd(count);
  for (uint32_t i = 0; i < count; i++) {
    inner[i] = slh_item{items[i].param, items[i].key_slot, jobs[i].out_off, jobs[i].out_len, items[i].sig_off};
    rnd[i] = jobs[i].rnd_in == kNoRnd ? kNoRnd : jobs[i].rnd_out;
  }
  rc = launch_encode(c, jobs, total, msgs, stream);
  if (rc) return rc;
  return sign_impl(c, inner.data(), rnd.data(), count, c->xbuf, total, sigs, sigs_bytes, mode, stream);
}

int slh_verify_batch_ext(slh_ctx* c, const slh_verify_item_ext* items, uint32_t count, const uint8_t* msgs,
                         uint64_t msgs_bytes, const uint8_t* sigs, uint64_t sigs_bytes, const uint8_t* pks,
                         uint64_t pks_bytes, int32_t* results, void* stream) {
  if (!c) return fail(nullptr, SLH_EINVAL, "null context");
  if (count == 0) return SLH_OK;
  if (!items) return fail(c, SLH_EINVAL, "null items");
  std::vector<ExtReq> reqs(count);
  for (uint32_t i = 0; i < count; i++) {
    const slh_verify_item_ext& it = items[i];
    reqs[i] = ExtReq{it.param, it.prehash, it.ctx_len, it.msg_off, it.msg_len, it.ctx_off, SLH_RND_NONE};
  }
  std::vector<ExtJob> jobs;
  uint64_t total = 0;
  int rc = plan_ext(c, reqs, msgs, msgs_bytes, &jobs, &total);
  if (rc) return rc;
  std::vector<slh_verify_item> inner(count);
  for (uint32_t i = 0; i < count; i++)
    inner[i] = slh_verify_item{items[i].param, 0, jobs[i].out_off, jobs[i].out_len, items[i].sig_off, items[i].pk_off};
  rc = launch_encode(c, jobs, total, msgs, stream);
  if (rc) return rc;
  return slh_verify_batch(c, inner.data(), count, c->xbuf, total, sigs, sigs_bytes, pks, pks_bytes, results,
                          stream);
}

int slh_verify_batch(slh_ctx* c, const slh_verify_item* items, uint32_t count, const uint8_t* msgs,
                     uint64_t msgs_bytes, const uint8_t* sigs, uint64_t sigs_bytes, const uint8_t* pks,
                     uint64_t pks_bytes, int32_t* results, void* stream) {
  if (!c) return fail(nullptr, SLH_EINVAL, "null context");
  if (count == 0) return SLH_OK;
  if (!items || !sigs || !pks || !results) return fail(c, SLH_EINVAL, "null argument");
  size_t per[kSets + 1] = {};
  for (uint32_t i = 0; i < count; i++) {
    const slh_verify_item& it = items[i];
    Sizes s;
    if (!sizes_of(it.param, &s)) return fail(c, SLH_EINVAL, "item " + std::to_string(i) + ": unknown parameter set");
    if (it.msg_len > msgs_bytes || it.msg_off > msgs_bytes - it.msg_len || (it.msg_len && !msgs))
      return fail(c, SLH_EINVAL, "item " + std::to_string(i) + ": message outside the buffer");
    if (s.sig > sigs_bytes || it.sig_off > sigs_bytes - s.sig)
      return fail(c, SLH_EINVAL, "item " + std::to_string(i) + ": signature outside the buffer");
    if (2 * s.n > pks_bytes || it.pk_off > pks_bytes - 2 * s.n)
      return fail(c, SLH_EINVAL, "item " + std::to_string(i) + ": public key outside the buffer");
    per[it.param]++;
  }
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (c->pending) HIPCHK(c, hipEventSynchronize(c->done));
  if (c->vstage_cap < count) {
    if (c->vstage) HIPCHK(c, hipHostFree(c->vstage));
    c->vstage = nullptr;
    c->vstage_cap = 0;
    if (hipHostMalloc(&c->vstage, size_t(count) * sizeof(VerifyItem)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, SLH_ENOMEM, "pinned staging allocation failed");
    }
    c->vstage_cap = count;
  }
  const size_t need = up(size_t(count) * sizeof(VerifyItem));
  if (c->vbuf_bytes < need) {
    if (c->vbuf) HIPCHK(c, hipFree(c->vbuf));
    c->vbuf = nullptr;
    c->vbuf_bytes = 0;
    if (hipMalloc(&c->vbuf, need) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, SLH_ENOMEM, "hipMalloc of verify items failed");
    }
    c->vbuf_bytes = need;
  }
  size_t start[kSets + 1] = {}, fill[kSets + 1] = {};
  for (int p = 2; p <= kSets; p++) start[p] = start[p - 1] + per[p - 1];
  for (uint32_t i = 0; i < count; i++) {
    const slh_verify_item& it = items[i];
    c->vstage[start[it.param] + fill[it.param]++] = VerifyItem{it.msg_off, it.msg_len, it.sig_off, it.pk_off, i};
  }
  VerifyItem* d = reinterpret_cast<VerifyItem*>(c->vbuf);
  HIPCHK(c, hipMemcpyAsync(d, c->vstage, size_t(count) * sizeof(VerifyItem), hipMemcpyHostToDevice, s));
  for (int p = 1; p <= kSets; p++) {
    if (!per[p]) continue;
    with_set(uint32_t(p), [&](auto id) {
      constexpr int ID = decltype(id)::value;
      // 16 lanes per signature give 1024 signatures one wave per SIMD; below
      // kVerifyWideMax signatures 32 lanes each keep more of the chip busy
      if (per[p] <= kVerifyWideMax) {
        constexpr uint32_t sigs_per_wg = kVerifyThreads / kVerifyGroupWide;
        hipLaunchKernelGGL((k_verify<ID, kVerifyGroupWide>), dim3(uint32_t((per[p] + sigs_per_wg - 1) / sigs_per_wg)),
                           dim3(kVerifyThreads), 0, s, d + start[p], uint32_t(per[p]), msgs, sigs, pks, results);
      } else {
        constexpr uint32_t sigs_per_wg = kVerifyThreads / kVerifyGroup;
        hipLaunchKernelGGL((k_verify<ID, kVerifyGroup>), dim3(uint32_t((per[p] + sigs_per_wg - 1) / sigs_per_wg)),
                           dim3(kVerifyThreads), 0, s, d + start[p], uint32_t(per[p]), msgs, sigs, pks, results);
      }
      return 0;
    });
  }
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipEventRecord(c->done, s));
  c->pending = true;
  return SLH_OK;
}

int slh_ctx_set_tuning(slh_ctx* c, uint32_t param, const slh_tuning* t) {
  Sizes sz;
  if (!c) return fail(nullptr, SLH_EINVAL, "null context");
  if (!t || !sizes_of(param, &sz)) return fail(c, SLH_EINVAL, "unknown parameter set or null tuning");
  const uint32_t fg = t->fors_trees_per_group ? t->fors_trees_per_group : fg_default(param);
  if (!fg_ok(param, fg)) return fail(c, SLH_EINVAL, "no compiled FORS variant with that many trees per group");
  if (t->wgs_per_cu > 64) return fail(c, SLH_EINVAL, "wgs_per_cu above 64");
  if (t->keep_chains > 1) return fail(c, SLH_EINVAL, "keep_chains must be 0 or 1");
  if (c->pending) HIPCHK(c, hipEventSynchronize(c->done));
  drop_graphs(c);
  c->tune[param].fg = fg;
  c->tune[param].wgs_per_cu = t->wgs_per_cu;
  c->tune[param].keep = t->keep_chains;
  c->tune[param].split = t->split_max_blocks;
  return SLH_OK;
}

int slh_ctx_get_tuning(const slh_ctx* c, uint32_t param, slh_tuning* t) {
  Sizes sz;
  if (!c || !t || !sizes_of(param, &sz)) return fail(nullptr, SLH_EINVAL, "null argument or unknown parameter set");
  t->fors_trees_per_group = c->tune[param].fg;
  t->wgs_per_cu = c->tune[param].wgs_per_cu;
  t->keep_chains = c->tune[param].keep;
  t->split_max_blocks = c->tune[param].split;
  return SLH_OK;
}

int slh_keygen(uint32_t param, const uint8_t* seed, uint8_t* pk, uint8_t* sk) {
  if (!seed || !pk || !sk) return fail(nullptr, SLH_EINVAL, "null pointer");
  Sizes sz;
  if (!sizes_of(param, &sz)) return fail(nullptr, SLH_EINVAL, "unknown parameter set");
  return with_set(param, [&](auto id) { return keygen_impl<decltype(id)::value>(seed, pk, sk); });
}

int slh_verify(uint32_t param, const uint8_t* msg, size_t msg_len, const uint8_t* sig, size_t sig_len,
               const uint8_t* pk) {
  Sizes s;
  if (!sizes_of(param, &s)) return fail(nullptr, SLH_EINVAL, "unknown parameter set");
  if (!sig || !pk || (msg_len && !msg)) return fail(nullptr, SLH_EINVAL, "null pointer");
  if (sig_len != s.sig) return 0;
  return with_set(param, [&](auto id) { return verify_impl<decltype(id)::value>(msg, msg_len, sig, pk); });
}

}  // extern "C"
