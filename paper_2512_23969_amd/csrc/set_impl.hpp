// set_impl.hpp -- the per-parameter-set half of the host code: working-memory
// plans, the launch sequence of one batch chunk, key generation, the tree
// cache build and batched verification, as templates over the parameter set.
// Each set_<id>.hip instantiates them for one set (SLH_DEFINE_SET_OPS), so
// the twelve sets compile as separate translation units in parallel; api.hip
// reaches them through the SetOps table of ctx.hpp.
#pragma once
#include <type_traits>

#include "ctx.hpp"

namespace slh {

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


// Call f(std::integral_constant<int, LPL>) for FORS leaves per lane 2 or 4,
// f(std::integral_constant<int, FT>) for FORS workgroups of 128, 256 or 512
// lanes, f(std::integral_constant<int, NWAV>) for TREE blocks of 2, 4 or 8
// waves.
template <typename F>
void with_lpl(uint32_t lpl, F&& f) {
  if (lpl == 4) f(FgC<4>{}); else f(FgC<2>{});
}
template <typename F>
void with_ft(uint32_t ft, F&& f) {
  if (ft == 128) f(FgC<128>{}); else if (ft == 512) f(FgC<512>{}); else f(FgC<256>{});
}
template <typename F>
void with_nwav(uint32_t nwav, F&& f) {
  if (nwav == 2) f(FgC<2>{}); else if (nwav == 8) f(FgC<8>{}); else f(FgC<4>{});
}

template <typename F>
void with_fused_waves(uint32_t nwav, F&& f) {
  if (nwav == 2) f(FgC<2>{}); else f(FgC<4>{});
}

// Workgroups of the fused kernel variant that fit one CU (its persistent
// grid): the item kernel of NWAV waves, or with CHUNKS the chunk-scheduled
// kernel (four waves).
template <int ID, int FG, int LPL, int NWAV, bool CHUNKS>
int occupancy_of() {
  static int occ = -1;
  if (occ < 0) {
    int nb = 0;
    const void* k = CHUNKS ? reinterpret_cast<const void*>(&k_fused_chunks<ID, FG, LPL>)
                           : reinterpret_cast<const void*>(&k_fused<ID, FG, LPL, NWAV>);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 64 * NWAV, 0) != hipSuccess || nb < 1) nb = 1;
    occ = nb;
  }
  return occ;
}
template <int ID>
int occupancy(uint32_t fg, uint32_t lpl, uint32_t nwav, bool chunks) {
  if constexpr (!whole_trees<ID>()) {
    return 1;
  } else {
    int occ = 1;
    with_fg<ID>(fg, [&](auto fgc) {
      with_lpl(lpl, [&](auto l) {
        constexpr int FG = decltype(fgc)::value, LPL = decltype(l)::value;
        if (chunks) {
          occ = occupancy_of<ID, FG, LPL, 4, true>();
          return;
        }
        with_fused_waves(nwav, [&](auto nw) { occ = occupancy_of<ID, FG, LPL, decltype(nw)::value, false>(); });
      });
    });
    return occ;
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
  bool inorder = false;  // layers signed in order: one TREE launch per layer, WOTS+ captured
  uint32_t parts = 0;  // > 0: TREE blocks' chains split over this many workgroups (small batches)
  uint32_t fg = 8, grid = 0, ntb = 0, nfg = 0, table = 0;
  uint32_t lpl = 2, ft = kForsThreads, nwav = 4, vtree = 0, vfors = 0;  // kernel shapes and variants
  uint32_t w0 = 0;  // fused kernel: wave 0's chunks per TREE block (0 = default)
  uint32_t fwav = 4;  // fused kernel: waves per workgroup
  uint32_t bpi = 1;   // fused kernel: TREE blocks per work item
  bool fchunks = false;  // fused kernel scheduled per chains chunk (k_fused_chunks)
  size_t o_recs = 0, o_items = 0, o_stage = 0, o_spill = 0, o_roots = 0, o_queue = 0;
  size_t o_table = 0, o_rep = 0, o_ulist = 0, o_lown = 0, o_nodes = 0, o_troots = 0, o_uroots = 0, total = 0;
  static constexpr size_t stage_per_block = size_t(Q::len) * kLeavesPerBlock * Q::NW * 4;
  Plan(size_t n_, uint32_t mode, const Tuning& t, int cus)
      : n(n_),
        fused(whole_trees<ID>() && (mode & SLH_MODE_FUSED) != 0),
        dedup(whole_trees<ID>() && (mode & SLH_MODE_DEDUP) != 0),
        keep(t.keep != 0) {
    fg = t.fg ? t.fg : fg_default(ID);
    if constexpr (whole_trees<ID>()) {
      lpl = t.lpl;
      ft = t.fors_threads;
      nwav = t.tree_waves;
      vtree = t.vtree;
      vfors = t.vfors;
      w0 = t.fused_w0;
      fwav = t.fused_waves;
      bpi = t.fused_bpi;
      fchunks = t.fused_sched == SLH_FUSED_CHUNKS;
      inorder = t.inorder != 0 && !dedup;
    }
    const size_t trees = n * Q::d;
    ntb = uint32_t((trees * Q::tree_units + TPB - 1) / TPB);
    nfg = uint32_t((n * Q::k * Q::fors_units + fg - 1) / fg);
    if (inorder) {
      // per-phase path, one TREE launch per layer of n trees; nothing kept
      fused = false;
      keep = false;
      ntb = uint32_t((n + TPB - 1) / TPB);
    }
    // With few TREE blocks the batch cannot fill the chip and its time is
    // one block's chain latency: split each block's chains over up to len
    // one-wave workgroups, about 8 waves per CU in all (the per-phase path;
    // the same bytes in every mode).  Measured on MI355X, the split wins up
    // to about 1.4 blocks per CU, ties to 2 and loses above.
    const uint32_t split_max =
        t.split == SLH_SPLIT_NEVER ? 0u : (t.split ? t.split : 3u * uint32_t(cus) / 2u);
    if (ntb <= split_max && !inorder) {
      parts = std::max<uint32_t>(1u, std::min<uint32_t>(Q::len, 8u * uint32_t(cus) / std::max(1u, ntb)));
      fused = false;
    }
    fchunks = fchunks && fused;
    if (fused) {
      const uint32_t per_cu = t.wgs_per_cu ? t.wgs_per_cu : uint32_t(occupancy<ID>(fg, lpl, fwav, fchunks));
      grid = std::min<uint32_t>(per_cu * uint32_t(cus), fchunks ? ntb + nfg : (ntb + bpi - 1) / bpi + nfg);
    } else {
      grid = std::min(ntb, kMaxTreeBlocks);
    }
    o_recs = 0;
    o_items = o_recs + up(n * sizeof(WorkRec));
    o_stage = o_items + up(n * sizeof(DevItem));
    // the fused kernels double-buffer their staging per workgroup, bpi
    // blocks each (the chunk-scheduled one works on one block at a time)
    o_spill = o_stage + up(size_t(grid) * stage_per_block * (fused ? 2 * (fchunks ? 1 : bpi) : 1));
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

// Dedup buffers of a chunk (all null without dedup).
struct DedupBufs {
  DedupSlot* table = nullptr;
  uint32_t* rep = nullptr;
  uint32_t* ulist = nullptr;
  uint32_t* ucount = nullptr;
  uint32_t* lown = nullptr;
  uint32_t* nodes = nullptr;
};

// Arguments of one launch of the TREE kernel over signing trees.
struct TreeLaunch {
  uint32_t nblocks, ntrees, first, stride;
  uint8_t* sigs;
  WorkRec* recs;
  uint32_t* stage;
  uint32_t* spill;
  const DedupBufs* db;
  uint32_t* uroots;
};

// The FORS kernel of the plan's shape (trees per group, leaves per lane,
// workgroup lanes) and instruction variant.  The fast sets' instantiations
// of these two selectors compile in translation units of their own
// (set_<id>_fors.hip, set_<id>_tree.hip; SLH_EXTERN_SELECTORS).
template <int ID>
void launch_fors_sel(slh_ctx* c, const Plan<ID>& pl, uint8_t* sigs, WorkRec* recs, uint32_t* roots, hipStream_t s) {
  const uint32_t nunits = uint32_t(pl.n * P<ID>::k * P<ID>::fors_units);
  with_fg<ID>(pl.fg, [&](auto fgc) {
    constexpr int FG = decltype(fgc)::value;
    auto go = [&](auto lpl, auto ft, auto var) {
      constexpr int LPL = decltype(lpl)::value, FT = decltype(ft)::value, V = decltype(var)::value;
      hipLaunchKernelGGL((k_fors<ID, FG, LPL, FT, V>), dim3(pl.nfg), dim3(FT), 0, s, c->keys, recs, nunits, sigs,
                         roots);
    };
    if constexpr (!whole_trees<ID>()) {
      go(FgC<2>{}, FgC<kForsThreads>{}, FgC<0>{});
    } else {
      if constexpr (ID <= 3) {  // SHA2 fast sets: the instruction variants, at the default shape
        if (pl.vfors == 1) return go(FgC<2>{}, FgC<kForsThreads>{}, FgC<1>{});
        if (pl.vfors == 2) return go(FgC<2>{}, FgC<kForsThreads>{}, FgC<2>{});
      }
      with_lpl(pl.lpl, [&](auto l) { with_ft(pl.ft, [&](auto f) { go(l, f, FgC<0>{}); }); });
    }
  });
}

// The TREE kernel (signing trees) of the plan's block size and instruction
// variant; `cap`: one layer of the batch, WOTS+ captured (layers in order).
template <int ID>
void launch_tree_sel(slh_ctx* c, const Plan<ID>& pl, bool cap, const TreeLaunch& a, hipStream_t s) {
  auto go = [&](auto nw, auto var, auto cp) {
    constexpr int NWAV = decltype(nw)::value, V = decltype(var)::value;
    constexpr bool CAP = decltype(cp)::value;
    hipLaunchKernelGGL((k_tree<ID, kSignTrees, NWAV, V, CAP>), dim3(a.nblocks), dim3(64 * NWAV), 0, s, c->keys,
                       a.recs, a.ntrees, a.sigs, a.stage, a.spill, 0u, nullptr, a.db->ulist, a.db->ucount,
                       a.db->lown, a.db->nodes, a.first, a.uroots, a.stride);
  };
  if constexpr (!whole_trees<ID>()) {
    go(FgC<4>{}, FgC<0>{}, std::false_type{});
  } else {
    auto with_cap = [&](auto nw, auto var) {
      if (cap) go(nw, var, std::true_type{}); else go(nw, var, std::false_type{});
    };
    if constexpr (ID <= 3) {  // SHA2 fast sets: the instruction variants, at four waves
      if (pl.vtree == 1) return with_cap(FgC<4>{}, FgC<1>{});
      if (pl.vtree == 2) return with_cap(FgC<4>{}, FgC<2>{});
    }
    with_nwav(pl.nwav, [&](auto nw) { with_cap(nw, FgC<0>{}); });
  }
}

// The fused kernel of the plan's shape (trees per group, leaves per lane,
// waves per workgroup); the fast sets' instantiations compile in
// set_<id>_fused.hip.
template <int ID>
void launch_fused_sel(slh_ctx* c, const Plan<ID>& pl, uint8_t* sigs, WorkRec* recs, uint32_t* stage, uint32_t* spill,
                      uint32_t* roots, uint32_t* queue, const DedupBufs& db, hipStream_t s) {
  if constexpr (whole_trees<ID>()) {
    with_fg<ID>(pl.fg, [&](auto fgc) {
      with_lpl(pl.lpl, [&](auto l) {
        with_fused_waves(pl.fchunks ? 4u : pl.fwav, [&](auto nw) {
          constexpr int FG = decltype(fgc)::value, LPL = decltype(l)::value, NWAV = decltype(nw)::value;
          if (pl.fchunks) {
            if constexpr (NWAV == 4)
              hipLaunchKernelGGL((k_fused_chunks<ID, FG, LPL>), dim3(pl.grid), dim3(256), 0, s, c->keys, recs,
                                 uint32_t(pl.n), sigs, stage, spill, roots, queue, pl.ntb, pl.nfg, db.ulist,
                                 db.ucount, db.lown, db.nodes);
            return;
          }
          hipLaunchKernelGGL((k_fused<ID, FG, LPL, NWAV>), dim3(pl.grid), dim3(64 * NWAV), 0, s, c->keys, recs,
                             uint32_t(pl.n), sigs, stage, spill, roots, queue, pl.ntb, pl.nfg, db.ulist, db.ucount,
                             db.lown, db.nodes, pl.w0, pl.bpi);
        });
      });
    });
  }
}

// Enqueue one chunk on stream s with working memory at `base`.  `src` is
// the pinned host copy of the chunk's requests (uploaded into the working
// memory), or with `src_on_device` their device copy, read in place.
// `timing` is false while a graph is captured.
//   parallel layers: prelude -> FORS -> TREE (all layers) -> FORS pk, WOTS+
//   layers in order: prelude -> FORS, FORS pk -> TREE layer 0 -> ... ->
//                    TREE layer d-1 (each writes its layer's WOTS+ part)
template <int ID>
int launch_chunk(slh_ctx* c, const Plan<ID>& pl, uint8_t* base, const DevItem* src, bool src_on_device,
                 const uint8_t* msgs, uint8_t* sigs, hipStream_t s, bool timing) {
  using Q = P<ID>;
  WorkRec* recs = reinterpret_cast<WorkRec*>(base + pl.o_recs);
  const DevItem* items = src_on_device ? src : reinterpret_cast<const DevItem*>(base + pl.o_items);
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
  if (!src_on_device)
    HIPCHK(c, hipMemcpyAsync(base + pl.o_items, src, pl.n * sizeof(DevItem), hipMemcpyHostToDevice, s));
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
  const uint32_t* troots =
      Q::fors_units > 1 ? reinterpret_cast<const uint32_t*>(base + pl.o_troots) : roots;  // FORS tree roots
  if constexpr (whole_trees<ID>()) {
    if (pl.fused) {
      PhaseTimer t(c, s, SLH_PHASE_FUSED, n, timing);
      launch_fused_sel<ID>(c, pl, sigs, recs, stage, spill, roots, queue, db, s);
    }
  }
  if (!pl.fused) {
    {
      PhaseTimer t(c, s, SLH_PHASE_FORS, n, timing);
      launch_fors_sel<ID>(c, pl, sigs, recs, roots, s);
      if constexpr (Q::fors_units > 1) {
        const uint32_t nft = n * Q::k;
        hipLaunchKernelGGL((k_fors_top<ID>), dim3((nft + 63) / 64), dim3(64), 0, s, c->keys, recs, nft, sigs, roots,
                           reinterpret_cast<uint32_t*>(base + pl.o_troots));
      }
      // layers in order: layer 0 signs the FORS public key, so T_k comes first
      if (pl.inorder)
        hipLaunchKernelGGL((k_fors_pk<ID>), dim3((n + 63) / 64), dim3(64), 0, s, c->keys, recs, n, troots);
    }
    {
      PhaseTimer t(c, s, SLH_PHASE_TREE, n, timing);
      uint32_t* uroots = Q::tree_units > 1 ? reinterpret_cast<uint32_t*>(base + pl.o_uroots) : nullptr;
      if (pl.inorder) {
        // one launch per layer over the n trees of that layer (tree of
        // message m: flat id m * d + layer), at most kMaxTreeBlocks blocks
        for (uint32_t layer = 0; layer < uint32_t(Q::d); layer++)
          for (uint32_t b0 = 0; b0 < pl.ntb; b0 += kMaxTreeBlocks) {
            const uint32_t nb = std::min(kMaxTreeBlocks, pl.ntb - b0), m0 = b0 * Plan<ID>::TPB;
            const uint32_t nt = std::min(n - m0, nb * Plan<ID>::TPB);
            launch_tree_sel<ID>(c, pl, true,
                                TreeLaunch{nb, nt, layer + m0 * uint32_t(Q::d), uint32_t(Q::d), sigs, recs, stage,
                                           nullptr, &db, nullptr},
                                s);
          }
      } else {
        const uint32_t units = trees * Q::tree_units;
        // at most kMaxTreeBlocks blocks per launch, reusing the staging
        for (uint32_t b0 = 0; b0 < pl.ntb; b0 += kMaxTreeBlocks) {
          const uint32_t nb = std::min(kMaxTreeBlocks, pl.ntb - b0), first = b0 * Plan<ID>::TPB;
          const uint32_t nu = std::min(units - first, nb * Plan<ID>::TPB);
          if (pl.parts) {
            hipLaunchKernelGGL((k_tree_chains<ID, kSignTrees>), dim3(nb, pl.parts), dim3(64), 0, s, c->keys, recs,
                               nu, sigs, stage, spill, 0u, nullptr, db.ulist, db.ucount, db.lown, first, uroots);
            hipLaunchKernelGGL((k_tree_finish<ID, kSignTrees>), dim3(nb), dim3(64), 0, s, c->keys, recs, nu, sigs,
                               stage, spill, 0u, nullptr, db.ulist, db.ucount, db.lown, db.nodes, first, uroots);
          } else {
            launch_tree_sel<ID>(c, pl, false, TreeLaunch{nb, nu, first, 1u, sigs, recs, stage, spill, &db, uroots},
                                s);
          }
        }
        if constexpr (Q::tree_units > 1)
          hipLaunchKernelGGL((k_tree_top<ID, kSignTrees>), dim3((trees + 63) / 64), dim3(64), 0, s, c->keys, recs,
                             trees, sigs, 0u, nullptr, 0u, uroots);
      }
    }
  }
  if (!pl.inorder) {
    PhaseTimer t(c, s, SLH_PHASE_WOTS, n, timing);
    if constexpr (whole_trees<ID>()) {
      if (pl.dedup)
        hipLaunchKernelGGL((k_dedup_scatter<ID>), dim3((trees + 255) / 256), dim3(256), 0, s, c->keys, recs, n,
                           sigs, db.rep, db.nodes, c->cache);
    }
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

// Messages per chunk for parameter set ID within `budget` bytes (at least
// one; the caller checks that one fits).
template <int ID>
size_t chunk_size(const slh_ctx* c, size_t count, uint32_t mode, uint64_t budget) {
  const Tuning& t = c->tune[ID];
  const Plan<ID> one(1, mode, t, c->cus), big(1024, mode, t, c->cus);
  const size_t per = (big.total - one.total) / 1023 + 1;
  const size_t fixed = one.total > per ? one.total - per : 0;
  size_t chunk = budget > fixed ? (budget - fixed) / per : 1;
  chunk = std::max<size_t>(1, std::min(chunk, count));
  // the dedup table is rounded up to a power of two and the fused grid
  // saturates: shrink until the plan fits
  while (chunk > 1 && Plan<ID>(chunk, mode, t, c->cus).total > budget) chunk -= chunk / 64 + 1;
  return chunk;
}

template <int ID>
size_t plan_bytes(const slh_ctx* c, size_t n, uint32_t mode) {
  return Plan<ID>(n, mode, c->tune[ID], c->cus).total;
}

template <int ID>
int enqueue_group(slh_ctx* c, uint8_t* ws, const DevItem* items, bool on_device, size_t count, size_t chunk,
                  const uint8_t* msgs, uint8_t* sigs, hipStream_t s, uint32_t mode, bool timing) {
  for (size_t off = 0; off < count; off += chunk) {
    const size_t cnt = std::min(chunk, count - off);
    const Plan<ID> pl(cnt, mode, c->tune[ID], c->cus);
    const int rc = launch_chunk<ID>(c, pl, ws, items + off, on_device, msgs, sigs, s, timing);
    if (rc) return rc;
  }
  return SLH_OK;
}

// Key generation (FIPS 205 Algorithm 18): PK.root = root of the single XMSS
// tree of layer d-1.  Device buffer layout: DevKey (uploaded by the caller)
// | root (32 B) | unit roots | chain-end staging.
template <int ID>
struct KeygenLayout {
  using Q = P<ID>;
  static constexpr uint32_t UT = Q::tree_units;  // TREE blocks of the top tree (1 for the fast sets)
  static constexpr size_t o_root = kKeygenRootOff;
  static constexpr size_t o_uroots = o_root + 256;
  static constexpr size_t o_stage = o_uroots + ((size_t(UT) * Q::NW * 4 + 255) / 256) * 256;
  static constexpr size_t bytes = o_stage + size_t(UT) * Q::len * kLeavesPerBlock * Q::NW * 4;
};

template <int ID>
int keygen_impl(uint8_t* dev, hipStream_t s) {
  using Q = P<ID>;
  using L = KeygenLayout<ID>;
  constexpr uint32_t UT = L::UT;
  DevKey* dk = reinterpret_cast<DevKey*>(dev);
  uint32_t* root = reinterpret_cast<uint32_t*>(dev + L::o_root);
  uint32_t* uroots = reinterpret_cast<uint32_t*>(dev + L::o_uroots);
  uint32_t* stage = reinterpret_cast<uint32_t*>(dev + L::o_stage);
  hipLaunchKernelGGL(k_key_midstates, dim3(1), dim3(64), 0, s, dk, 0u, 1u);
  // one tree: its chains split over len one-wave workgroups per unit
  hipLaunchKernelGGL((k_tree_chains<ID, kKeygenTree>), dim3(UT, Q::len), dim3(64), 0, s, dk, nullptr, UT, nullptr,
                     stage, nullptr, 0u, root, nullptr, nullptr, nullptr, 0u, uroots);
  hipLaunchKernelGGL((k_tree_finish<ID, kKeygenTree>), dim3(UT), dim3(64), 0, s, dk, nullptr, UT, nullptr, stage,
                     nullptr, 0u, root, nullptr, nullptr, nullptr, nullptr, 0u, uroots);
  if constexpr (UT > 1)
    hipLaunchKernelGGL((k_tree_top<ID, kKeygenTree>), dim3(1), dim3(64), 0, s, dk, nullptr, 1u, nullptr, 0u, root,
                       0u, uroots);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SLH_OK : hip_fail(nullptr, e, "keygen launch");
}

// Build the cached upper layers of keys [first, first + count) (all of set
// ID) on stream s, and wait for them.
template <int ID>
int cache_impl(slh_ctx* c, uint32_t first, uint32_t count, uint32_t layers, hipStream_t s) {
  using Q = P<ID>;
  if constexpr (!whole_trees<ID>()) {
    return fail(c, SLH_EINVAL, "the small parameter sets have no tree cache");
  } else {
    const uint64_t per = CacheShape<ID>::trees(layers);
    const uint64_t per_bytes = per * TreeNodes<ID>::count * Q::NW * 4;
    const uint64_t need = per_bytes * count;
    if (uint64_t(count) * per >= (1ull << 31)) return fail(c, SLH_EINVAL, "too many cached trees in one call");
    if (c->cache_used + need > c->cache_bytes) {
      // grow: the captured graphs hold the old address
      const size_t nb = std::max<size_t>(c->cache_used + need, c->cache_bytes * 2);
      uint8_t* nc = nullptr;
      if (hipMalloc(&nc, nb) != hipSuccess) {
        (void)hipGetLastError();
        return fail(c, SLH_ENOMEM, "hipMalloc of the tree cache failed");
      }
      if (c->cache_used) HIPCHK(c, hipMemcpyAsync(nc, c->cache, c->cache_used, hipMemcpyDeviceToDevice, s));
      HIPCHK(c, hipStreamSynchronize(s));
      if (c->cache) HIPCHK(c, hipFree(c->cache));
      c->cache = nc;
      c->cache_bytes = nb;
      drop_graphs(c);
    }
    const uint64_t off0 = c->cache_used;
    hipLaunchKernelGGL(k_set_cache, dim3((count + 63) / 64), dim3(64), 0, s, c->keys, first, count, layers, off0,
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
      hipLaunchKernelGGL((k_tree<ID, kCacheTrees>), dim3((n + TPB - 1) / TPB), dim3(kTreeThreads), 0, s, c->keys,
                         nullptr, n, nullptr, stage, nullptr, first, nullptr, nullptr, nullptr, nullptr, nodes, t0,
                         nullptr, 1u);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(stage);
    if (e != hipSuccess) return hip_fail(c, e, "tree cache build");
    c->cache_used += need;
    for (uint32_t i = 0; i < count; i++) c->key_cached[first + i] = layers;
    return SLH_OK;
  }
}

// Batched verification of `count` items of set ID: 16 lanes per signature,
// or 32 (`wide`) for batches too small to give every SIMD a wave at 16;
// `variant`: instruction variant of the hashes (SHA2 fast sets).
template <int ID>
void verify_launch(const VerifyItem* items, uint32_t count, bool wide, uint32_t variant, const uint8_t* msgs,
                   const uint8_t* sigs, const uint8_t* pks, int* results, hipStream_t s) {
  auto go = [&](auto g, auto var) {
    constexpr int G = decltype(g)::value, V = decltype(var)::value;
    constexpr uint32_t per_wg = kVerifyThreads / G;
    hipLaunchKernelGGL((k_verify<ID, G, V>), dim3((count + per_wg - 1) / per_wg), dim3(kVerifyThreads), 0, s, items,
                       count, msgs, sigs, pks, results);
  };
  auto with_var = [&](auto g) {
    if constexpr (ID <= 3) {
      if (variant == 1) return go(g, FgC<1>{});
      if (variant == 2) return go(g, FgC<2>{});
    }
    go(g, FgC<0>{});
  };
  if (wide) with_var(FgC<kVerifyGroupWide>{}); else with_var(FgC<kVerifyGroup>{});
}

}  // namespace slh

// The SetOps table of parameter set ID (one per translation unit).  Taking
// the addresses of the launch functions instantiates them, and with them the
// kernels they launch, in both the host and the device pass; the table is
// not const, so the device pass does not emit it (it holds host addresses).
#define SLH_DEFINE_SET_OPS(ID)                                                                              \
  namespace slh {                                                                                           \
  SetOps kSetOps##ID = {&chunk_size<ID>,         &plan_bytes<ID>, &enqueue_group<ID>,                       \
                        KeygenLayout<ID>::bytes, &keygen_impl<ID>, &cache_impl<ID>,                         \
                        &verify_launch<ID>};                                                                \
  }

// The fast sets compile the FORS, TREE and fused selectors (every kernel
// shape and variant they launch) in translation units of their own: the
// set's main unit declares them (SLH_EXTERN_SELECTORS, before
// SLH_DEFINE_SET_OPS) and set_<id>_fors.hip / set_<id>_tree.hip /
// set_<id>_fused.hip instantiate them.
#define SLH_EXTERN_SELECTORS(ID)                                                                              \
  namespace slh {                                                                                           \
  extern template void launch_fors_sel<ID>(slh_ctx*, const Plan<ID>&, uint8_t*, WorkRec*, uint32_t*,         \
                                           hipStream_t);                                                     \
  extern template void launch_tree_sel<ID>(slh_ctx*, const Plan<ID>&, bool, const TreeLaunch&, hipStream_t); \
  extern template void launch_fused_sel<ID>(slh_ctx*, const Plan<ID>&, uint8_t*, WorkRec*, uint32_t*,        \
                                            uint32_t*, uint32_t*, uint32_t*, const DedupBufs&, hipStream_t); \
  extern template int occupancy<ID>(uint32_t, uint32_t, uint32_t, bool);                                     \
  }
#define SLH_DEFINE_FORS_SELECTOR(ID)                                                                         \
  namespace slh {                                                                                           \
  template void launch_fors_sel<ID>(slh_ctx*, const Plan<ID>&, uint8_t*, WorkRec*, uint32_t*, hipStream_t);  \
  }
#define SLH_DEFINE_FUSED_SELECTOR(ID)                                                                        \
  namespace slh {                                                                                           \
  template void launch_fused_sel<ID>(slh_ctx*, const Plan<ID>&, uint8_t*, WorkRec*, uint32_t*, uint32_t*,    \
                                     uint32_t*, uint32_t*, const DedupBufs&, hipStream_t);                   \
  template int occupancy<ID>(uint32_t, uint32_t, uint32_t, bool);                                            \
  }
#define SLH_DEFINE_TREE_SELECTOR(ID)                                                                         \
  namespace slh {                                                                                           \
  template void launch_tree_sel<ID>(slh_ctx*, const Plan<ID>&, bool, const TreeLaunch&, hipStream_t);        \
  }
