// ctx.hpp -- private host-side state shared by the translation units of the
// library: the signing context, error helpers, per-phase timing and the
// table of per-parameter-set entry points (one translation unit per set,
// see set_impl.hpp; compiled in parallel).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/slh.h"
#include "kernels.hpp"

namespace slh {

constexpr int kSets = 12;  // parameter sets 1..12 (slh.h SLH_SHA2_*, SLH_SHAKE_*)
// SHA2 set with the same shape (n, h, d, a, k): ids 7..12 are the SHAKE
// counterparts of ids 1..6.
constexpr uint32_t shape_of(uint32_t param) { return (param - 1) % 6 + 1; }
constexpr int kBranches = 3;  // branch streams per context
constexpr size_t kAlign = 256;
inline size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Knobs of one parameter set (see slh_tuning in slh.h), all resolved (no
// "0 = default" left).
struct Tuning {
  uint32_t fg = 0;          // FORS trees per workgroup (0 = default of the set)
  uint32_t wgs_per_cu = 0;  // fused mode: persistent workgroups per CU (0 = occupancy limit)
  uint32_t keep = 1;        // keep signing-leaf chain values for the WOTS gather
  uint32_t split = 0;       // split_max_blocks (0 = 1.5 x the CU count)
  uint32_t lpl = 2;         // FORS leaves per lane
  uint32_t fors_threads = kForsThreads;  // lanes of a per-phase FORS workgroup
  uint32_t tree_waves = 4;  // waves of a per-phase TREE block
  uint32_t inorder = 0;     // layers signed in order
  uint32_t vtree = 0, vfors = 0, vverify = 0;  // SHA-2 instruction variants
  uint32_t fused_w0 = 0;  // fused kernel: wave 0's chunks per TREE block (0 = default)
  uint32_t fused_waves = 4;  // fused kernel: waves per workgroup
  uint32_t fused_bpi = 1;    // fused kernel: TREE blocks per work item
  uint32_t fused_sched = SLH_FUSED_ITEMS;  // fused kernel: items with barriers, or chunks per wave
};

struct GraphKey {
  size_t n[kSets + 1];
  const void* msgs;
  void* sigs;
  const void* staging;  // pinned item copy the captured upload reads
  uint8_t* ws[kSets + 1];
  size_t ws_bytes[kSets + 1];
  Tuning tune[kSets + 1];
  bool operator==(const GraphKey& o) const { return std::memcmp(this, &o, sizeof o) == 0; }
};

// Calls alternate between two slots.  Each slot owns the pinned host copies
// a call hands to the GPU (sign items, verify items, encode jobs) and the
// event that marks the end of the call's GPU work.  A call waits on the host
// only for the call two before it (whose slot it reuses); it is ordered after
// the previous call on the GPU with a stream wait, so the host returns while
// the previous call still runs.
struct CallSlot {
  DevItem* staging = nullptr;  // sign items, grouped by parameter set
  size_t staging_cap = 0;
  VerifyItem* vstage = nullptr;  // verify items
  size_t vstage_cap = 0;
  ExtJob* xjobs = nullptr;  // encode jobs of the external interface
  size_t xjobs_cap = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
};

}  // namespace slh

struct slh_ctx {
  int device = 0;
  int cus = 0;
  uint64_t budget = 0;
  std::string err;
  slh::DevKey* keys = nullptr;
  uint32_t nkeys = 0, cap = 0;
  std::vector<uint32_t> key_param;
  uint8_t* ws[slh::kSets + 1] = {};  // working memory per parameter set
  size_t ws_bytes[slh::kSets + 1] = {};
  slh::Tuning tune[slh::kSets + 1];
  slh::CallSlot slot[2];
  int last = -1;                // slot of the most recent call (-1: none yet)
  uint8_t* vbuf = nullptr;      // device copy of a verify batch's items
  size_t vbuf_bytes = 0;
  hipStream_t cap_stream = nullptr;  // stream graphs are captured on
  hipStream_t aux = nullptr;         // set-up work (key upload, tree cache)
  // concurrent branches of a mixed fused batch: the g-th parameter set with
  // work runs on branch[g % kBranches].  A few streams per context, not one
  // per set: a process has only a few hardware queues, and more streams
  // make the busy ones of different contexts (server lanes) share queues.
  hipStream_t branch[slh::kBranches] = {};
  hipEvent_t fork = nullptr, join[slh::kBranches] = {};
  std::vector<std::pair<slh::GraphKey, hipGraphExec_t>> graphs;
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
  uint8_t* xbuf = nullptr;               // device: encoded messages of the external interface
  size_t xbuf_bytes = 0;
  // device address of this GPU's slh_sign_batch_noalloc working array
  uint8_t* scratch = nullptr;
  // signature ranges of the batch being validated (reserved at creation for
  // SLH_NOALLOC_MAX_ITEMS requests, so that validating such a batch does not
  // allocate)
  std::vector<std::pair<uint64_t, uint64_t>> ranges;
};

namespace slh {

extern thread_local std::string g_free_err;  // errors of the context-free calls

inline int fail(slh_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg; else g_free_err = msg;
  return code;
}
inline int hip_fail(slh_ctx* c, hipError_t e, const char* what) {
  return fail(c, SLH_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}
#define HIPCHK(c, x)                                   \
  do {                                                 \
    hipError_t e_ = (x);                               \
    if (e_ != hipSuccess) return hip_fail((c), e_, #x); \
  } while (0)

// Wait on the host for every call of the context (before its working memory,
// tuning or graphs change).
inline int wait_all(slh_ctx* c) {
  for (CallSlot& s : c->slot)
    if (s.pending) {
      HIPCHK(c, hipEventSynchronize(s.done));
      s.pending = false;
    }
  return SLH_OK;
}

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

inline void drop_graphs(slh_ctx* c) {
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.second);
  c->graphs.clear();
}

// FORS trees per workgroup that have a compiled variant, per parameter set.
// Small sets: FORS units of 2^12 leaves, one or two per workgroup.
inline bool fg_ok(uint32_t param, uint32_t fg) {
  param = shape_of(param);
  if (param >= 4) return fg == 1 || fg == 2;
  if (param == 3) return fg == 2 || fg == 4 || fg == 8;
  return fg == 4 || fg == 8 || fg == 16;
}
inline uint32_t fg_default(uint32_t param) {
  param = shape_of(param);
  return param >= 4 ? 1u : (param == 3 ? 4u : 8u);
}
// Fast sets (whole XMSS and FORS trees): the shape knobs and in-order layers
// apply; SHA2 fast sets: the instruction variants too.
inline bool fast_set(uint32_t param) { return shape_of(param) <= 3; }
inline bool sha2_fast_set(uint32_t param) { return param <= 3; }

// Most cached layers per parameter set: at most 2^16 trees per key.
// (the small sets' trees are built in units; they are not cached)
inline uint32_t max_cache_layers(uint32_t param) {
  param = shape_of(param);
  return param >= 4 ? 0u : (param == 3 ? 4u : 6u);
}

// Entry points of one parameter set (defined in its own translation unit).
struct SetOps {
  // messages per chunk of a batch of `count` within `budget` bytes of
  // working memory, and the working memory a chunk of `n` needs
  size_t (*chunk)(const slh_ctx* c, size_t count, uint32_t mode, uint64_t budget);
  size_t (*plan_bytes)(const slh_ctx* c, size_t n, uint32_t mode);
  // enqueue `count` requests in chunks of `chunk` on stream s, working
  // memory at `ws`.  `items` is the pinned host copy of the requests, or
  // (items_on_device) their device copy, which the kernels then read in place.
  int (*enqueue)(slh_ctx* c, uint8_t* ws, const DevItem* items, bool items_on_device, size_t count, size_t chunk,
                 const uint8_t* msgs, uint8_t* sigs, hipStream_t s, uint32_t mode, bool timing);
  // key generation into device memory `dev` (keygen_bytes long; its first
  // 256 bytes hold the DevKey, which the caller uploads); PK.root as BE words
  // at dev + kKeygenRootOff.  Enqueued on s.
  size_t keygen_bytes;
  int (*keygen)(uint8_t* dev, hipStream_t s);
  int (*cache)(slh_ctx* c, uint32_t first, uint32_t count, uint32_t layers, hipStream_t s);
  void (*verify)(const VerifyItem* items, uint32_t count, bool wide, uint32_t variant, const uint8_t* msgs,
                 const uint8_t* sigs, const uint8_t* pks, int* results, hipStream_t s);
};
constexpr size_t kKeygenRootOff = 256;

extern SetOps kSetOps1, kSetOps2, kSetOps3, kSetOps4, kSetOps5, kSetOps6, kSetOps7, kSetOps8, kSetOps9,
    kSetOps10, kSetOps11, kSetOps12;

inline const SetOps& set_ops(uint32_t param) {
  static SetOps* const table[kSets + 1] = {nullptr,    &kSetOps1,  &kSetOps2, &kSetOps3, &kSetOps4,
                                                 &kSetOps5,  &kSetOps6,  &kSetOps7, &kSetOps8, &kSetOps9,
                                                 &kSetOps10, &kSetOps11, &kSetOps12};
  return *table[param];
}

}  // namespace slh
