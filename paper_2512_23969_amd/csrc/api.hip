// api.hip -- host side of the C ABI declared in include/slh.h.
//
// Validation, the device key table, the per-context working memory and the
// launch sequence of one batch: prelude -> FORS and TREE -> WOTS, per
// parameter set, in chunks that fit the context's memory budget.  The
// per-set launch code lives in set_impl.hpp (one translation unit per set);
// this file reaches it through the SetOps table.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ctx.hpp"

using namespace slh;

namespace slh {
thread_local std::string g_free_err;  // errors of the context-free calls
}

// Working memory of slh_sign_batch_noalloc: a fixed array in device memory,
// one per GPU (each device that loads this code holds its own copy).  In host
// code the name `scratch` does not denote device memory; the address of a
// device's copy comes from hipGetSymbolAddress with that device current
// (scratch_address) and is what every copy and kernel argument uses.
// Layout: the batch's requests (SLH_NOALLOC_MAX_ITEMS DevItems), then the
// working memory of one chunk.
static __device__ __align__(256) uint8_t scratch[SLH_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
constexpr size_t kScratchItemBytes = (size_t(SLH_NOALLOC_MAX_ITEMS) * sizeof(DevItem) + kAlign - 1) / kAlign * kAlign;
constexpr size_t kScratchWorkBytes = size_t(SLH_NOALLOC_SCRATCH_BYTES) - kScratchItemBytes;

std::mutex g_scratch_mu;
uint8_t* g_scratch[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up once per
// device, at the first context created on it).
int scratch_address(int device, uint8_t** out) {
  if (device < 0 || device >= kMaxDevices) return fail(nullptr, SLH_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetSymbolAddress of the no-allocation working array");
    if (!p) return fail(nullptr, SLH_EDEVICE, "no device address for the no-allocation working array");
    g_scratch[device] = static_cast<uint8_t*>(p);
  }
  *out = g_scratch[device];
  return SLH_OK;
}

}  // namespace

namespace {

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

// Validation of an external-interface batch's inner requests only checks
// that the message buffer is not null; the encode buffer it will read is
// allocated after validation.
const uint8_t kEncodeBufferStandIn = 0;

bool has_keys_of(const slh_ctx* c, int p) {
  return std::find(c->key_param.begin(), c->key_param.end(), uint32_t(p)) != c->key_param.end();
}

// Working-memory share of one parameter set: the budget split evenly over
// the sets the context holds keys of.
uint64_t budget_share(const slh_ctx* c) {
  int sets = 0;
  for (int p = 1; p <= kSets; p++) sets += has_keys_of(c, p) ? 1 : 0;
  return c->budget / uint64_t(sets ? sets : 1);
}

// Make sure parameter set p has `bytes` of working memory (waits for every
// pending call and drops captured graphs before replacing the buffer).
int ensure_ws(slh_ctx* c, int p, size_t bytes) {
  if (c->ws_bytes[p] >= bytes) return SLH_OK;
  if (int rc = wait_all(c)) return rc;
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

// Chunk size of set p for `count` requests, with its working memory allocated.
int prepare_group(slh_ctx* c, int p, size_t count, uint32_t mode, uint64_t budget, size_t* chunk) {
  const SetOps& ops = set_ops(uint32_t(p));
  *chunk = ops.chunk(c, count, mode, budget);
  return ensure_ws(c, p, ops.plan_bytes(c, *chunk, mode));
}

// Grow a pinned host array of a call slot to `count` elements.
template <class T>
int ensure_pinned(slh_ctx* c, T** buf, size_t* cap, size_t count, const char* what) {
  if (*cap >= count) return SLH_OK;
  if (*buf) HIPCHK(c, hipHostFree(*buf));
  *buf = nullptr;
  *cap = 0;
  if (hipHostMalloc(reinterpret_cast<void**>(buf), count * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(c, SLH_ENOMEM, std::string("pinned allocation failed: ") + what);
  }
  *cap = count;
  return SLH_OK;
}

// Start a call on stream s: take the slot the call two before this one used
// (waiting on the host until that call's GPU work is done, since its pinned
// copies are about to be rewritten) and order this call after the previous
// one on the GPU (they share the working memory), without waiting for it on
// the host.
int begin_call(slh_ctx* c, hipStream_t s, int* k_out) {
  const int k = c->last < 0 ? 0 : (c->last ^ 1);
  CallSlot& S = c->slot[k];
  if (S.pending) {
    HIPCHK(c, hipEventSynchronize(S.done));
    S.pending = false;
  }
  if (c->last >= 0 && c->slot[c->last].pending) HIPCHK(c, hipStreamWaitEvent(s, c->slot[c->last].done, 0));
  *k_out = k;
  return SLH_OK;
}
// End a call that holds slot k with result rc.  The slot's event is recorded
// even when the call failed part-way, since some of its work may be queued.
int finish_call(slh_ctx* c, int k, hipStream_t s, int rc) {
  const hipError_t e = hipEventRecord(c->slot[k].done, s);
  if (e == hipSuccess) {
    c->slot[k].pending = true;
    c->last = k;
  }
  if (rc) return rc;
  return e == hipSuccess ? SLH_OK : hip_fail(c, e, "hipEventRecord");
}

// Enqueue every parameter set's requests (grouped, set p at items + start[p]).
int enqueue_all(slh_ctx* c, uint8_t* const* ws, const DevItem* items, bool on_device, const size_t* per,
                const size_t* start, const size_t* chunk, const uint8_t* msgs, uint8_t* sigs, hipStream_t s,
                uint32_t mode, bool timing) {
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
    const int rc = set_ops(uint32_t(p)).enqueue(c, ws[p], items + start[p], on_device, per[p], chunk[p], msgs, sigs,
                                                b, mode, timing);
    if (rc) return rc;
    if (branches) {
      HIPCHK(c, hipEventRecord(c->join[br], b));
      HIPCHK(c, hipStreamWaitEvent(s, c->join[br], 0));
    }
  }
  return SLH_OK;
}

// Host-side validation of a signing batch; per[p] receives the number of
// requests of each parameter set.
int validate_sign(slh_ctx* c, const slh_item* items, uint32_t count, const uint8_t* msgs, uint64_t msgs_bytes,
                  uint8_t* sigs, uint64_t sigs_bytes, uint32_t mode, size_t* per) {
  if (!items || !sigs) return fail(c, SLH_EINVAL, "null items or signature buffer");
  if (mode & ~(SLH_MODE_FUSED | SLH_MODE_GRAPH | SLH_MODE_DEDUP)) return fail(c, SLH_EINVAL, "unknown mode");
  if (reinterpret_cast<uintptr_t>(sigs) % 16) return fail(c, SLH_EINVAL, "signature buffer not 16-byte aligned");
  std::vector<std::pair<uint64_t, uint64_t>>& ranges = c->ranges;
  ranges.clear();
  for (int p = 0; p <= kSets; p++) per[p] = 0;
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
  return SLH_OK;
}

// Requests grouped by parameter set (set p at out + start[p]); rnd[i] is the
// opt_rand location of request i (or null: deterministic).
void group_items(const slh_item* items, const uint64_t* rnd, uint32_t count, const size_t* per, size_t* start,
                 DevItem* out) {
  size_t fill[kSets + 1] = {};
  start[0] = 0;
  start[1] = 0;
  for (int p = 2; p <= kSets; p++) start[p] = start[p - 1] + per[p - 1];
  for (uint32_t i = 0; i < count; i++) {
    const slh_item& it = items[i];
    DevItem& d = out[start[it.param] + fill[it.param]++];
    d.param = it.param;
    d.key_slot = it.key_slot;
    d.msg_off = it.msg_off;
    d.msg_len = it.msg_len;
    d.sig_off = it.sig_off;
    d.rnd_off = rnd ? rnd[i] : kNoRnd;
  }
}

// The signing part of a call that holds slot k (validated requests).
int run_sign(slh_ctx* c, int k, const slh_item* items, const uint64_t* rnd, uint32_t count, const size_t* per,
             const uint8_t* msgs, uint8_t* sigs, uint32_t mode, hipStream_t s) {
  const bool graph = (mode & SLH_MODE_GRAPH) != 0;
  CallSlot& S = c->slot[k];
  if (S.staging_cap < count) drop_graphs(c);  // captured uploads read the old buffer
  if (int rc = ensure_pinned(c, &S.staging, &S.staging_cap, count, "sign items")) return rc;
  size_t start[kSets + 1];
  group_items(items, rnd, count, per, start, S.staging);
  // working memory: the budget is shared by the parameter sets the context
  // holds keys of, so that each set's share does not depend on the mix
  const uint64_t share = budget_share(c);
  size_t chunk[kSets + 1] = {};
  for (int p = 1; p <= kSets; p++)
    if (per[p])
      if (int rc = prepare_group(c, p, per[p], mode, share, &chunk[p])) return rc;
  if (!graph) return enqueue_all(c, c->ws, S.staging, false, per, start, chunk, msgs, sigs, s, mode, true);
  GraphKey key;
  std::memset(&key, 0, sizeof key);
  for (int p = 1; p <= kSets; p++) {
    key.n[p] = per[p];
    key.ws[p] = c->ws[p];
    key.ws_bytes[p] = c->ws_bytes[p];
    key.tune[p] = c->tune[p];
  }
  key.n[0] = mode & (SLH_MODE_FUSED | SLH_MODE_DEDUP);
  key.msgs = msgs;
  key.sigs = sigs;
  key.staging = S.staging;
  hipGraphExec_t exec = nullptr;
  for (auto& g : c->graphs)
    if (g.first == key) exec = g.second;
  if (!exec) {
    HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_all(c, c->ws, S.staging, false, per, start, chunk, msgs, sigs, c->cap_stream, mode, false);
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

// Encode the planned messages into the context's encode buffer on stream s
// (part of a call that holds slot k).
int launch_encode(slh_ctx* c, int k, const std::vector<ExtJob>& jobs, uint64_t total, const uint8_t* msgs,
                  hipStream_t s) {
  const size_t count = jobs.size();
  if (c->xbuf_bytes < total) {
    // the encode buffer may still be read by an earlier call
    if (int rc = wait_all(c)) return rc;
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
  CallSlot& S = c->slot[k];
  if (int rc = ensure_pinned(c, &S.xjobs, &S.xjobs_cap, count, "encode jobs")) return rc;
  std::memcpy(S.xjobs, jobs.data(), count * sizeof(ExtJob));
  HIPCHK(c, hipMemcpyAsync(c->xbuf, S.xjobs, count * sizeof(ExtJob), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_encode_ext, dim3(uint32_t(count)), dim3(kEncodeThreads), 0, s,
                     reinterpret_cast<const ExtJob*>(c->xbuf), msgs, c->xbuf);
  HIPCHK(c, hipGetLastError());
  return SLH_OK;
}

// Host-side validation of a verification batch; per[p] as in validate_sign.
int validate_verify(slh_ctx* c, const slh_verify_item* items, uint32_t count, const uint8_t* msgs,
                    uint64_t msgs_bytes, const uint8_t* sigs, uint64_t sigs_bytes, const uint8_t* pks,
                    uint64_t pks_bytes, const int32_t* results, size_t* per) {
  if (!items || !sigs || !pks || !results) return fail(c, SLH_EINVAL, "null argument");
  for (int p = 0; p <= kSets; p++) per[p] = 0;
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
  return SLH_OK;
}

// The verification part of a call that holds slot k (validated items).
int run_verify(slh_ctx* c, int k, const slh_verify_item* items, uint32_t count, const size_t* per,
               const uint8_t* msgs, const uint8_t* sigs, const uint8_t* pks, int32_t* results, hipStream_t s) {
  CallSlot& S = c->slot[k];
  if (int rc = ensure_pinned(c, &S.vstage, &S.vstage_cap, count, "verify items")) return rc;
  const size_t need = up(size_t(count) * sizeof(VerifyItem));
  if (c->vbuf_bytes < need) {
    // the device item copy may still be read by an earlier call
    if (int rc = wait_all(c)) return rc;
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
    S.vstage[start[it.param] + fill[it.param]++] = VerifyItem{it.msg_off, it.msg_len, it.sig_off, it.pk_off, i};
  }
  VerifyItem* d = reinterpret_cast<VerifyItem*>(c->vbuf);
  HIPCHK(c, hipMemcpyAsync(d, S.vstage, size_t(count) * sizeof(VerifyItem), hipMemcpyHostToDevice, s));
  for (int p = 1; p <= kSets; p++) {
    if (!per[p]) continue;
    // 16 lanes per signature give 1024 signatures one wave per SIMD; below
    // kVerifyWideMax signatures 32 lanes each keep more of the chip busy
    set_ops(uint32_t(p)).verify(d + start[p], uint32_t(per[p]), per[p] <= kVerifyWideMax, c->tune[p].vverify,
                                msgs, sigs, pks, results, s);
  }
  HIPCHK(c, hipGetLastError());
  return SLH_OK;
}

// Buffers of the context-free calls (slh_keygen, slh_verify) on one device:
// a stream of their own, and device and pinned host memory that grow to the
// largest request seen and are then reused, so that these calls neither
// allocate nor wait for the whole GPU once warm.  Locked while in use.
struct DevicePool {
  std::mutex mu;
  hipStream_t stream = nullptr;
  uint8_t* dev = nullptr;
  size_t dev_bytes = 0;
  uint8_t* host = nullptr;
  size_t host_bytes = 0;
};
DevicePool g_pool[kMaxDevices];

// Lock the pool of the current device and grow it to the requested sizes.
int pool_acquire(std::unique_lock<std::mutex>* lk, DevicePool** out, size_t dev_bytes, size_t host_bytes) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, SLH_EINVAL, "device index out of range");
  DevicePool& P = g_pool[dev];
  *lk = std::unique_lock<std::mutex>(P.mu);
  if (!P.stream) {
    // a non-blocking stream at the default priority
    e = hipStreamCreateWithFlags(&P.stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipStreamCreateWithFlags");
  }
  if (P.dev_bytes < dev_bytes) {
    if (P.dev) (void)hipFree(P.dev);
    P.dev = nullptr;
    P.dev_bytes = 0;
    if (hipMalloc(&P.dev, dev_bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(nullptr, SLH_ENOMEM, "device buffer allocation failed");
    }
    P.dev_bytes = dev_bytes;
  }
  if (P.host_bytes < host_bytes) {
    if (P.host) (void)hipHostFree(P.host);
    P.host = nullptr;
    P.host_bytes = 0;
    if (hipHostMalloc(reinterpret_cast<void**>(&P.host), host_bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(nullptr, SLH_ENOMEM, "pinned buffer allocation failed");
    }
    P.host_bytes = host_bytes;
  }
  *out = &P;
  return SLH_OK;
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
  for (int k = 0; k < 2 && e == hipSuccess; k++) e = hipEventCreateWithFlags(&c->slot[k].done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipMalloc(&c->dstats, 2 * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMemset(c->dstats, 0, 2 * sizeof(unsigned long long));
  // all streams at the default priority
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking);
  for (int b = 0; b < kBranches && e == hipSuccess; b++) {
    e = hipStreamCreateWithFlags(&c->branch[b], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->join[b], hipEventDisableTiming);
  }
  // what slh_sign_batch_noalloc needs on the host and the device, set up now
  int rc = e == hipSuccess ? scratch_address(device, &c->scratch) : SLH_OK;
  for (int k = 0; k < 2 && rc == SLH_OK && e == hipSuccess; k++)
    rc = ensure_pinned(c, &c->slot[k].staging, &c->slot[k].staging_cap, SLH_NOALLOC_MAX_ITEMS, "sign items");
  if (e != hipSuccess || rc != SLH_OK) {
    const std::string msg = e != hipSuccess ? std::string("context set-up: ") + hipGetErrorString(e)
                                            : (c->err.empty() ? g_free_err : c->err);
    slh_ctx_destroy(c);
    return fail(nullptr, e != hipSuccess ? SLH_EDEVICE : rc, msg);
  }
  c->ranges.reserve(SLH_NOALLOC_MAX_ITEMS);
  for (int p = 1; p <= kSets; p++) c->tune[p].fg = fg_default(uint32_t(p));
  *out = c;
  return SLH_OK;
}

int slh_ctx_destroy(slh_ctx* c) {
  if (!c) return SLH_OK;
  (void)hipSetDevice(c->device);
  (void)wait_all(c);
  for (hipStream_t s : {c->aux, c->cap_stream})
    if (s) (void)hipStreamSynchronize(s);
  for (hipStream_t s : c->branch)
    if (s) (void)hipStreamSynchronize(s);
  drop_graphs(c);
  for (int p = 0; p <= kSets; p++)
    if (c->ws[p]) (void)hipFree(c->ws[p]);
  for (int b = 0; b < kBranches; b++) {
    if (c->branch[b]) (void)hipStreamDestroy(c->branch[b]);
    if (c->join[b]) (void)hipEventDestroy(c->join[b]);
  }
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->aux) (void)hipStreamDestroy(c->aux);
  if (c->keys) (void)hipFree(c->keys);
  if (c->dstats) (void)hipFree(c->dstats);
  if (c->cache) (void)hipFree(c->cache);
  if (c->xbuf) (void)hipFree(c->xbuf);
  if (c->vbuf) (void)hipFree(c->vbuf);
  for (CallSlot& S : c->slot) {
    if (S.staging) (void)hipHostFree(S.staging);
    if (S.vstage) (void)hipHostFree(S.vstage);
    if (S.xjobs) (void)hipHostFree(S.xjobs);
    if (S.done) (void)hipEventDestroy(S.done);
  }
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
  if (int rc = wait_all(c)) return rc;
  unsigned long long h[2] = {0, 0};
  HIPCHK(c, hipMemcpyAsync(h, c->dstats, sizeof h, hipMemcpyDeviceToHost, c->aux));
  if (reset) HIPCHK(c, hipMemsetAsync(c->dstats, 0, sizeof h, c->aux));
  HIPCHK(c, hipStreamSynchronize(c->aux));
  *trees = h[0];
  *distinct = h[1];
  return SLH_OK;
}

int slh_ctx_reserve(slh_ctx* c, uint32_t count, uint32_t mode) {
  if (!c) return fail(nullptr, SLH_EINVAL, "null context");
  if (mode & ~(SLH_MODE_FUSED | SLH_MODE_GRAPH | SLH_MODE_DEDUP)) return fail(c, SLH_EINVAL, "unknown mode");
  if (count == 0) return SLH_OK;
  HIPCHK(c, hipSetDevice(c->device));
  if (int rc = wait_all(c)) return rc;
  for (CallSlot& S : c->slot) {
    if (S.staging_cap < count) drop_graphs(c);
    if (int rc = ensure_pinned(c, &S.staging, &S.staging_cap, count, "sign items")) return rc;
  }
  const uint64_t share = budget_share(c);
  size_t chunk = 0;
  for (int p = 1; p <= kSets; p++) {
    if (!has_keys_of(c, p)) continue;
    if (int rc = prepare_group(c, p, count, mode, share, &chunk)) return rc;
  }
  return SLH_OK;
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
  // the key records and the cache buffer change under the context's calls
  if (int rc = wait_all(c)) return rc;
  return set_ops(param).cache(c, first_slot, count, layers, c->aux);
}

int slh_ctx_add_keys(slh_ctx* c, uint32_t param, const uint8_t* sks, uint32_t count, uint32_t* first_slot) {
  Sizes s;
  if (!c) return fail(nullptr, SLH_EINVAL, "null context");
  if (!sizes_of(param, &s)) return fail(c, SLH_EINVAL, "unknown parameter set");
  if (!sks || !first_slot || count == 0) return fail(c, SLH_EINVAL, "null keys, null slot or zero count");
  if (uint64_t(c->nkeys) + count > (1u << 24)) return fail(c, SLH_EINVAL, "too many keys");
  HIPCHK(c, hipSetDevice(c->device));
  // captured graphs hold the key table's address (which a reallocation
  // below frees) and working-memory chunks sized for the sets that had keys
  drop_graphs(c);
  if (c->nkeys + count > c->cap) {
    if (int rc = wait_all(c)) return rc;  // calls in flight read the old table
    uint32_t ncap = std::max<uint32_t>(64, c->cap);
    while (ncap < c->nkeys + count) ncap *= 2;
    DevKey* nk = nullptr;
    if (hipMalloc(&nk, size_t(ncap) * sizeof(DevKey)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, SLH_ENOMEM, "hipMalloc of the key table failed");
    }
    if (c->keys) {
      HIPCHK(c, hipMemcpyAsync(nk, c->keys, size_t(c->nkeys) * sizeof(DevKey), hipMemcpyDeviceToDevice, c->aux));
      HIPCHK(c, hipStreamSynchronize(c->aux));
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
  HIPCHK(c, hipMemcpyAsync(c->keys + c->nkeys, hk.data(), count * sizeof(DevKey), hipMemcpyHostToDevice, c->aux));
  hipLaunchKernelGGL(k_key_midstates, dim3((count + 63) / 64), dim3(64), 0, c->aux, c->keys, c->nkeys, count);
  HIPCHK(c, hipGetLastError());
  // the keys are complete before any later call on any stream reads them
  HIPCHK(c, hipStreamSynchronize(c->aux));
  *first_slot = c->nkeys;
  c->nkeys += count;
  c->key_param.resize(c->nkeys, param);
  c->key_cached.resize(c->nkeys, 0);
  return SLH_OK;
}

int slh_sign_batch(slh_ctx* c, const slh_item* items, uint32_t count, const uint8_t* msgs, uint64_t msgs_bytes,
                   uint8_t* sigs, uint64_t sigs_bytes, uint32_t mode, void* stream) {
  if (!c) return fail(nullptr, SLH_EINVAL, "null context");
  if (count == 0) return SLH_OK;
  size_t per[kSets + 1];
  if (int rc = validate_sign(c, items, count, msgs, msgs_bytes, sigs, sigs_bytes, mode, per)) return rc;
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int k = 0;
  if (int rc = begin_call(c, s, &k)) return rc;
  return finish_call(c, k, s, run_sign(c, k, items, nullptr, count, per, msgs, sigs, mode, s));
}

int slh_sign_batch_noalloc(slh_ctx* c, const slh_item* items, uint32_t count, const uint8_t* msgs,
                           uint64_t msgs_bytes, uint8_t* sigs, uint64_t sigs_bytes, uint32_t mode, void* stream) {
  if (!c) return fail(nullptr, SLH_EINVAL, "null context");
  if (count == 0) return SLH_OK;
  if (count > SLH_NOALLOC_MAX_ITEMS)
    return fail(c, SLH_EINVAL, "more than SLH_NOALLOC_MAX_ITEMS requests in one call");
  if (mode & SLH_MODE_GRAPH) return fail(c, SLH_EINVAL, "SLH_MODE_GRAPH allocates a graph; not without allocation");
  size_t per[kSets + 1];
  if (int rc = validate_sign(c, items, count, msgs, msgs_bytes, sigs, sigs_bytes, mode, per)) return rc;
  for (int p = 1; p <= kSets; p++)
    if (per[p] && set_ops(uint32_t(p)).plan_bytes(c, 1, mode) > kScratchWorkBytes)
      return fail(c, SLH_EINVAL, "one request of parameter set " + std::to_string(p) +
                                     " needs more working memory than the no-allocation array holds in this mode");
  if (!c->scratch) return fail(c, SLH_EDEVICE, "no no-allocation working array on this device");
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int k = 0;
  if (int rc = begin_call(c, s, &k)) return rc;
  // the slot's pinned item copy was sized for SLH_NOALLOC_MAX_ITEMS at creation
  CallSlot& S = c->slot[k];
  size_t start[kSets + 1];
  group_items(items, nullptr, count, per, start, S.staging);
  DevItem* d_items = reinterpret_cast<DevItem*>(c->scratch);
  uint8_t* ws = c->scratch + kScratchItemBytes;
  int rc = SLH_OK;
  const hipError_t e = hipMemcpyAsync(d_items, S.staging, size_t(count) * sizeof(DevItem), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) rc = hip_fail(c, e, "upload of the requests");
  // one parameter set after another, each in chunks that fit the array
  for (int p = 1; p <= kSets && rc == SLH_OK; p++) {
    if (!per[p]) continue;
    const SetOps& ops = set_ops(uint32_t(p));
    const size_t chunk = ops.chunk(c, per[p], mode, kScratchWorkBytes);
    rc = ops.enqueue(c, ws, d_items + start[p], true, per[p], chunk, msgs, sigs, s, mode, false);
  }
  return finish_call(c, k, s, rc);
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
  if (int rc = plan_ext(c, reqs, msgs, msgs_bytes, &jobs, &total)) return rc;
  std::vector<slh_item> inner(count);
  std::vector<uint64_t> rnd(count);
  for (uint32_t i = 0; i < count; i++) {
    inner[i] = slh_item{items[i].param, items[i].key_slot, jobs[i].out_off, jobs[i].out_len, items[i].sig_off};
    rnd[i] = jobs[i].rnd_in == kNoRnd ? kNoRnd : jobs[i].rnd_out;
  }
  // the inner batch reads the encode buffer (allocated below, so any
  // non-null pointer stands for it here); the signature checks still apply
  size_t per[kSets + 1];
  if (int rc = validate_sign(c, inner.data(), count, &kEncodeBufferStandIn, total, sigs, sigs_bytes, mode, per))
    return rc;
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int k = 0;
  if (int rc = begin_call(c, s, &k)) return rc;
  int rc = launch_encode(c, k, jobs, total, msgs, s);
  if (!rc) rc = run_sign(c, k, inner.data(), rnd.data(), count, per, c->xbuf, sigs, mode, s);
  return finish_call(c, k, s, rc);
}

int slh_verify_batch(slh_ctx* c, const slh_verify_item* items, uint32_t count, const uint8_t* msgs,
                     uint64_t msgs_bytes, const uint8_t* sigs, uint64_t sigs_bytes, const uint8_t* pks,
                     uint64_t pks_bytes, int32_t* results, void* stream) {
  if (!c) return fail(nullptr, SLH_EINVAL, "null context");
  if (count == 0) return SLH_OK;
  size_t per[kSets + 1];
  if (int rc = validate_verify(c, items, count, msgs, msgs_bytes, sigs, sigs_bytes, pks, pks_bytes, results, per))
    return rc;
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int k = 0;
  if (int rc = begin_call(c, s, &k)) return rc;
  return finish_call(c, k, s, run_verify(c, k, items, count, per, msgs, sigs, pks, results, s));
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
  if (int rc = plan_ext(c, reqs, msgs, msgs_bytes, &jobs, &total)) return rc;
  std::vector<slh_verify_item> inner(count);
  for (uint32_t i = 0; i < count; i++)
    inner[i] = slh_verify_item{items[i].param, 0, jobs[i].out_off, jobs[i].out_len, items[i].sig_off, items[i].pk_off};
  size_t per[kSets + 1];
  if (int rc = validate_verify(c, inner.data(), count, &kEncodeBufferStandIn, total, sigs, sigs_bytes, pks,
                               pks_bytes, results, per))
    return rc;
  HIPCHK(c, hipSetDevice(c->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int k = 0;
  if (int rc = begin_call(c, s, &k)) return rc;
  int rc = launch_encode(c, k, jobs, total, msgs, s);
  if (!rc) rc = run_verify(c, k, inner.data(), count, per, c->xbuf, sigs, pks, results, s);
  return finish_call(c, k, s, rc);
}

}  // extern "C"

namespace {

uint32_t len_of(uint32_t param) {
  Sizes sz;
  return sizes_of(param, &sz) ? sz.len : 0u;
}

// Knobs of set `param` from a caller's slh_tuning (0 = default), checked
// against the compiled kernels; on error *msg says why.
bool resolve_tuning(uint32_t param, const slh_tuning& t, Tuning* out, std::string* msg) {
  Tuning r;
  r.fg = t.fors_trees_per_group ? t.fors_trees_per_group : fg_default(param);
  if (!fg_ok(param, r.fg)) return *msg = "no compiled FORS variant with that many trees per group", false;
  if (t.wgs_per_cu > 64) return *msg = "wgs_per_cu above 64", false;
  if (t.keep_chains > 1) return *msg = "keep_chains must be 0 or 1", false;
  r.wgs_per_cu = t.wgs_per_cu;
  r.keep = t.keep_chains;
  r.split = t.split_max_blocks;
  r.lpl = t.fors_leaves_per_lane ? t.fors_leaves_per_lane : 2u;
  r.fors_threads = t.fors_threads ? t.fors_threads : uint32_t(kForsThreads);
  r.tree_waves = t.tree_waves ? t.tree_waves : 4u;
  r.inorder = t.layer_order;
  r.vtree = t.variant_tree;
  r.vfors = t.variant_fors;
  r.vverify = t.variant_verify;
  if (r.lpl != 2 && r.lpl != 4) return *msg = "fors_leaves_per_lane must be 2 or 4", false;
  if (r.fors_threads != 128 && r.fors_threads != 256 && r.fors_threads != 512)
    return *msg = "fors_threads must be 128, 256 or 512", false;
  if (r.tree_waves != 2 && r.tree_waves != 4 && r.tree_waves != 8) return *msg = "tree_waves must be 2, 4 or 8", false;
  if (r.inorder > SLH_LAYERS_IN_ORDER) return *msg = "unknown layer_order", false;
  if (r.vtree > SLH_VARIANT_SPLIT_ADDS || r.vfors > SLH_VARIANT_SPLIT_ADDS || r.vverify > SLH_VARIANT_SPLIT_ADDS)
    return *msg = "unknown instruction variant", false;
  r.fused_waves = t.fused_waves ? t.fused_waves : 4u;
  if (r.fused_waves != 2 && r.fused_waves != 4) return *msg = "fused_waves must be 2 or 4", false;
  r.fused_bpi = t.fused_blocks_per_item ? t.fused_blocks_per_item : 1u;
  if (r.fused_bpi != 1 && r.fused_bpi != 2) return *msg = "fused_blocks_per_item must be 1 or 2", false;
  r.fused_w0 = t.fused_wave0_chunks;
  r.fused_sched = t.fused_schedule ? t.fused_schedule : uint32_t(SLH_FUSED_ITEMS);
  if (r.fused_sched != SLH_FUSED_ITEMS && r.fused_sched != SLH_FUSED_CHUNKS)
    return *msg = "fused_schedule must be SLH_FUSED_ITEMS or SLH_FUSED_CHUNKS", false;
  if (r.fused_sched == SLH_FUSED_CHUNKS && (r.fused_waves != 4 || r.fused_bpi != 1 || t.fused_wave0_chunks))
    return *msg = "the chunk-scheduled fused kernel has four waves and no work items (fused_waves 4, "
                  "fused_blocks_per_item and fused_wave0_chunks 0)", false;
  if (r.fused_w0 && (r.fused_w0 < 2 || r.fused_w0 > r.fused_bpi * len_of(param) - 6))
    return *msg = "fused_wave0_chunks must be 0 or 2 .. blocks per item x len - 6", false;
  if (!fast_set(param) &&
      (r.lpl != 2 || r.fors_threads != uint32_t(kForsThreads) || r.tree_waves != 4 || r.inorder || r.fused_waves != 4 ||
       r.fused_bpi != 1 || r.fused_sched != SLH_FUSED_ITEMS))
    return *msg = "the small parameter sets have the default kernel shapes and layer order only", false;
  if (!sha2_fast_set(param) && (r.vtree || r.vfors || r.vverify))
    return *msg = "instruction variants exist for the SHA2 fast sets only", false;
  if (r.vtree && r.tree_waves != 4) return *msg = "TREE instruction variants exist at tree_waves 4 only", false;
  if (r.vfors && (r.lpl != 2 || r.fors_threads != uint32_t(kForsThreads)))
    return *msg = "FORS instruction variants exist at 2 leaves per lane and 256 lanes only", false;
  *out = r;
  return true;
}

}  // namespace

extern "C" {

int slh_ctx_set_tuning(slh_ctx* c, uint32_t param, const slh_tuning* t) {
  Sizes sz;
  if (!c) return fail(nullptr, SLH_EINVAL, "null context");
  if (!t || !sizes_of(param, &sz)) return fail(c, SLH_EINVAL, "unknown parameter set or null tuning");
  Tuning r;
  std::string msg;
  if (!resolve_tuning(param, *t, &r, &msg)) return fail(c, SLH_EINVAL, msg);
  if (int rc = wait_all(c)) return rc;
  drop_graphs(c);
  c->tune[param] = r;
  return SLH_OK;
}

int slh_ctx_get_tuning(const slh_ctx* c, uint32_t param, slh_tuning* t) {
  Sizes sz;
  if (!c || !t || !sizes_of(param, &sz)) return fail(nullptr, SLH_EINVAL, "null argument or unknown parameter set");
  const Tuning& r = c->tune[param];
  *t = slh_tuning{};
  t->fors_trees_per_group = r.fg;
  t->wgs_per_cu = r.wgs_per_cu;
  t->keep_chains = r.keep;
  t->split_max_blocks = r.split;
  t->fors_leaves_per_lane = r.lpl;
  t->fors_threads = r.fors_threads;
  t->tree_waves = r.tree_waves;
  t->layer_order = r.inorder;
  t->variant_tree = r.vtree;
  t->variant_fors = r.vfors;
  t->variant_verify = r.vverify;
  t->fused_wave0_chunks = r.fused_w0;
  t->fused_waves = r.fused_waves;
  t->fused_blocks_per_item = r.fused_bpi;
  t->fused_schedule = r.fused_sched;
  return SLH_OK;
}

int slh_keygen(uint32_t param, const uint8_t* seed, uint8_t* pk, uint8_t* sk) {
  if (!seed || !pk || !sk) return fail(nullptr, SLH_EINVAL, "null pointer");
  Sizes sz;
  if (!sizes_of(param, &sz)) return fail(nullptr, SLH_EINVAL, "unknown parameter set");
  const SetOps& ops = set_ops(param);
  const uint32_t n = sz.n;
  std::unique_lock<std::mutex> lk;
  DevicePool* P = nullptr;
  if (int rc = pool_acquire(&lk, &P, ops.keygen_bytes, 512)) return rc;
  const DevKey hk = make_devkey(param, n, seed, seed + n, seed + 2 * n, nullptr);
  std::memcpy(P->host, &hk, sizeof hk);
  hipError_t e = hipMemcpyAsync(P->dev, P->host, sizeof hk, hipMemcpyHostToDevice, P->stream);
  if (e != hipSuccess) return hip_fail(nullptr, e, "keygen upload");
  if (int rc = ops.keygen(P->dev, P->stream)) return rc;
  uint32_t* hroot = reinterpret_cast<uint32_t*>(P->host + 256);
  e = hipMemcpyAsync(hroot, P->dev + kKeygenRootOff, 32, hipMemcpyDeviceToHost, P->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
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

int slh_verify(uint32_t param, const uint8_t* msg, size_t msg_len, const uint8_t* sig, size_t sig_len,
               const uint8_t* pk) {
  Sizes s;
  if (!sizes_of(param, &s)) return fail(nullptr, SLH_EINVAL, "unknown parameter set");
  if (!sig || !pk || (msg_len && !msg)) return fail(nullptr, SLH_EINVAL, "null pointer");
  if (sig_len != s.sig) return 0;
  // one buffer, uploaded by one copy: item | message | signature | pk | result
  const size_t o_msg = up(sizeof(VerifyItem));
  const size_t o_sig = o_msg + up(std::max<size_t>(msg_len, 1));
  const size_t o_pk = o_sig + up(s.sig);
  const size_t o_res = o_pk + up(2 * s.n);
  const size_t total = o_res + up(sizeof(int));
  std::unique_lock<std::mutex> lk;
  DevicePool* P = nullptr;
  if (int rc = pool_acquire(&lk, &P, total, total)) return rc;
  const VerifyItem it{0, msg_len, 0, 0, 0};
  std::memcpy(P->host, &it, sizeof it);
  if (msg_len) std::memcpy(P->host + o_msg, msg, msg_len);
  std::memcpy(P->host + o_sig, sig, s.sig);
  std::memcpy(P->host + o_pk, pk, 2 * s.n);
  hipError_t e = hipMemcpyAsync(P->dev, P->host, o_res, hipMemcpyHostToDevice, P->stream);
  if (e != hipSuccess) return hip_fail(nullptr, e, "verify upload");
  int* d_res = reinterpret_cast<int*>(P->dev + o_res);
  set_ops(param).verify(reinterpret_cast<const VerifyItem*>(P->dev), 1u, true, 0u, P->dev + o_msg, P->dev + o_sig,
                        P->dev + o_pk, d_res, P->stream);
  e = hipGetLastError();
  int* h_res = reinterpret_cast<int*>(P->host + o_res);
  *h_res = -1;
  if (e == hipSuccess) e = hipMemcpyAsync(h_res, d_res, sizeof(int), hipMemcpyDeviceToHost, P->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
  if (e != hipSuccess) return hip_fail(nullptr, e, "verify");
  return *h_res;
}

}  // extern "C"
