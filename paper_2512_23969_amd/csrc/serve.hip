// serve.hip -- continuous-batching signing server on top of the C ABI.
//
// Requests of any parameter set, key and message length arrive one by one.
// A scheduler keeps L "lanes" (each: its own signing context and working
// memory, stream, device message and signature buffers and pinned host
// staging).  Whenever a lane is free it admits waiting requests in arrival
// order, as many as its message and signature buffers hold (admission by
// memory budget), copies their messages in, signs them with slh_sign_batch
// and copies the signatures out, all asynchronously on the lane's stream;
// with several lanes busy, batches overlap on the GPU.  A batch is launched
// when it is full, when no lane is busy (the GPU would otherwise idle), or
// when its oldest request has waited max_wait.  A request's latency is the
// time from its arrival to the moment the scheduler sees its batch complete.
//
// The paper signs fixed batches (Section IV-A, Fig. 9: batch size trades
// throughput against overlap of transfers and compute); this serving layer is
// this library's own and not described there.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/slh.h"

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

uint32_t sig_bytes_of(uint32_t param) {
  slh_sizes s;
  return slh_params(param, &s) == SLH_OK ? s.sig_bytes : 0;
}

// Most upper layers slh_ctx_cache_keys caches for a set: 6 for the fast
// sets with h' = 3, 4 for those with h' = 4, none for the small sets.
uint32_t cache_limit(uint32_t param) {
  slh_sizes z;
  if (slh_params(param, &z) != SLH_OK) return 0;
  return z.hp == 3 ? 6u : (z.hp == 4 ? 4u : 0u);
}

struct Req {
  uint32_t param, slot;
  const uint8_t* msg;   // host bytes (owned by the caller or by `own`)
  uint64_t len;
  uint8_t* sig_dst;     // host destination or null (online mode: outbox)
  double arrival;
  uint64_t id;          // replay: index; online: caller's tag
  std::vector<uint8_t> own;
};

struct Lane {
  slh_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  uint8_t *d_msgs = nullptr, *d_sigs = nullptr, *h_msgs = nullptr, *h_sigs = nullptr;
  uint64_t msg_cap = 0, sig_cap = 0, sig_used = 0;
  std::vector<Req> reqs;
  std::vector<uint64_t> sig_off;
  std::vector<slh_item> items;
  bool busy = false;                 // launched, not yet seen complete (scheduler only)
  std::atomic<bool> draining{false};  // results being delivered by the drain thread
  double t_done = 0;
  Lane() = default;
  // the lane vector is sized once at creation and never grows, so a lane is
  // never really moved; this only satisfies std::vector's requirements
  Lane(Lane&&) noexcept {}
};

}  // namespace

struct slh_server {
  int device = 0;
  slh_serve_config cfg{};
  std::vector<Lane> lanes;
  std::vector<uint32_t> key_param;  // parameter set of every key slot (same on every lane)
  std::string err;
  // scheduler state
  std::deque<Req> pending;
  uint64_t launches = 0, launched_reqs = 0;
  // online mode
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Req> inbox;
  struct Done {
    uint64_t tag;
    uint32_t param;
    double latency;
    std::vector<uint8_t> sig;
  };
  std::deque<Done> outbox;
  std::thread worker;
  // delivery of completed lanes (copies results out) off the scheduler thread
  std::thread drainer[2];
  std::mutex dmu;
  std::condition_variable dcv;
  std::deque<Lane*> drainq;
  std::atomic<bool> drain_exit{false};
  double* drain_lat = nullptr;
  bool drain_online = false;
  std::atomic<uint64_t> delivered{0};
  std::atomic<bool> running{false};   // the online scheduler thread exists
  std::atomic<bool> stopping{false};  // drain and leave
  std::atomic<int> worker_error{0};
};

namespace {

int sfail(slh_server* s, int code, const std::string& m) {
  if (s) s->err = m;
  return code;
}

int lane_error(slh_server* s, Lane& L, int rc) {
  return sfail(s, rc, std::string("lane: ") + slh_last_error(L.ctx));
}

// Launch as many pending requests as lane L holds.  Returns the number
// launched (0 if none) or a negative error.
int launch(slh_server* s, Lane& L) {
  L.reqs.clear();
  L.items.clear();
  L.sig_off.clear();
  // moff: where the next message may start (4-byte aligned, so messages
  // stream as dwords); mend: end of the last message placed, the bytes to
  // upload (never past msg_cap, whatever its alignment)
  uint64_t moff = 0, mend = 0, soff = 0;
  while (!s->pending.empty() && L.reqs.size() < s->cfg.max_batch) {
    Req& r = s->pending.front();
    const uint64_t sb = (uint64_t(sig_bytes_of(r.param)) + 15) / 16 * 16;
    if (moff + r.len > L.msg_cap || soff + sb > L.sig_cap) break;  // admission by memory
    std::memcpy(L.h_msgs + moff, r.msg, r.len);
    L.items.push_back({r.param, r.slot, moff, r.len, soff});
    L.sig_off.push_back(soff);
    mend = moff + r.len;
    moff = (mend + 3) / 4 * 4;
    soff += sb;
    L.reqs.push_back(std::move(r));
    s->pending.pop_front();
  }
  if (L.reqs.empty()) return 0;
  L.sig_used = soff;
  if (mend && hipMemcpyAsync(L.d_msgs, L.h_msgs, mend, hipMemcpyHostToDevice, L.stream) != hipSuccess)
    return sfail(s, SLH_EDEVICE, "message upload failed");
  int rc = slh_sign_batch(L.ctx, L.items.data(), uint32_t(L.items.size()), L.d_msgs, L.msg_cap, L.d_sigs,
                          L.sig_cap, s->cfg.mode, L.stream);
  if (rc) return lane_error(s, L, rc);
  if (hipMemcpyAsync(L.h_sigs, L.d_sigs, soff, hipMemcpyDeviceToHost, L.stream) != hipSuccess)
    return sfail(s, SLH_EDEVICE, "signature download failed");
  if (hipEventRecord(L.done, L.stream) != hipSuccess) return sfail(s, SLH_EDEVICE, "event record failed");
  L.busy = true;
  s->launches++;
  s->launched_reqs += L.reqs.size();
  return int(L.reqs.size());
}

// Deliver the results of a completed lane.  `lat` (replay) receives each
// request's latency by index; online results go to the outbox.
void complete(slh_server* s, Lane& L, double t, double* lat, bool online) {
  for (size_t i = 0; i < L.reqs.size(); i++) {
    Req& r = L.reqs[i];
    const uint32_t sb = sig_bytes_of(r.param);
    if (!online) {
      std::memcpy(r.sig_dst, L.h_sigs + L.sig_off[i], sb);
      if (lat) lat[r.id] = t - r.arrival;
    } else {
      slh_server::Done d;
      d.tag = r.id;
      d.param = r.param;
      d.latency = t - r.arrival;
      d.sig.assign(L.h_sigs + L.sig_off[i], L.h_sigs + L.sig_off[i] + sb);
      std::lock_guard<std::mutex> g(s->mu);
      s->outbox.push_back(std::move(d));
    }
  }
  L.reqs.clear();
}

void drain_main(slh_server* s) {
  for (;;) {
    Lane* L = nullptr;
    {
      std::unique_lock<std::mutex> g(s->dmu);
      s->dcv.wait(g, [&] { return !s->drainq.empty() || s->drain_exit; });
      if (s->drainq.empty()) return;
      L = s->drainq.front();
      s->drainq.pop_front();
    }
    const uint64_t n = L->reqs.size();
    complete(s, *L, L->t_done, s->drain_lat, s->drain_online);
    L->draining = false;
    s->delivered += n;
  }
}

// One scheduling pass at time t: reap completed lanes, then launch on free
// lanes if the launch rule holds.  Returns the number of requests completed
// or a negative error.
int step(slh_server* s, double t, double* lat, bool online) {
  int completed = 0;
  int busy = 0;
  for (Lane& L : s->lanes) {
    if (!L.busy) continue;
    hipError_t q = hipEventQuery(L.done);
    if (q == hipSuccess) {
      // hand the results to the drain thread; the lane is free once delivered
      completed += int(L.reqs.size());
      L.busy = false;
      L.t_done = t;
      L.draining = true;
      {
        std::lock_guard<std::mutex> g(s->dmu);
        s->drain_lat = lat;
        s->drain_online = online;
        s->drainq.push_back(&L);
      }
      s->dcv.notify_one();
    } else if (q == hipErrorNotReady) {
      busy++;
    } else {
      return sfail(s, SLH_EDEVICE, std::string("lane failed: ") + hipGetErrorString(q));
    }
  }
  for (Lane& L : s->lanes) {
    if (L.busy || L.draining || s->pending.empty()) continue;
    const bool full = s->pending.size() >= s->cfg.max_batch;
    const bool idle = busy == 0;
    // with batches already in flight the GPU is fed; let the next one grow
    // longer (max_wait per busy lane) so that batches stay efficient
    const double wait = s->cfg.max_wait_us * 1e-6 * double(busy < 1 ? 1 : busy);
    const bool old = t - s->pending.front().arrival >= wait;
    const bool enough = s->cfg.min_batch && s->pending.size() >= s->cfg.min_batch;
    if (!(full || idle || old || enough)) break;
    const int rc = launch(s, L);
    if (rc < 0) return rc;
    if (rc > 0) busy++;
  }
  return completed;
}

void worker_main(slh_server* s) {
  if (hipSetDevice(s->device) != hipSuccess) {
    s->worker_error = SLH_EDEVICE;
    return;
  }
  for (;;) {
    bool inbox_empty;
    {
      std::unique_lock<std::mutex> g(s->mu);
      while (!s->inbox.empty()) {
        s->pending.push_back(std::move(s->inbox.front()));
        s->inbox.pop_front();
      }
      inbox_empty = true;
    }
    const int rc = step(s, now_s(), nullptr, true);
    if (rc < 0) {
      s->worker_error = rc;
      return;
    }
    bool any_busy = false;
    for (Lane& L : s->lanes) any_busy |= L.busy || L.draining;
    if (!any_busy && s->pending.empty()) {
      std::unique_lock<std::mutex> g(s->mu);
      if (s->stopping && s->inbox.empty()) return;  // drained
      s->cv.wait_for(g, std::chrono::microseconds(200), [&] { return !s->inbox.empty() || s->stopping; });
    } else {
      (void)inbox_empty;
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  }
}

void free_lane(Lane& L) {
  if (L.stream) (void)hipStreamSynchronize(L.stream);
  if (L.ctx) slh_ctx_destroy(L.ctx);
  if (L.d_msgs) (void)hipFree(L.d_msgs);
  if (L.d_sigs) (void)hipFree(L.d_sigs);
  if (L.h_msgs) (void)hipHostFree(L.h_msgs);
  if (L.h_sigs) (void)hipHostFree(L.h_sigs);
  if (L.done) (void)hipEventDestroy(L.done);
  if (L.stream) (void)hipStreamDestroy(L.stream);
  L.ctx = nullptr;
  L.stream = nullptr;
  L.done = nullptr;
  L.d_msgs = L.d_sigs = L.h_msgs = L.h_sigs = nullptr;
  L.busy = false;
}

}  // namespace

extern "C" {

int slh_serve_create(int device, const slh_serve_config* cfg_in, slh_server** out) {
  if (!out) return SLH_EINVAL;
  *out = nullptr;
  slh_serve_config cfg{};
  if (cfg_in) cfg = *cfg_in;
  if (cfg.lanes == 0) cfg.lanes = 4;
  if (cfg.max_batch == 0) cfg.max_batch = 4096;
  if (cfg.max_wait_us == 0) cfg.max_wait_us = 2000;
  if (cfg.msg_bytes == 0) cfg.msg_bytes = uint64_t(64) << 20;
  if (cfg.hbm_budget == 0) cfg.hbm_budget = uint64_t(4) << 30;
  if (cfg.queue_limit == 0) cfg.queue_limit = 1u << 20;
  if (cfg.lanes > 8 || cfg.max_batch > (1u << 20) || cfg.min_batch > cfg.max_batch ||
      (cfg.mode & ~(SLH_MODE_FUSED | SLH_MODE_GRAPH | SLH_MODE_DEDUP)))
    return SLH_EINVAL;
  slh_server* s = new slh_server();
  s->device = device;
  s->cfg = cfg;
  s->lanes.resize(cfg.lanes);
  const uint64_t sig_cap = uint64_t(cfg.max_batch) * ((sig_bytes_of(SLH_SHA2_256F) + 15) / 16 * 16);
  int rc = SLH_OK;
  for (Lane& L : s->lanes) {
    rc = slh_ctx_create(device, cfg.hbm_budget, &L.ctx);
    if (rc) break;
    L.msg_cap = cfg.msg_bytes;
    L.sig_cap = sig_cap;
    // the lane stream at the default priority
    if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&L.done, hipEventDisableTiming) != hipSuccess ||
        hipMalloc(&L.d_msgs, L.msg_cap) != hipSuccess || hipMalloc(&L.d_sigs, L.sig_cap) != hipSuccess ||
        hipHostMalloc(&L.h_msgs, L.msg_cap) != hipSuccess || hipHostMalloc(&L.h_sigs, L.sig_cap) != hipSuccess) {
      (void)hipGetLastError();
      rc = SLH_ENOMEM;
      break;
    }
  }
  if (rc) {
    for (Lane& L : s->lanes) free_lane(L);
    delete s;
    return rc;
  }
  for (auto& t : s->drainer) t = std::thread(drain_main, s);
  *out = s;
  return SLH_OK;
}

int slh_serve_destroy(slh_server* s) {
  if (!s) return SLH_OK;
  slh_serve_stop(s);
  {
    std::lock_guard<std::mutex> g(s->dmu);
    s->drain_exit = true;
  }
  s->dcv.notify_all();
  for (auto& t : s->drainer)
    if (t.joinable()) t.join();
  for (Lane& L : s->lanes) free_lane(L);
  delete s;
  return SLH_OK;
}

const char* slh_serve_last_error(const slh_server* s) { return s ? s->err.c_str() : ""; }

int slh_serve_add_keys(slh_server* s, uint32_t param, const uint8_t* sks, uint32_t count, uint32_t* first_slot) {
  if (!s || !first_slot) return SLH_EINVAL;
  if (s->running) return sfail(s, SLH_EBUSY, "stop the server before adding keys");
  uint32_t first = 0;
  for (size_t i = 0; i < s->lanes.size(); i++) {
    uint32_t f = 0;
    int rc = slh_ctx_add_keys(s->lanes[i].ctx, param, sks, count, &f);
    if (rc) return lane_error(s, s->lanes[i], rc);
    if (i == 0) first = f;
    else if (f != first) return sfail(s, SLH_EDEVICE, "lane key tables diverged");
    const uint32_t lim = cache_limit(param);
    if (s->cfg.cache_layers && lim) {
      rc = slh_ctx_cache_keys(s->lanes[i].ctx, f, count, std::min(s->cfg.cache_layers, lim));
      if (rc) return lane_error(s, s->lanes[i], rc);
    }
    // full-size working memory now, so that serving never allocates
    rc = slh_ctx_reserve(s->lanes[i].ctx, s->cfg.max_batch, s->cfg.mode);
    if (rc) return lane_error(s, s->lanes[i], rc);
  }
  s->key_param.resize(size_t(first) + count, param);
  *first_slot = first;
  return SLH_OK;
}

int slh_serve_set_tuning(slh_server* s, uint32_t param, const slh_tuning* t) {
  if (!s) return SLH_EINVAL;
  if (s->running) return sfail(s, SLH_EBUSY, "stop the server before tuning");
  for (Lane& L : s->lanes) {
    const int rc = slh_ctx_set_tuning(L.ctx, param, t);
    if (rc) return lane_error(s, L, rc);
  }
  return SLH_OK;
}

int slh_serve_replay(slh_server* s, const slh_serve_request* reqs, uint64_t n, const uint8_t* msgs,
                     uint64_t msgs_bytes, uint8_t* sigs, uint64_t sigs_bytes, double* latency_s, uint64_t skip,
                     slh_serve_stats* stats) {
  if (!s || (n && (!reqs || !sigs))) return SLH_EINVAL;
  if (s->running) return sfail(s, SLH_EBUSY, "replay needs the online scheduler stopped");
  for (uint64_t i = 0; i < n; i++) {
    const slh_serve_request& r = reqs[i];
    const uint32_t sb = sig_bytes_of(r.param);
    if (!sb) return sfail(s, SLH_EINVAL, "request " + std::to_string(i) + ": unknown parameter set");
    if (r.key_slot >= s->key_param.size() || s->key_param[r.key_slot] != r.param)
      return sfail(s, SLH_EINVAL, "request " + std::to_string(i) + ": key slot missing or of another parameter set");
    if (r.msg_len > msgs_bytes || r.msg_off > msgs_bytes - r.msg_len || (r.msg_len && !msgs))
      return sfail(s, SLH_EINVAL, "request " + std::to_string(i) + ": message outside the buffer");
    if (r.msg_len > s->lanes[0].msg_cap)
      return sfail(s, SLH_EINVAL, "request " + std::to_string(i) + ": message larger than a lane's buffer");
    if (sb > sigs_bytes || r.sig_off > sigs_bytes - sb)
      return sfail(s, SLH_EINVAL, "request " + std::to_string(i) + ": signature outside the buffer");
    if (i && r.arrival_s < reqs[i - 1].arrival_s) return sfail(s, SLH_EINVAL, "arrivals must not decrease");
  }
  if (hipSetDevice(s->device) != hipSuccess) return sfail(s, SLH_EDEVICE, "hipSetDevice");
  std::vector<double> lat_local;
  double* lat = latency_s;
  if (!lat) {
    lat_local.assign(n, 0.0);
    lat = lat_local.data();
  }
  const uint64_t launches0 = s->launches, reqs0 = s->launched_reqs;
  const uint64_t delivered0 = s->delivered;
  const double t0 = now_s();
  uint64_t next = 0, done = 0;
  double t_first_done = 0, t_last = t0;
  while (done < n) {
    const double t = now_s();
    while (next < n && reqs[next].arrival_s <= t - t0) {
      const slh_serve_request& r = reqs[next];
      Req q;
      q.param = r.param;
      q.slot = r.key_slot;
      q.msg = msgs + r.msg_off;
      q.len = r.msg_len;
      q.sig_dst = sigs + r.sig_off;
      q.arrival = t0 + r.arrival_s;
      q.id = next;
      s->pending.push_back(std::move(q));
      next++;
    }
    const int rc = step(s, t, lat, false);
    if (rc < 0) {
      for (Lane& L : s->lanes) (void)hipStreamSynchronize(L.stream);
      for (Lane& L : s->lanes) L.busy = false;
      while (std::any_of(s->lanes.begin(), s->lanes.end(), [](const Lane& L) { return L.draining.load(); }))
        std::this_thread::sleep_for(std::chrono::microseconds(50));
      s->pending.clear();
      return rc;
    }
    if (rc > 0) {
      done += uint64_t(rc);
      t_last = t;
      if (!t_first_done) t_first_done = t;
    } else {
      // nothing finished: wait a little (the next arrival or a completion)
      std::this_thread::sleep_for(std::chrono::microseconds(10));
    }
  }
  // every result delivered before the buffers are read
  while (s->delivered - delivered0 < n) std::this_thread::sleep_for(std::chrono::microseconds(20));
  if (stats) {
    std::vector<double> v;
    for (uint64_t i = skip; i < n; i++) v.push_back(lat[i]);
    std::sort(v.begin(), v.end());
    slh_serve_stats st{};
    st.completed = n;
    st.launches = s->launches - launches0;
    st.wall_s = t_last - t0;
    st.sig_per_s = st.wall_s > 0 ? double(n) / st.wall_s : 0;
    if (!v.empty()) {
      auto pct = [&](double p) { return v[std::min(v.size() - 1, size_t(p * double(v.size() - 1) + 0.5))]; };
      st.p50_s = pct(0.50);
      st.p99_s = pct(0.99);
      double sum = 0;
      for (double x : v) sum += x;
      st.mean_s = sum / double(v.size());
      st.max_s = v.back();
    }
    st.mean_batch = st.launches ? double(s->launched_reqs - reqs0) / double(st.launches) : 0;
    *stats = st;
  }
  return SLH_OK;
}

int slh_serve_start(slh_server* s) {
  if (!s) return SLH_EINVAL;
  if (s->running) return SLH_OK;
  s->worker_error = 0;
  s->stopping = false;
  s->running = true;
  s->worker = std::thread(worker_main, s);
  return SLH_OK;
}

// Stop the online scheduler after every submitted request has completed.
int slh_serve_stop(slh_server* s) {
  if (!s) return SLH_EINVAL;
  if (!s->running) return SLH_OK;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stopping = true;
  }
  s->cv.notify_all();
  if (s->worker.joinable()) s->worker.join();
  s->running = false;
  // after a worker error, wait for the lanes' streams before returning
  for (Lane& L : s->lanes)
    if (L.busy) (void)hipStreamSynchronize(L.stream);
  while (std::any_of(s->lanes.begin(), s->lanes.end(), [](const Lane& L) { return L.draining.load(); }))
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  return s->worker_error ? int(s->worker_error) : SLH_OK;
}

int slh_serve_submit(slh_server* s, uint32_t param, uint32_t key_slot, const uint8_t* msg, uint64_t len,
                     uint64_t tag) {
  if (!s || (len && !msg)) return SLH_EINVAL;
  if (!sig_bytes_of(param)) return SLH_EINVAL;
  if (len > s->lanes[0].msg_cap) return SLH_EINVAL;
  if (!s->running || s->stopping) return sfail(s, SLH_EINVAL, "server not started");
  // key_param only changes while the scheduler is stopped
  if (key_slot >= s->key_param.size() || s->key_param[key_slot] != param)
    return sfail(s, SLH_EINVAL, "key slot missing or of another parameter set");
  if (s->worker_error) return int(s->worker_error);
  Req q;
  q.param = param;
  q.slot = key_slot;
  q.own.assign(msg, msg + len);
  q.msg = q.own.data();
  q.len = len;
  q.sig_dst = nullptr;
  q.arrival = now_s();
  q.id = tag;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->inbox.size() >= s->cfg.queue_limit) return SLH_EBUSY;
    s->inbox.push_back(std::move(q));
    // the vector moved, so the message pointer must follow it
    s->inbox.back().msg = s->inbox.back().own.data();
  }
  s->cv.notify_one();
  return SLH_OK;
}

int slh_serve_poll(slh_server* s, uint64_t* tags, uint8_t* sigs, uint64_t sig_stride, double* latency_s,
                   uint32_t max, uint32_t* n) {
  if (!s || !n || (max && (!tags || !sigs))) return SLH_EINVAL;
  if (sig_stride < sig_bytes_of(SLH_SHA2_256F)) return SLH_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  uint32_t k = 0;
  while (k < max && !s->outbox.empty()) {
    slh_server::Done& d = s->outbox.front();
    tags[k] = d.tag;
    std::memcpy(sigs + uint64_t(k) * sig_stride, d.sig.data(), d.sig.size());
    if (latency_s) latency_s[k] = d.latency;
    s->outbox.pop_front();
    k++;
  }
  *n = k;
  return s->worker_error ? int(s->worker_error) : SLH_OK;
}

}  // extern "C"
