// Serving engine: continuous batching of contraction requests on one GPU.
//
// Not a method of the paper; a serving form of its contraction path.  Each
// request is a circuit + Pauli-sum observable (+ gradient).  At submit the
// request's plan is built on the host (network, greedy path, tables), or
// taken from a cache keyed by circuit/observable structure.  Admission
// reserves the plan's whole workspace (tables, parameters, every live
// intermediate) in a device pool, so a request is admitted only when its
// HBM footprint fits.  Every engine step launches, for each kernel class,
// one merged kernel that carries the current launch of every live request
// (same-level tree nodes of different requests run in the same kernel);
// requests that arrive while others run join at the next step, and a
// finished request frees its pool region and slot.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <unordered_map>

#include "exec.h"

namespace tcx {

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Pool {
  std::map<uint64_t, uint64_t> free_;  // offset -> bytes
  uint64_t size = 0;
  explicit Pool(uint64_t n = 0) : size(n) {
    if (n) free_[0] = n;
  }
  static uint64_t align(uint64_t x) { return (x + 255) & ~uint64_t(255); }
  bool alloc(uint64_t n, uint64_t* off) {
    n = align(n);
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= n) {
        *off = it->first;
        uint64_t rest = it->second - n;
        uint64_t o2 = it->first + n;
        free_.erase(it);
        if (rest) free_[o2] = rest;
        return true;
      }
    return false;
  }
  void release(uint64_t off, uint64_t n) {
    n = align(n);
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  uint64_t free_bytes() const {
    uint64_t s = 0;
    for (auto& kv : free_) s += kv.second;
    return s;
  }
};

struct Slot {
  double* host = nullptr;   // pinned: value (2) + grad (n_params)
  float* pin_params = nullptr;
  uint64_t cap_out = 0, cap_params = 0;
  hipEvent_t done = nullptr;
  bool busy = false;
};

struct Request {
  int64_t id = 0;
  double t_submit = 0, t_planned = 0, t_admit = 0, t_done = 0;
  int want_grad = 0;
  std::shared_ptr<Plan> plan;
  std::vector<float> params;
  WorkspaceLayout lay{};
  uint64_t off = 0;
  char* ws = nullptr;
  std::vector<const Launch*> seq;
  size_t cursor = 0;
  int slot = -1;
  double value = 0, value_im = 0;
  std::vector<double> grad;
  int status = TC_OK;
};

}  // namespace

struct Server {
  tc_serve_opts opts{};
  int n_cu = 256;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  char* pool_base = nullptr;
  Pool pool;
  std::vector<Slot> slots;
  std::mutex mu;
  int64_t next_id = 1;
  std::deque<std::unique_ptr<Request>> queue;
  std::vector<std::unique_ptr<Request>> active;
  std::unordered_map<int64_t, std::unique_ptr<Request>> done;
  std::unordered_map<uint64_t, std::shared_ptr<Plan>> cache;

  ~Server() {
    (void)hipSetDevice(opts.device);
    if (stream) (void)hipStreamSynchronize(stream);
    for (Slot& s : slots) {
      if (s.host) (void)hipHostFree(s.host);
      if (s.pin_params) (void)hipHostFree(s.pin_params);
      if (s.done) (void)hipEventDestroy(s.done);
    }
    if (pool_base) (void)hipFree(pool_base);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }

  void ensure_slot(Slot& s, uint64_t n_out, uint64_t n_params) {
    if (n_out > s.cap_out) {
      if (s.host) HIP_CHECK(hipHostFree(s.host));
      s.host = nullptr;
      HIP_CHECK(hipHostMalloc((void**)&s.host, n_out * sizeof(double), hipHostMallocDefault));
      s.cap_out = n_out;
    }
    if (n_params > s.cap_params) {
      if (s.pin_params) HIP_CHECK(hipHostFree(s.pin_params));
      s.pin_params = nullptr;
      HIP_CHECK(hipHostMalloc((void**)&s.pin_params, n_params * sizeof(float),
                              hipHostMallocDefault));
      s.cap_params = n_params;
    }
  }

  // finished requests: results are in their slot's pinned buffer
  void retire() {
    for (size_t i = 0; i < active.size();) {
      Request& r = *active[i];
      if (r.cursor < r.seq.size()) {
        ++i;
        continue;
      }
      Slot& s = slots[r.slot];
      hipError_t q = hipEventQuery(s.done);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      if (q != hipSuccess) {
        (void)hipGetLastError();
        r.status = TC_ERR_DEVICE;
      } else {
        r.value = s.host[0];
        r.value_im = s.host[1];
        if (r.want_grad) r.grad.assign(s.host + 2, s.host + 2 + r.plan->n_params);
      }
      r.t_done = now_s();
      pool.release(r.off, r.lay.total);
      s.busy = false;
      r.slot = -1;
      int64_t id = r.id;
      done[id] = std::move(active[i]);
      active.erase(active.begin() + i);
    }
  }

  void admit() {
    while (!queue.empty()) {
      int si = -1;
      for (size_t k = 0; k < slots.size(); ++k)
        if (!slots[k].busy) {
          si = (int)k;
          break;
        }
      if (si < 0) return;
      Request& r = *queue.front();
      uint64_t off;
      if (!pool.alloc(r.lay.total, &off)) return;  // wait for memory (FIFO)
      Slot& s = slots[si];
      ensure_slot(s, 2 + (uint64_t)r.plan->n_params, std::max<uint64_t>(1, r.params.size()));
      s.busy = true;
      r.slot = si;
      r.t_admit = now_s();
      r.off = off;
      r.ws = pool_base + off;
      upload_tables(*r.plan, r.ws, r.lay, stream);
      if (!r.params.empty()) {
        std::memcpy(s.pin_params, r.params.data(), r.params.size() * sizeof(float));
        HIP_CHECK(hipMemcpyAsync(r.ws + r.lay.params, s.pin_params,
                                 r.params.size() * sizeof(float), hipMemcpyHostToDevice,
                                 stream));
      }
      r.seq = launch_order(*r.plan, r.want_grad != 0);
      r.cursor = 0;
      active.push_back(std::move(queue.front()));
      queue.pop_front();
    }
  }

  // one merged launch per kernel class over every live request's next launch
  void launch_step() {
    static const int kinds[4] = {L_LEAF, L_LEVEL, L_ROOT, L_GRAD};
    for (int kind : kinds) {
      std::vector<SegRef> segs;
      for (auto& rp : active) {
        Request& r = *rp;
        if (r.cursor >= r.seq.size() || r.seq[r.cursor]->kind != kind) continue;
        segs.push_back(SegRef{r.plan.get(), r.ws, &r.lay, r.seq[r.cursor]});
      }
      for (size_t i = 0; i < segs.size(); i += MAX_SEG) {
        int n = (int)std::min<size_t>(MAX_SEG, segs.size() - i);
        launch_segments(kind, segs.data() + i, n, stream, n_cu, TC_PREC_C64);
      }
    }
    for (auto& rp : active) {
      Request& r = *rp;
      if (r.cursor >= r.seq.size()) continue;
      ++r.cursor;
      if (r.cursor == r.seq.size()) {
        Slot& s = slots[r.slot];
        HIP_CHECK(hipMemcpyAsync(s.host, r.ws + r.lay.value, 2 * sizeof(double),
                                 hipMemcpyDeviceToHost, stream));
        if (r.want_grad && r.plan->n_params)
          HIP_CHECK(hipMemcpyAsync(s.host + 2, r.ws + r.lay.grad,
                                   (uint64_t)r.plan->n_params * sizeof(double),
                                   hipMemcpyDeviceToHost, stream));
        HIP_CHECK(hipEventRecord(s.done, stream));
      }
    }
  }
};

}  // namespace tcx

struct tc_server {
  tcx::Server s;
};

namespace tcx {
const Network& network_of(const tc_network* n);
}

#define TC_GUARD_BEGIN try {
#define TC_GUARD_END                                               \
  }                                                                \
  catch (const tcx::Error& e) {                                    \
    tcx::set_error(e.msg);                                         \
    return e.status;                                               \
  }                                                                \
  catch (const std::bad_alloc&) {                                  \
    tcx::set_error("host allocation failed");                      \
    return TC_ERR_OUT_OF_MEMORY;                                   \
  }                                                                \
  catch (const std::exception& e) {                                \
    tcx::set_error(std::string("internal error: ") + e.what());    \
    return TC_ERR_INVALID_ARG;                                     \
  }

extern "C" {

tc_status tc_serve_create(const tc_serve_opts* opts, tc_server** out) {
  TC_GUARD_BEGIN
  if (!opts || !out) tcx::fail(TC_ERR_INVALID_ARG, "NULL argument");
  if (opts->max_active < 1 || opts->pool_bytes < 1024)
    tcx::fail(TC_ERR_INVALID_ARG, "max_active >= 1 and pool_bytes >= 1 KiB required");
  auto srv = std::make_unique<tc_server>();
  tcx::Server& S = srv->s;
  S.opts = *opts;
  if (S.opts.max_request_bytes == 0 || S.opts.max_request_bytes > S.opts.pool_bytes)
    S.opts.max_request_bytes = S.opts.pool_bytes;
  if (S.opts.path_trials < 1) S.opts.path_trials = 1;
  HIP_CHECK(hipSetDevice(S.opts.device));
  S.n_cu = tcx::device_cu_count(S.opts.device);
  if (S.opts.stream) {
    S.stream = (hipStream_t)S.opts.stream;
  } else {
    HIP_CHECK(hipStreamCreateWithFlags(&S.stream, hipStreamNonBlocking));
    S.own_stream = true;
  }
  uint64_t pb = tcx::Pool::align(S.opts.pool_bytes);
  hipError_t e = hipMalloc(&S.pool_base, pb);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    S.pool_base = nullptr;
    tcx::fail(TC_ERR_OUT_OF_MEMORY, "hipMalloc of the serving pool failed");
  }
  S.pool = tcx::Pool(pb);
  S.slots.resize(S.opts.max_active);
  for (auto& sl : S.slots)
    HIP_CHECK(hipEventCreateWithFlags(&sl.done, hipEventDisableTiming));
  *out = srv.release();
  return TC_OK;
  TC_GUARD_END
}

tc_status tc_serve_submit(tc_server* srv, const tc_circuit* circuit,
                          const tc_observable* observable, const float* params,
                          int32_t want_grad, int64_t* id) {
  TC_GUARD_BEGIN
  if (!srv || !id) tcx::fail(TC_ERR_INVALID_ARG, "NULL argument");
  tcx::Server& S = srv->s;
  auto req = std::make_unique<tcx::Request>();
  req->t_submit = tcx::now_s();
  req->want_grad = want_grad ? 1 : 0;
  // host planning happens outside the engine lock
  tc_build_opts bo{1, 1, 1};
  tcx::Network net = tcx::build_network(circuit, observable, &bo);
  uint64_t key = tcx::hash_mix(net.structure_hash, (uint64_t)req->want_grad);
  std::shared_ptr<tcx::Plan> plan;
  {
    std::lock_guard<std::mutex> g(S.mu);
    auto it = S.cache.find(key);
    if (it != S.cache.end()) plan = it->second;
  }
  if (!plan) {
    tc_path_opts po{0x5eed, S.opts.path_trials, TC_SCORE_COMBO, 0.1, 0, 0};
    tcx::Path path = tcx::greedy_path(net, po);
    auto make = [&](int32_t wide_tiles, const tcx::Network& nw, const tcx::Path& pa) {
      auto p = std::make_shared<tcx::Plan>();
      p->batch = 1;
      p->want_grad = req->want_grad;
      p->device = S.opts.device;
      p->budget = S.opts.max_request_bytes;
      p->exec_mode = 1;  // requests advance one level per engine step
      p->wide_tiles = wide_tiles;
      tcx::build_plan(*p, nw, pa);  // TOO_LARGE when over the per-request cap
      return p;
    };
    auto fit = [&](const tcx::Network& nw, const tcx::Path& pa) {
      try {
        return make(1, nw, pa);
      } catch (const tcx::Error& e) {
        // the wide tiles' operand planes may be what does not fit; the
        // 64 x 64 tiles need none
        if (e.status != TC_ERR_TOO_LARGE) throw;
        return make(0, nw, pa);
      }
    };
    try {
      plan = fit(net, path);
    } catch (const tcx::Error& e) {
      // still too large (even one term at a time, or an intermediate of
      // more than 2^31 elements): slice bonds, first until every
      // intermediate fits an eighth of the cap, then two legs further each
      // time (each sliced bond halves every intermediate that holds it, so
      // also what a term keeps for its reverse sweep), and run the slices
      // as terms (in groups)
      if (e.status != TC_ERR_TOO_LARGE) throw;
      const tcx::Error original = e;
      int32_t lg = 0;
      while (lg < 27 && (uint64_t(8) << (lg + 1)) <= S.opts.max_request_bytes / 8) ++lg;
      int32_t peak = 0;
      for (size_t t = 0; t < net.terms.size(); ++t)
        peak = std::max(peak, (int32_t)std::lround(std::log2(
                                  std::max(1.0, tcx::tree_stats(net.terms[t], path.terms[t]).size))));
      lg = std::min(lg, std::max(1, peak - 1));
      // (when slicing cannot make it fit, the request is rejected for the
      // original reason)
      for (int attempt = 0;; ++attempt) {
        tcx::Network snet;
        tcx::Path spath;
        int32_t s = 0;
        try {
          tcx::slice_network(net, path, lg, 12, snet, spath, s);  // TOO_LARGE past 12 bonds
          plan = fit(snet, spath);
          break;
        } catch (const tcx::Error& e2) {
          if (e2.status != TC_ERR_TOO_LARGE) throw;
          if (attempt >= 5 || lg <= 3 || s == 0) throw original;
          lg -= 2;
        }
      }
    }
    if (S.opts.max_request_flops > 0 &&
        plan->info.flops + plan->info.grad_flops > S.opts.max_request_flops)
      tcx::fail(TC_ERR_TOO_LARGE, "contraction needs " +
                                      std::to_string(plan->info.flops + plan->info.grad_flops) +
                                      " flops, more than the per-request limit");
    std::lock_guard<std::mutex> g(S.mu);
    if (S.cache.size() >= 512) S.cache.clear();
    S.cache.emplace(key, plan);
  }
  if (circuit->n_params > 0 && !params) tcx::fail(TC_ERR_INVALID_ARG, "params is NULL");
  req->params.assign(params, params + circuit->n_params);
  req->plan = plan;
  req->lay = tcx::workspace_layout(*plan);
  req->t_planned = tcx::now_s();
  std::lock_guard<std::mutex> g(S.mu);
  req->id = S.next_id++;
  *id = req->id;
  S.queue.push_back(std::move(req));
  return TC_OK;
  TC_GUARD_END
}

tc_status tc_serve_step(tc_server* srv, int32_t* n_live) {
  TC_GUARD_BEGIN
  if (!srv) tcx::fail(TC_ERR_INVALID_ARG, "NULL argument");
  tcx::Server& S = srv->s;
  std::lock_guard<std::mutex> g(S.mu);
  HIP_CHECK(hipSetDevice(S.opts.device));
  S.retire();
  S.admit();
  S.launch_step();
  if (n_live) *n_live = (int32_t)(S.queue.size() + S.active.size());
  return TC_OK;
  TC_GUARD_END
}

tc_status tc_serve_result_get(tc_server* srv, int64_t id, tc_serve_result* out,
                              double* grad) {
  TC_GUARD_BEGIN
  if (!srv || !out) tcx::fail(TC_ERR_INVALID_ARG, "NULL argument");
  tcx::Server& S = srv->s;
  std::lock_guard<std::mutex> g(S.mu);
  auto it = S.done.find(id);
  if (it == S.done.end()) {
    tcx::set_error("request not finished");
    return TC_ERR_BUSY;
  }
  tcx::Request& r = *it->second;
  out->id = r.id;
  out->value = r.value;
  out->value_im = r.value_im;
  out->submit_to_done_s = r.t_done - r.t_submit;
  out->want_grad = r.want_grad;
  out->status = r.status;
  out->plan_s = r.t_planned - r.t_submit;
  out->admit_to_done_s = r.t_done - r.t_admit;
  if (grad && r.want_grad)
    for (size_t k = 0; k < r.grad.size(); ++k) grad[k] = r.grad[k];
  S.done.erase(it);
  return TC_OK;
  TC_GUARD_END
}

void tc_serve_free(tc_server* srv) { delete srv; }

}  // extern "C"
