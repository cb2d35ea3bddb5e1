// Request server: continuous batching of covariance / S/N requests onto one
// GPU (see include/wlcov_serve.h).
//
// One worker thread owns every HIP call.  Requests wait in arrival order;
// the head request is admitted as soon as an execution slot (a stream of
// default priority) is free and its device footprint fits the arena, so a
// request that arrives while others run starts beside them and their kernels
// overlap on the device.  Device memory comes from one arena allocated at
// creation (first-fit free list on the host), so admission and release never
// call the device allocator.  Plans are cached per (n_z, l_max, precision).
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "engine.h"
#include "wlcov_serve.h"

namespace wlc {

// First-fit allocator over [0, size) in 256-byte units.
class Arena {
 public:
  explicit Arena(size_t size) : size_(size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t &off) {
    bytes = (bytes + 255) / 256 * 256;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        off = it->first;
        const size_t rest = it->second - bytes;
        const size_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        if (used_ > peak_) peak_ = used_;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
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
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  size_t size() const { return size_; }

 private:
  size_t size_, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;  // offset -> length
};

enum class State { Queued, Running, Done };

struct Request {
  wlc_request q{};
  uint64_t ticket = 0;
  std::vector<double> W;  // host copy of the kernels
  std::shared_ptr<Plan> plan;
  State state = State::Queued;
  int status = WLC_OK;
  size_t footprint = 0, off = 0;
  int slot = -1;
  double t_submit = 0, t_admit = 0, t_done = 0, snr2 = 0;
  // device pointers inside the arena
  char *ws_run = nullptr, *ws_snr = nullptr;
  double *d = nullptr, *r = nullptr, *P = nullptr, *nm = nullptr, *Wd = nullptr;
  void *C = nullptr;
  int32_t *t = nullptr;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  double *pinned_W = nullptr;    // staging for the kernels upload
  double *pinned_out = nullptr;  // [flag, snr2]
  uint64_t ticket = 0;
  bool busy = false;
};

static inline size_t a256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace wlc

using namespace wlc;

struct wlc_server_s {
  wlc_config base{};
  wlc_tables fid{};
  char *arena_base = nullptr;
  std::unique_ptr<Arena> arena;
  std::vector<Slot> slots;
  size_t w_stage_doubles = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> pending;
  std::unordered_map<uint64_t, Request> reqs;
  std::map<std::tuple<int, double, int>, std::shared_ptr<Plan>> plans;
  uint64_t next_ticket = 1;
  int64_t completed = 0;
  bool stop = false;
  std::thread worker;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  int device = 0;
  // triangles of the base configuration: a request's triangles are a prefix
  // of them (ell-bins cut from the top; the largest bin is the slowest index
  // of the triangle order), so the optional fiducial counts serve requests
  // with at most this many
  int64_t base_n_tri = 0;

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }

  // Enqueue all device work of an admitted request on its slot's stream.
  int launch(Request &R, Slot &S) {
    const Plan &p = *R.plan;
    const int64_t n = p.n_out;
    char *mem = arena_base + R.off;
    size_t o = 0;
    auto take = [&](size_t bytes) {
      char *ptr = mem + o;
      o += a256(bytes);
      return ptr;
    };
    R.ws_run = take(p.ws_run);
    R.ws_snr = take(p.ws_snr);
    R.d = (double *)take(n * 8);
    R.r = (double *)take(n * 8);
    R.t = (int32_t *)take(n * 4);
    R.C = take((size_t)n * n * (prec_f64(p.cfg.precision) ? 8 : 4));
    R.P = (double *)take((size_t)base_cfg().n_chi * base_cfg().n_k * 8);
    R.nm = (double *)take((size_t)base_cfg().n_m * 8);
    R.Wd = (double *)take(R.W.size() * 8);
    hipStream_t s = S.stream;
    std::memcpy(S.pinned_W, R.W.data(), R.W.size() * 8);
    int rc = hip_check(hipMemcpyAsync(R.Wd, S.pinned_W, R.W.size() * 8, hipMemcpyHostToDevice, s), "W upload");
    if (rc) return rc;
    launch_scale(fid.P, R.P, (int64_t)base.n_chi * base.n_k, R.q.p_scale, s);
    launch_scale(fid.n_m, R.nm, base.n_m, R.q.n_scale, s);
    wlc_tables tb = fid;
    tb.P = R.P;
    tb.n_m = R.nm;
    tb.W = R.Wd;
    rc = run_enqueue(p, tb, R.ws_run, R.d, R.r, R.C, R.t, s, nullptr, R.q.rho_mean);
    if (rc) return rc;
    int32_t *flag = nullptr;
    double *out = nullptr;
    rc = snr_enqueue(p, R.C, R.t, R.d, R.ws_snr, s, nullptr, nullptr, &flag, &out);
    if (rc) return rc;
    rc = hip_check(hipMemcpyAsync(S.pinned_out, flag, 4, hipMemcpyDeviceToHost, s), "result copy");
    if (!rc) rc = hip_check(hipMemcpyAsync(S.pinned_out + 1, out, 8, hipMemcpyDeviceToHost, s), "result copy");
    if (!rc) rc = hip_check(hipEventRecord(S.done, s), "event record");
    return rc;
  }

  const wlc_config &base_cfg() const { return base; }

  void loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      // completions
      for (Slot &S : slots) {
        if (!S.busy) continue;
        const hipError_t q = hipEventQuery(S.done);
        if (q == hipErrorNotReady) continue;
        Request &R = reqs[S.ticket];
        if (q != hipSuccess) {
          R.status = WLC_EDEVICE;
        } else {
          int32_t flag;
          std::memcpy(&flag, S.pinned_out, 4);
          R.snr2 = S.pinned_out[1];
          R.status = flag ? WLC_ENOTPD : WLC_OK;
        }
        R.t_done = now_ms();
        R.state = State::Done;
        R.slot = -1;
        S.busy = false;
        ++completed;
        cv_done.notify_all();
      }
      if (stop) {
        bool any = false;
        for (Slot &S : slots) any |= S.busy;
        if (!any) break;
      }
      // admission in arrival order
      while (!stop && !pending.empty()) {
        int free_slot = -1;
        for (size_t i = 0; i < slots.size(); ++i)
          if (!slots[i].busy) { free_slot = (int)i; break; }
        if (free_slot < 0) break;
        Request &R = reqs[pending.front()];
        size_t off = 0;
        if (!arena->alloc(R.footprint, off)) break;
        pending.pop_front();
        R.off = off;
        R.slot = free_slot;
        R.t_admit = now_ms();
        R.state = State::Running;
        Slot &S = slots[free_slot];
        S.ticket = R.ticket;
        S.busy = true;
        // a running request cannot be released, and map nodes do not move:
        // enqueue its work without holding the lock
        lk.unlock();
        const int rc = launch(R, S);
        lk.lock();
        if (rc) {
          R.status = rc;
          R.state = State::Done;
          R.t_done = now_ms();
          (void)hipStreamSynchronize(S.stream);
          S.busy = false;
          ++completed;
          cv_done.notify_all();
        }
      }
      cv_work.wait_for(lk, std::chrono::microseconds(100));
    }
  }
};

static void fill_result(const Request &R, wlc_result *res) {
  res->status = R.status;
  res->n_data = R.plan->n_out;
  res->c_elem_bytes = prec_f64(R.plan->cfg.precision) ? 8 : 4;
  res->snr2 = R.snr2;
  res->t_submit_ms = R.t_submit;
  res->t_admit_ms = R.t_admit;
  res->t_done_ms = R.t_done;
  res->d = R.d;
  res->r = R.r;
  res->C = R.C;
  res->row_exp2 = R.t;
}

extern "C" {

int wlc_server_create(const wlc_config *base, const wlc_tables *fiducial, size_t hbm_budget, int32_t max_inflight,
                      wlc_server *out) {
  if (!base || !fiducial || !out || max_inflight < 1 || max_inflight > 64 || hbm_budget < (1u << 20))
    return fail(WLC_EINVAL, "bad server arguments");
  *out = nullptr;
  if (!fiducial->chi || !fiducial->w_chi || !fiducial->k || !fiducial->m || !fiducial->w_m || !fiducial->P ||
      !fiducial->u || !fiducial->n_m)
    return fail(WLC_EINVAL, "missing fiducial table");
  auto *h = new (std::nothrow) wlc_server_s();
  if (!h) return fail(WLC_ENOMEM, "host allocation failed");
  int rc;
  h->base = *base;
  h->base.flags |= WLC_FLAG_NOCHECK;
  h->fid = *fiducial;
  {
    Plan bp;
    rc = plan_build(h->base, bp);
    if (rc) {
      delete h;
      return rc;
    }
    h->base_n_tri = bp.n_tri;
  }
  (void)hipGetDevice(&h->device);
  rc = hip_check(hipMalloc((void **)&h->arena_base, hbm_budget), "arena allocation");
  if (rc) {
    delete h;
    return rc;
  }
  h->arena.reset(new Arena(hbm_budget));
  h->w_stage_doubles = (size_t)64 * base->n_chi;
  h->slots.resize(max_inflight);
  for (Slot &S : h->slots) {
    rc = hip_check(hipStreamCreateWithFlags(&S.stream, hipStreamNonBlocking), "stream create");
    if (!rc) rc = hip_check(hipEventCreateWithFlags(&S.done, hipEventDisableTiming), "event create");
    if (!rc) rc = hip_check(hipHostMalloc((void **)&S.pinned_W, h->w_stage_doubles * 8, hipHostMallocDefault),
                            "pinned allocation");
    if (!rc) rc = hip_check(hipHostMalloc((void **)&S.pinned_out, 16, hipHostMallocDefault), "pinned allocation");
    if (rc) {
      wlc_server_destroy(h);
      return rc;
    }
  }
  h->worker = std::thread([h] { h->loop(); });
  *out = h;
  return WLC_OK;
}

int wlc_server_submit(wlc_server srv, const wlc_request *q, uint64_t *ticket) {
  if (!srv || !q || !ticket || !q->W) return fail(WLC_EINVAL, "null argument");
  if (q->n_z < 1 || q->n_z > 64 || !(q->p_scale > 0.0) || !(q->n_scale > 0.0) || !(q->rho_mean > 0.0) ||
      !prec_valid(q->precision))
    return fail(WLC_EINVAL, "bad request");
  wlc_config cfg = srv->base;
  cfg.n_z = q->n_z;
  cfg.precision = q->precision;
  cfg.ell_cut = q->ell_max;
  std::shared_ptr<Plan> plan;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    auto key = std::make_tuple(q->n_z, q->ell_max > 0.0 ? q->ell_max : 0.0, q->precision);
    auto it = srv->plans.find(key);
    if (it != srv->plans.end()) plan = it->second;
  }
  if (!plan) {
    plan = std::make_shared<Plan>();
    const int rc = plan_build(cfg, *plan);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->plans[std::make_tuple(q->n_z, q->ell_max > 0.0 ? q->ell_max : 0.0, q->precision)] = plan;
  }
  if (srv->fid.n_tri && plan->n_tri > srv->base_n_tri)
    return fail(WLC_EINVAL, "the request has more triangles than the fiducial triangle counts cover");
  const int64_t n = plan->n_out;
  const size_t foot = a256(plan->ws_run) + a256(plan->ws_snr) + 2 * a256(n * 8) + a256(n * 4) +
                      a256((size_t)n * n * (prec_f64(q->precision) ? 8 : 4)) +
                      a256((size_t)cfg.n_chi * cfg.n_k * 8) + a256((size_t)cfg.n_m * 8) +
                      a256((size_t)q->n_z * cfg.n_chi * 8);
  if (foot > srv->arena->size()) return fail(WLC_EBUSY, "request footprint exceeds the server arena");
  Request R;
  R.q = *q;
  R.W.assign(q->W, q->W + (size_t)q->n_z * cfg.n_chi);
  R.q.W = nullptr;
  R.plan = plan;
  R.footprint = foot;
  std::lock_guard<std::mutex> lk(srv->mu);
  R.t_submit = srv->now_ms();
  const uint64_t t = srv->next_ticket++;
  R.ticket = t;
  srv->reqs.emplace(t, std::move(R));
  srv->pending.push_back(t);
  *ticket = t;
  srv->cv_work.notify_all();
  return WLC_OK;
}

int wlc_server_poll(wlc_server srv, uint64_t ticket, int32_t *done, wlc_result *res) {
  if (!srv || !done) return fail(WLC_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return fail(WLC_EINVAL, "unknown ticket");
  *done = it->second.state == State::Done;
  if (*done && res) fill_result(it->second, res);
  return WLC_OK;
}

int wlc_server_wait(wlc_server srv, uint64_t ticket, wlc_result *res) {
  if (!srv) return fail(WLC_EINVAL, "null argument");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return fail(WLC_EINVAL, "unknown ticket");
  srv->cv_done.wait(lk, [&] { return it->second.state == State::Done; });
  if (res) fill_result(it->second, res);
  return WLC_OK;
}

int wlc_server_copy(wlc_server srv, uint64_t ticket, double *d, double *r, void *C, int32_t *row_exp2, void *stream) {
  if (!srv) return fail(WLC_EINVAL, "null argument");
  Request *R;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end() || it->second.state != State::Done || it->second.d == nullptr)
      return fail(WLC_EINVAL, "request not finished");
    R = &it->second;
  }
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = R->plan->n_out;
  const size_t ce = prec_f64(R->plan->cfg.precision) ? 8 : 4;
  int rc = WLC_OK;
  if (d && !rc) rc = hip_check(hipMemcpyAsync(d, R->d, n * 8, hipMemcpyDeviceToDevice, s), "copy d");
  if (r && !rc) rc = hip_check(hipMemcpyAsync(r, R->r, n * 8, hipMemcpyDeviceToDevice, s), "copy r");
  if (C && !rc) rc = hip_check(hipMemcpyAsync(C, R->C, (size_t)n * n * ce, hipMemcpyDeviceToDevice, s), "copy C");
  if (row_exp2 && !rc) rc = hip_check(hipMemcpyAsync(row_exp2, R->t, n * 4, hipMemcpyDeviceToDevice, s), "copy t");
  return rc;
}

int wlc_server_release(wlc_server srv, uint64_t ticket) {
  if (!srv) return fail(WLC_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return fail(WLC_EINVAL, "unknown ticket");
  if (it->second.state != State::Done) return fail(WLC_EBUSY, "request still queued or running");
  if (it->second.d) srv->arena->release(it->second.off, it->second.footprint);
  srv->reqs.erase(it);
  srv->cv_work.notify_all();
  return WLC_OK;
}

int wlc_server_get_stats(wlc_server srv, wlc_server_stats *out) {
  if (!srv || !out) return fail(WLC_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  *out = wlc_server_stats{};
  for (auto &kv : srv->reqs) {
    if (kv.second.state == State::Queued) ++out->queued;
    else if (kv.second.state == State::Running) ++out->running;
    else ++out->done;
  }
  out->arena_bytes = srv->arena->size();
  out->arena_used = srv->arena->used();
  out->arena_peak = srv->arena->peak();
  out->completed_total = srv->completed;
  return WLC_OK;
}

int wlc_server_destroy(wlc_server srv) {
  if (!srv) return WLC_OK;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
    srv->pending.clear();
    srv->cv_work.notify_all();
  }
  if (srv->worker.joinable()) srv->worker.join();
  for (Slot &S : srv->slots) {
    if (S.stream) {
      (void)hipStreamSynchronize(S.stream);
      (void)hipStreamDestroy(S.stream);
    }
    if (S.done) (void)hipEventDestroy(S.done);
    if (S.pinned_W) (void)hipHostFree(S.pinned_W);
    if (S.pinned_out) (void)hipHostFree(S.pinned_out);
  }
  if (srv->arena_base) (void)hipFree(srv->arena_base);
  delete srv;
  return WLC_OK;
}

}  // extern "C"
