// Request server: continuous batching of covariance / S/N requests onto one
// GPU (see include/wlcov_serve.h).
//
// One worker thread owns every HIP call.  Requests wait in arrival order;
// the head request is admitted as soon as an execution slot (a stream of
// default priority) is free and its device footprint fits the arena.  Device
// memory comes from one arena allocated at creation (first-fit free list on
// the host), so admission and release never call the device allocator.
// Plans are cached per (n_z, l_max, precision).
//
// Each admitted request runs its table staging, quadrature, projection and
// A-build on its slot's stream.  The one-halo Gram products of bf16 and split
// bf16 requests are then batched: whenever a batch lane is idle, every
// admitted request whose A-build has been enqueued (and not yet batched)
// joins one persistent Gram launch on that lane's stream, which drains a
// device queue holding the tile work items of all of them (k_gram_bf16_batch:
// each request's items are the ones its own launch would run, so its result
// does not depend on the batch).  Requests arriving while a batch runs wait
// for the next one.  Two lanes keep small requests from waiting behind the
// Gram of a large one: products of less than LANE_SPLIT work units go to the
// narrow lane, the others to the wide lane, and the two lanes' launches run
// side by side.  After its batch, each request's split-K reduction, assembly
// and FP64 S/N (the Cholesky of the whole covariance, or of the distinct-row
// system when the request asks for the structured method) run on its own
// stream again, overlapping with other requests' work.  FP64 and FP32
// requests run their own Gram on their stream.
#include <hip/hip_runtime.h>

#include <algorithm>
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
  bool batched = false;       // Gram in a batched persistent launch
  bool back_enqueued = false; // its done event is recorded
  double t_submit = 0, t_admit = 0, t_done = 0, snr2 = 0;
  // device pointers inside the arena
  char *ws_run = nullptr, *ws_snr = nullptr;
  double *d = nullptr, *r = nullptr, *P = nullptr, *nm = nullptr, *Wd = nullptr;
  void *C = nullptr;
  int32_t *t = nullptr;
  wlc_tables tb{};
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  hipEvent_t front = nullptr;    // the request's A-build is complete
  double *pinned_W = nullptr;    // staging for the kernels upload
  double *pinned_out = nullptr;  // [flag, snr2]
  uint64_t ticket = 0;
  bool busy = false;
};

// Products below this many work units (items x k per item, about tiles x K)
// go to the narrow batch lane: at the serving grid (K = 32768, 512 tiles) that
// is every request but the largest (n_z = 7 with l_max >= 3000, and n_z = 10).
constexpr double LANE_SPLIT = 16777216.0;
constexpr int MAX_BATCH = 64;

// A batch lane: one stream for its persistent launches, the device job
// list and queue counters, and the pinned staging of the job list (rewritten
// only while the lane is idle, so the previous upload has completed).
struct Lane {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  GramJob *jobs_dev = nullptr;
  GramJob *jobs_host = nullptr;
  uint32_t *counters = nullptr;
  bool busy = false;
};

static inline size_t a256(size_t x) { return (x + 255) / 256 * 256; }

// S/N workspace of a request (0: the method is not available for the plan).
static size_t snr_bytes(const Plan &p, int method) {
  return method == WLC_SNR_STRUCTURED ? snr_structured_ws_bytes(p) : p.ws_snr;
}

}  // namespace wlc

using namespace wlc;

struct wlc_server_s {
  wlc_config base{};
  wlc_tables fid{};
  char *arena_base = nullptr;
  std::unique_ptr<Arena> arena;
  std::vector<Slot> slots;
  Lane lanes[2];
  size_t w_stage_doubles = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> pending;
  std::deque<uint64_t> gram_ready;  // admitted, A-build enqueued, waiting for a batch
  std::unordered_map<uint64_t, Request> reqs;
  std::map<std::tuple<int, double, int>, std::shared_ptr<Plan>> plans;
  uint64_t next_ticket = 1;
  int64_t completed = 0;
  int64_t n_batches = 0, n_batched = 0, max_batch = 0;
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

  // Carve the request's buffers out of its arena block, upload its kernels,
  // rescale the shared tables and enqueue everything up to the A-build (and
  // the Gram itself when it is not batched).
  int launch_front(Request &R, Slot &S) {
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
    R.ws_snr = take(snr_bytes(p, R.q.snr_method));
    R.d = (double *)take(n * 8);
    R.r = (double *)take(n * 8);
    R.t = (int32_t *)take(n * 4);
    R.C = take((size_t)n * n * (prec_f64(p.cfg.precision) ? 8 : 4));
    R.P = (double *)take((size_t)base.n_chi * base.n_k * 8);
    R.nm = (double *)take((size_t)base.n_m * 8);
    R.Wd = (double *)take(R.W.size() * 8);
    hipStream_t s = S.stream;
    std::memcpy(S.pinned_W, R.W.data(), R.W.size() * 8);
    int rc = hip_check(hipMemcpyAsync(R.Wd, S.pinned_W, R.W.size() * 8, hipMemcpyHostToDevice, s), "W upload");
    if (rc) return rc;
    launch_scale(fid.P, R.P, (int64_t)base.n_chi * base.n_k, R.q.p_scale, s);
    launch_scale(fid.n_m, R.nm, base.n_m, R.q.n_scale, s);
    R.tb = fid;
    R.tb.P = R.P;
    R.tb.n_m = R.nm;
    R.tb.W = R.Wd;
    rc = run_enqueue_front(p, R.tb, R.ws_run, s, nullptr, R.q.rho_mean);
    if (rc) return rc;
    if (R.batched) return hip_check(hipEventRecord(S.front, s), "event record");
    return run_enqueue_gram(p, R.ws_run, s, nullptr);
  }

  // Everything after the Gram product, on the request's stream: for a
  // batched request, wait for its batch and reduce its split-K slices; then
  // assembly, the FP64 Cholesky and the result copies.
  int launch_back(Request &R, Slot &S, hipEvent_t batch_done) {
    const Plan &p = *R.plan;
    hipStream_t s = S.stream;
    int rc = WLC_OK;
    if (R.batched) {
      rc = hip_check(hipStreamWaitEvent(s, batch_done, 0), "wait for the batch");
      if (!rc) rc = run_enqueue_gram_reduce(p, R.ws_run, s);
      if (rc) return rc;
    }
    rc = run_enqueue_back(p, R.tb, R.ws_run, R.d, R.r, R.C, R.t, s, nullptr);
    if (rc) return rc;
    int32_t *flag = nullptr;
    double *out = nullptr;
    if (R.q.snr_method == WLC_SNR_STRUCTURED)
      rc = snr_structured_enqueue(p, R.ws_run, R.ws_snr, s, nullptr, nullptr, &flag, &out);
    else
      rc = snr_enqueue(p, R.C, R.t, R.d, R.ws_snr, s, nullptr, nullptr, &flag, &out);
    if (rc) return rc;
    rc = hip_check(hipMemcpyAsync(S.pinned_out, flag, 4, hipMemcpyDeviceToHost, s), "result copy");
    if (!rc) rc = hip_check(hipMemcpyAsync(S.pinned_out + 1, out, 8, hipMemcpyDeviceToHost, s), "result copy");
    if (!rc) rc = hip_check(hipEventRecord(S.done, s), "event record");
    return rc;
  }

  // One persistent Gram launch over the members' work items on a lane, then
  // every member's remaining work on its own stream.  Returns an error that
  // concerns the whole batch; a member whose own work could not be enqueued
  // gets its error in err.
  int launch_batch(Lane &L, std::vector<Request *> &mem, std::vector<int> &err) {
    hipStream_t s = L.stream;
    int64_t total = 0;
    for (size_t i = 0; i < mem.size(); ++i) {
      Request &R = *mem[i];
      int rc = hip_check(hipStreamWaitEvent(s, slots[R.slot].front, 0), "wait for the A-build");
      if (rc) return rc;
      run_gram_job(*R.plan, R.ws_run, L.jobs_host[i]);
      L.jobs_host[i].item0 = total;
      total += L.jobs_host[i].n_work;
    }
    const int prec = mem[0]->plan->cfg.precision;
    int rc = hip_check(hipMemcpyAsync(L.jobs_dev, L.jobs_host, mem.size() * sizeof(GramJob), hipMemcpyHostToDevice, s),
                       "job upload");
    if (rc) return rc;
    if (launch_gram_batch(prec, L.jobs_dev, (int)mem.size(), total, L.counters, s))
      return fail(WLC_EINVAL, "no batched Gram for this precision");
    rc = hip_check(hipGetLastError(), "batched gram launch");
    if (!rc) rc = hip_check(hipEventRecord(L.done, s), "event record");
    if (rc) return rc;
    for (size_t i = 0; i < mem.size(); ++i) err[i] = launch_back(*mem[i], slots[mem[i]->slot], L.done);
    return WLC_OK;
  }

  static int lane_of(const Request &R) {
    GramJob j{};
    run_gram_job(*R.plan, R.ws_run, j);
    return (double)j.n_work * (double)j.k_split >= LANE_SPLIT ? 1 : 0;
  }

  // Finish a request that failed before its done event was recorded.
  void fail_request(Request &R, int rc) {
    Slot &S = slots[R.slot];
    (void)hipStreamSynchronize(S.stream);
    R.status = rc;
    R.state = State::Done;
    R.t_done = now_ms();
    R.slot = -1;
    S.busy = false;
    ++completed;
    cv_done.notify_all();
  }

  // Form and launch a batch on every idle lane from the ready requests: all
  // ready requests of the lane with the precision of the oldest of them.
  // Called with the lock held; releases it while enqueueing (running
  // requests cannot be released, and map nodes do not move).
  void batch(std::unique_lock<std::mutex> &lk) {
    for (int li = 0; li < 2; ++li) {
      Lane &L = lanes[li];
      if (L.busy) continue;
      std::vector<Request *> mem;
      int prec = -1;
      for (auto it = gram_ready.begin(); it != gram_ready.end() && (int)mem.size() < MAX_BATCH;) {
        Request &R = reqs[*it];
        if (lane_of(R) == li && (prec < 0 || R.plan->cfg.precision == prec)) {
          prec = R.plan->cfg.precision;
          mem.push_back(&R);
          it = gram_ready.erase(it);
        } else {
          ++it;
        }
      }
      if (mem.empty()) continue;
      std::vector<int> err(mem.size(), WLC_OK);
      L.busy = true;
      ++n_batches;
      n_batched += (int64_t)mem.size();
      max_batch = std::max<int64_t>(max_batch, (int64_t)mem.size());
      lk.unlock();
      const int rc = launch_batch(L, mem, err);
      lk.lock();
      if (rc) {
        (void)hipStreamSynchronize(L.stream);
        L.busy = false;
      }
      for (size_t i = 0; i < mem.size(); ++i) {
        const int e = rc ? rc : err[i];
        if (e)
          fail_request(*mem[i], e);
        else
          mem[i]->back_enqueued = true;
      }
    }
  }

  void loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
      // completions
      for (Slot &S : slots) {
        if (!S.busy) continue;
        Request &R = reqs[S.ticket];
        if (!R.back_enqueued) continue;  // waiting for its batch: no done event yet
        const hipError_t q = hipEventQuery(S.done);
        if (q == hipErrorNotReady) continue;
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
      for (Lane &L : lanes)
        if (L.busy && hipEventQuery(L.done) != hipErrorNotReady) L.busy = false;
      if (stop) {
        bool any = !gram_ready.empty();
        for (Slot &S : slots) any |= S.busy;
        for (Lane &L : lanes) any |= L.busy;
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
        R.batched = run_gram_batchable(*R.plan);
        Slot &S = slots[free_slot];
        S.ticket = R.ticket;
        S.busy = true;
        lk.unlock();
        int rc = launch_front(R, S);
        if (!rc && !R.batched) rc = launch_back(R, S, nullptr);
        lk.lock();
        if (rc)
          fail_request(R, rc);
        else if (R.batched)
          gram_ready.push_back(R.ticket);
        else
          R.back_enqueued = true;
      }
      // batches (also while stopping: admitted requests must finish)
      if (!gram_ready.empty()) batch(lk);
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
  if (!base || !fiducial || !out || max_inflight < 1 || max_inflight > MAX_BATCH || hbm_budget < (1u << 20))
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
    if (!rc) rc = hip_check(hipEventCreateWithFlags(&S.front, hipEventDisableTiming), "event create");
    if (!rc) rc = hip_check(hipHostMalloc((void **)&S.pinned_W, h->w_stage_doubles * 8, hipHostMallocDefault),
                            "pinned allocation");
    if (!rc) rc = hip_check(hipHostMalloc((void **)&S.pinned_out, 16, hipHostMallocDefault), "pinned allocation");
    if (rc) {
      wlc_server_destroy(h);
      return rc;
    }
  }
  for (Lane &L : h->lanes) {
    rc = hip_check(hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking), "stream create");
    if (!rc) rc = hip_check(hipEventCreateWithFlags(&L.done, hipEventDisableTiming), "event create");
    if (!rc) rc = hip_check(hipMalloc((void **)&L.jobs_dev, MAX_BATCH * sizeof(GramJob)), "job list allocation");
    if (!rc) rc = hip_check(hipMalloc((void **)&L.counters, GRAM_BATCH_COUNTERS * sizeof(uint32_t)),
                            "queue counter allocation");
    if (!rc) rc = hip_check(hipHostMalloc((void **)&L.jobs_host, MAX_BATCH * sizeof(GramJob), hipHostMallocDefault),
                            "pinned allocation");
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
      !prec_valid(q->precision) || (q->snr_method != WLC_SNR_DIRECT && q->snr_method != WLC_SNR_STRUCTURED))
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
  const size_t ws_snr = snr_bytes(*plan, q->snr_method);
  if (!ws_snr) return fail(WLC_EINVAL, "the structured S/N is not available for this request");
  const int64_t n = plan->n_out;
  const size_t foot = a256(plan->ws_run) + a256(ws_snr) + 2 * a256(n * 8) + a256(n * 4) +
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
  out->batches = srv->n_batches;
  out->batched_requests = srv->n_batched;
  out->max_batch = srv->max_batch;
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
    if (S.front) (void)hipEventDestroy(S.front);
    if (S.pinned_W) (void)hipHostFree(S.pinned_W);
    if (S.pinned_out) (void)hipHostFree(S.pinned_out);
  }
  for (Lane &L : srv->lanes) {
    if (L.stream) {
      (void)hipStreamSynchronize(L.stream);
      (void)hipStreamDestroy(L.stream);
    }
    if (L.done) (void)hipEventDestroy(L.done);
    if (L.jobs_dev) (void)hipFree(L.jobs_dev);
    if (L.counters) (void)hipFree(L.counters);
    if (L.jobs_host) (void)hipHostFree(L.jobs_host);
  }
  if (srv->arena_base) (void)hipFree(srv->arena_base);
  delete srv;
  return WLC_OK;
}

}  // extern "C"
