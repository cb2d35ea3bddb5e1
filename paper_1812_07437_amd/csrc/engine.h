// Asynchronous building blocks of the C ABI, shared by the entry points in
// api.hip and the request server in server.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"
#include "plan.h"

namespace wlc {

// Hooks around the phases of a run (WLC_PHASE_*); may be null.
struct PhaseHooks {
  virtual void begin(int phase) = 0;
  virtual void end(int phase) = 0;
  virtual ~PhaseHooks() = default;
};

// Device workspace sizes of a plan.
size_t run_ws_bytes(const Plan &p);
size_t snr_ws_bytes(const Plan &p);

// Validate the tables on the device and synchronise the stream
// (WLC_EINVAL / WLC_ERANGE).  Uses the run workspace.
int validate_tables(const Plan &p, const wlc_tables &tb, void *ws, hipStream_t s);

// Enqueue the hot path (no synchronisation): index upload, staging,
// quadrature, projection, A-build, Gram product, assembly.
// rho > 0 replaces the plan's mean matter density.
int run_enqueue(const Plan &p, const wlc_tables &tb, void *ws, double *d, double *r, void *C, int32_t *row_exp2,
                hipStream_t s, PhaseHooks *hooks, double rho = 0.0);

// The same path in three parts, so that the Gram products of several runs
// can share one batched launch (the request server): front = index upload,
// staging, quadrature, projection and A-build; gram = the one-halo product
// with its split-K reduction; back = mirror, row exponents and assembly.
int run_enqueue_front(const Plan &p, const wlc_tables &tb, void *ws, hipStream_t s, PhaseHooks *hooks,
                      double rho = 0.0);
int run_enqueue_gram(const Plan &p, void *ws, hipStream_t s, PhaseHooks *hooks);
int run_enqueue_back(const Plan &p, const wlc_tables &tb, void *ws, double *d, double *r, void *C, int32_t *row_exp2,
                     hipStream_t s, PhaseHooks *hooks);
// For a batched Gram instead of run_enqueue_gram: whether the plan's
// precision has a batched kernel, the plan's product as a batch job (item0
// left 0), and its split-K reduction, enqueued after the batch.
bool run_gram_batchable(const Plan &p);
void run_gram_job(const Plan &p, void *ws, GramJob &job);
int run_enqueue_gram_reduce(const Plan &p, void *ws, hipStream_t s);

// Enqueue the S/N factorisation (no synchronisation).  On completion
// *flag_dev != 0 marks a non-positive pivot and *out_dev holds (S/N)^2.
// With lmax, the rows are taken in ell_max order and *out_dev holds the
// (S/N)^2 of every ell_max cut, one per used ell-bin (wlc_snr2_lmax).
int snr_enqueue(const Plan &p, const void *C, const int32_t *row_exp2, const double *d, void *ws, hipStream_t s,
                PhaseHooks *hooks, KernelProbe *probe, int32_t **flag_dev, double **out_dev, bool lmax = false);

// The same (S/N)^2 through the distinct rows, from the run workspace of a
// completed wlc_run (PAPER tomography only): the bordered Cholesky of
// I + L^T M L on n_R rows.  Same completion protocol as snr_enqueue.
size_t snr_structured_ws_bytes(const Plan &p);
int snr_structured_enqueue(const Plan &p, const void *ws_run, void *ws, hipStream_t s, PhaseHooks *hooks,
                           KernelProbe *probe, int32_t **flag_dev, double **out_dev);

int hip_check(hipError_t e, const char *what);

// Enumerate and size a plan.
int plan_build(const wlc_config &cfg, Plan &p);

// y[i] = a * x[i] (device), used to rescale shared tables per request.
void launch_scale(const double *x, double *y, int64_t n, double a, hipStream_t s);

}  // namespace wlc
