/*
 * wlcov_serve.h -- request server of libwlcov: likelihood / MCMC-style
 * requests (perturbed cosmology, number of redshift bins, maximum multipole)
 * against device-resident fiducial tables, continuously batched onto the GPU.
 *
 * The paper computes the data vector, covariance and S/N for one survey set-up
 * at a time (Rizzato et al. 2019, Secs. 3 and 5, eq. eq:SN for the cut at
 * l_max); a likelihood code needs the same quantities for many nearby set-ups.
 * The server keeps the chi / k / M tables on the device and admits requests in
 * arrival order as soon as their device-memory footprint fits a fixed arena
 * and an execution slot is free.  An admitted request runs its quadrature
 * and A-build on its own HIP stream; the one-halo Gram products of the bf16
 * and split-bf16 requests admitted so far are then batched into one
 * persistent kernel that drains a device queue of their tile work items
 * (requests of different sizes in one launch; a narrow and a wide batch lane
 * so that small requests do not wait behind the product of a large one);
 * assembly and the FP64 Cholesky follow on the request's own stream, so
 * requests that arrive while others run overlap with them on the device.
 * FP64 and FP32 requests compute their Gram product on their own stream.
 * Each request's result does not depend on what else is running: a product
 * in a batch runs the same tiles, k slices and summation order as alone.
 *
 * Conventions as in wlcov.h (int return codes, wlc_last_error()).
 */
#ifndef WLCOV_SERVE_H
#define WLCOV_SERVE_H

#include <stddef.h>
#include <stdint.h>

#include "wlcov.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wlc_server_s *wlc_server;

/* One request.  Its configuration is the server's base configuration with
 * n_z, precision, ell_cut and rho_mean replaced; its tables are the fiducial
 * ones with P multiplied by p_scale, n(M) by n_scale, and its own lensing
 * kernels W.  (A change of sigma_8 rescales P by (sigma_8/sigma_8,fid)^2; a
 * change of Omega_m rescales rho and n(M) together, keeping the mass
 * normalisation of eq. BoundinMass.) */
/* How a request's (S/N)^2 is computed (both FP64, both exact):
 * DIRECT     : bordered Cholesky of the whole covariance, as wlc_snr2;
 * STRUCTURED : through the distinct rows, as wlc_snr2_structured (PAPER
 *              tomography, n_z <= 32; one Cholesky on n_distinct rows). */
enum { WLC_SNR_DIRECT = 0, WLC_SNR_STRUCTURED = 1 };

typedef struct {
  int32_t n_z;        /* redshift bins of this request (1..64)                 */
  int32_t precision;  /* WLC_FP64 / WLC_BF16 / WLC_BF16X3 / WLC_FP32           */
  int32_t snr_method; /* WLC_SNR_DIRECT / WLC_SNR_STRUCTURED                    */
  int32_t pad;
  double ell_max;     /* keep ell-bins with centre below (<= 0: all), eq. eq:SN */
  double p_scale;     /* multiplies the fiducial P table                       */
  double n_scale;     /* multiplies the fiducial n(M) table                    */
  double rho_mean;    /* comoving mean matter density of this request          */
  const double *W;    /* HOST [n_z][n_chi] lensing kernels; copied by submit   */
} wlc_request;

typedef struct {
  int32_t status;      /* WLC_OK, or the request's error (e.g. WLC_ENOTPD)     */
  int32_t pad;
  int64_t n_data;      /* length of d and r; C is n_data x n_data              */
  size_t c_elem_bytes; /* 8 (FP64) or 4                                         */
  double snr2;         /* (S/N)^2 = d^T C^-1 d (eq. SNprim)                     */
  double t_submit_ms, t_admit_ms, t_done_ms;  /* server clock                   */
  const double *d, *r; /* DEVICE results, valid until wlc_server_release       */
  const void *C;
  const int32_t *row_exp2;
} wlc_result;

typedef struct {
  int64_t queued, running, done;
  size_t arena_bytes, arena_used, arena_peak;
  int64_t completed_total;
  int64_t batches;           /* batched Gram launches so far                    */
  int64_t batched_requests;  /* requests whose Gram ran in a batched launch     */
  int64_t max_batch;         /* most requests in one batched launch             */
} wlc_server_stats;

/* Create a server.  fiducial: DEVICE tables of the base configuration (W is
 * ignored; b1, b2, n_tri optional), kept alive by the caller until destroy.
 * n_tri, if given, holds the counts of the base configuration's triangles;
 * a request uses the leading entries (its triangles are a prefix of the
 * base ones), and wlc_server_submit refuses one with more triangles
 * (WLC_EINVAL).
 * hbm_budget: bytes of the arena reserved on the current device for request
 * workspaces and results.  max_inflight: execution slots (streams), 1..64,
 * which also bounds the requests of one batch. */
int wlc_server_create(const wlc_config *base, const wlc_tables *fiducial, size_t hbm_budget, int32_t max_inflight,
                      wlc_server *out);

/* Enqueue a request (non-blocking); *ticket identifies it.  WLC_EINVAL for a
 * bad request (including WLC_SNR_STRUCTURED where wlc_snr2_structured is not
 * available), WLC_EBUSY if its footprint alone exceeds the arena. */
int wlc_server_submit(wlc_server srv, const wlc_request *req, uint64_t *ticket);

/* Non-blocking status: *done = 1 when finished (res filled), 0 otherwise. */
int wlc_server_poll(wlc_server srv, uint64_t ticket, int32_t *done, wlc_result *res);

/* Block until the request has finished, then fill res. */
int wlc_server_wait(wlc_server srv, uint64_t ticket, wlc_result *res);

/* Copy a finished request's d, r, C, row_exp2 into caller DEVICE buffers
 * (any may be NULL) on the given stream. */
int wlc_server_copy(wlc_server srv, uint64_t ticket, double *d, double *r, void *C, int32_t *row_exp2, void *stream);

/* Free a finished request's device memory; its result pointers become invalid. */
int wlc_server_release(wlc_server srv, uint64_t ticket);

int wlc_server_get_stats(wlc_server srv, wlc_server_stats *out);

/* Wait for running requests, stop the worker and free everything. */
int wlc_server_destroy(wlc_server srv);

#ifdef __cplusplus
}
#endif
#endif /* WLCOV_SERVE_H */
