/*
 * wlcov.h -- C ABI of libwlcov, an MI355X (gfx950) library that predicts the
 * binned tomographic weak-lensing convergence power spectrum and bispectrum
 * and their joint non-Gaussian covariance, following Rizzato, Benabed,
 * Bernardeau & Lacasa (2019), "Tomographic weak lensing bispectrum"
 * (arXiv 1812.07437).
 *
 * Conventions shared by every entry point
 *   - Every call returns int: WLC_OK (0) or a negative WLC_E* code; the text
 *     of the last error of the calling thread is wlc_last_error().  No C++
 *     exception crosses this boundary.
 *   - "device" pointers are HIP device allocations on the current device;
 *     "host" pointers are ordinary host memory.  The caller owns every buffer
 *     it passes; the library owns plans.  Nothing returned aliases a caller
 *     buffer.
 *   - Work is enqueued on the given HIP stream (NULL = the null stream) and is
 *     asynchronous unless the entry point says it synchronises.
 *   - Matrices are row-major.  The covariance is returned scaled:
 *       C_true[a][b] = C[a][b] * 2^-(row_exp2[a] + row_exp2[b]),
 *     so that every diagonal entry of C lies in [1, 4); the scaling is exact.
 */
#ifndef WLCOV_H
#define WLCOV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes */
enum {
  WLC_OK = 0,
  WLC_EINVAL = -1,  /* bad argument or table (non-finite, non-positive, unsorted)   */
  WLC_ERANGE = -2,  /* the k table does not cover some ell/chi below k_max        */
  WLC_ENOMEM = -3,  /* host allocation failed                                      */
  WLC_ENOTPD = -4,  /* covariance not positive definite (Cholesky pivot <= 0)      */
  WLC_EDEVICE = -5, /* HIP runtime error                                           */
  WLC_EBUSY = -6,   /* serving: request refused by memory admission               */
  WLC_ENOCONV = -7  /* an iteration did not converge within its sweep limit        */
};

/* ---- data-vector tomography convention (Sec. 5, ordering of eq. eq:SN2)
 * PAPER : bispectrum triplets as in the paper (all n^3 for scalene triangles,
 *         one ordering of the bins on equal sides);
 * SORTED: only i <= j <= k for every triangle (the distinct values). */
enum { WLC_TOMO_PAPER = 0, WLC_TOMO_SORTED = 1 };

/* ---- arithmetic of the one-halo Gram product (everything else is FP64)
 * FP64     : f64 MFMA on the flattened (chi, M) axis, FP64 covariance output;
 * BF16     : bf16 MFMA with FP32 accumulation, FP32 covariance output;
 * BF16X3   : split bf16 (hi + lo) compensated product hi.hi + hi.lo + lo.hi;
 * FP32     : f32 MFMA;
 * FP64_CHI : FP64, the same sum taken over M first and then over chi (the
 *            factorisation of eq. General1h along the line of sight),
 *            N_M times fewer operations; FP64 covariance output.
 * BF16_AUTO: per 256 x 256 tile of the product, the split product where an
 *            a-priori bound needs it and one bf16 product elsewhere.  With
 *            f_a the one-halo share of the diagonal entry C_aa (in FP64, before
 *            the product) and F_I the largest f_a of the rows of panel I (256
 *            rows of the product's row order, wlc_plan_gram_order), a
 *            single bf16 product changes an entry of tile (I, J) by at most
 *            (2u + u^2 + K 2^-24) sqrt(F_I F_J) sqrt(C_aa C_bb) (u = 2^-8
 *            for bf16 operands, K 2^-24 for the FP32 accumulation of K
 *            terms, Cauchy-Schwarz over the products); tiles where that bound
 *            exceeds gram_tol take the split product.
 * BF16X3, FP32 and BF16_AUTO also return an FP32 covariance. */
enum { WLC_FP64 = 0, WLC_BF16 = 1, WLC_BF16X3 = 2, WLC_FP32 = 3, WLC_FP64_CHI = 4, WLC_BF16_AUTO = 5 };

/* ---- flags */
enum {
  WLC_FLAG_NOCHECK = 1, /* skip the table validation pass (and its one stream sync) */
  WLC_FLAG_NGINS = 2,   /* add the in-survey terms built from lower-order spectra:
                           B.B and P.T between bispectra (eq. CovBB), P.B between
                           power spectrum and bispectrum (eq. Covpb); the P.T term
                           uses the projected one-halo trispectrum of the two other
                           legs of each triangle.  Not combinable with
                           wlc_snr2_structured. */
  WLC_FLAG_SSC_CHI = 4  /* super-sample term resolved along the line of sight
                           (eq. WLSSCflatskyLimber with sigma_W^2(chi)):
                             sum_n w_n sigma_W^2(chi_n) T_a R_a T_b R_b at chi_n,
                           T the projection function of eq. nProjection, R the
                           3-D response, sigma_W^2 as in wlc_sigma_w2; it joins
                           the Gram product as one more column per chi node
                           (k_len = n_chi (n_m + 1)) and sigma_b2 is not used.
                           Needs k[0] chi_max Theta <= 0.1 (WLC_ERANGE). */
};

typedef struct {
  int32_t n_z;        /* tomographic (redshift) bins                          */
  int32_t n_ell;      /* log-spaced ell-bins over [ell_min, ell_max]          */
  int32_t n_chi;      /* line-of-sight nodes of the tables                     */
  int32_t n_k;        /* k nodes of the P and u tables                         */
  int32_t n_m;        /* mass nodes                                            */
  int32_t tomo_mode;  /* WLC_TOMO_*                                            */
  int32_t precision;  /* WLC_FP64 / WLC_BF16 / WLC_BF16X3 / WLC_FP32 / ...     */
  int32_t flags;      /* WLC_FLAG_*                                            */
  double ell_min, ell_max;
  double ell_cut;     /* keep only ell-bins whose centre is below this (<= 0: all), eq. eq:SN */
  double f_sky;       /* sky fraction; Omega_sky = 4 pi f_sky                  */
  double sigma_eps;   /* shape noise (eq. ShotNoise)                           */
  double n_gal_arcmin2; /* total source density, split evenly over the bins    */
  double sigma_b2;    /* variance of the long background mode (super-sample)   */
  double k_max;       /* line-of-sight integrand vanishes above this k (Sec. 4.4) */
  double rho_mean;    /* comoving mean matter density, (M_sun/h)/(Mpc/h)^3     */
  int32_t n_sub;      /* bin averaging: 0 or 1 evaluates every polyspectrum at the
                         bin centres (the paper's approximation, Sec. 3.2.2 and
                         App. B); 2..8 averages it over n_sub equal sub-bins per
                         ell-bin: a power-spectrum bin over its sub-bins with
                         weights proportional to the number of modes (ell), a
                         triangle bin over the cells of sub-bin triples whose
                         centres obey the strict triangle inequality, weighted
                         by the continuum count of mode pairs in the cell
                         (App. B), the polyspectra taken at the cell centres.
                         The data vector, the responses and
                         the one-halo and super-sample terms average; the
                         Gaussian term keeps its form with the averaged power
                         spectra.  Not combinable with WLC_FLAG_NGINS. */
  double gram_tol;    /* WLC_BF16_AUTO: bound on the one-halo rounding error of
                         an entry relative to sqrt(C_aa C_bb) above which a tile
                         takes the split product (<= 0: 2^-17, below the 1e-5
                         target on the diagonal); ignored otherwise */
} wlc_config;

/* Input tables, all DEVICE pointers to float64, row-major:
 *   chi, w_chi [n_chi]  line-of-sight nodes (increasing, > 0) and weights;
 *   k [n_k]             strictly increasing, > 0;
 *   m, w_m [n_m]        masses and quadrature weights of the mass integrals;
 *   W [n_z][n_chi]      lensing kernels (eqs. KernelLensing1, LensEff), >= 0;
 *   P [n_chi][n_k]      linear matter power at each chi node, > 0;
 *   u [n_m][n_k]        Fourier halo profile, > 0;
 *   n_m [n_m]           halo mass function, > 0;
 *   b1, b2 [n_m]        halo biases or NULL (b1 = 1, b2 = 0);
 *   n_tri [n_tri]       optional triangle counts replacing the closed form
 *                       (e.g. from wlc_lattice_counts), or NULL.
 * Values at k = ell/chi are read by linear interpolation of ln X in ln k. */
typedef struct {
  const double *chi, *w_chi, *k, *m, *w_m;
  const double *W, *P, *u, *n_m, *b1, *b2;
  const double *n_tri;
} wlc_tables;

typedef struct {
  int64_t n_data;      /* rows of the data vector in the chosen convention    */
  int64_t n_distinct;  /* distinct rows (= SORTED vector length)              */
  int64_t n_p;         /* power-spectrum rows of the data vector              */
  int64_t n_tri;       /* binned triangles                                    */
  int64_t n_cfg;       /* ell-configurations: ell-bins + triangles            */
  int64_t n_ell_used;  /* ell-bins below ell_cut                              */
  int64_t k_len;       /* contraction length of the Gram product: n_chi * n_m,
                          n_chi * (n_m + 1) with WLC_FLAG_SSC_CHI            */
  size_t c_elem_bytes; /* 8 (FP64) or 4 (mixed precisions)                    */
  size_t ws_run_bytes; /* device workspace needed by wlc_run                  */
  size_t ws_snr_bytes; /* device workspace needed by wlc_snr2                 */
  size_t ws_snr_structured_bytes; /* ... by wlc_snr2_structured (0: not available
                                     for this plan: SORTED tomography or n_z > 32) */
  int64_t n_avg;       /* entries of the bin-averaging lists (n_cfg at n_sub <= 1) */
  size_t ws_pca_bytes; /* device workspace needed by wlc_pca (0: n_data > 65472) */
} wlc_sizes;

typedef struct wlc_plan_s *wlc_plan;

/* Build a plan (host only, no device work): the ell-bins (Sec. 3.2.1,
 * App. A), the binned triangles l1 <= l2 <= l3 with strict triangle inequality
 * on the bin centres, the tomographic rows in data-vector order (Sec. 5) and
 * the map from each row to its distinct row.  Errors: WLC_EINVAL for
 * non-positive sizes or inconsistent scalars, WLC_ENOMEM. */
int wlc_plan_create(const wlc_config *cfg, wlc_plan *out);
void wlc_plan_destroy(wlc_plan plan);
int wlc_plan_sizes(wlc_plan plan, wlc_sizes *out);

/* Copy the plan's index tables into HOST buffers (any may be NULL):
 *   tri [n_tri][3]          ell-bin indices of each triangle, data-vector order;
 *   rows [n_data][8]        kind (2 = P, 3 = B), cfg, ell-bins l1 l2 l3 and
 *                           redshift bins z1 z2 z3 (-1 where unused);
 *   distinct [n_data]       index of the row's distinct (sorted) row. */
int wlc_plan_index(wlc_plan plan, int32_t *tri, int32_t *rows, int32_t *distinct);

/* Row order of the one-halo Gram product (eq. General1h over the distinct
 * rows), into a HOST buffer of n_distinct int32: pos[e] is the product row of
 * distinct row e.  The flattened products (every precision but FP64_CHI)
 * order the distinct rows stably by their lowest redshift bin, so that a
 * 256-row panel's factor ends where the lensing kernel of that bin does (eq.
 * KernelLensing1) and a tile's product stops where the shorter of its two
 * panels' factors ends; the panels of wlc_gram_split_tiles and of the
 * gram_tol bound are runs of 256 in this order.  FP64_CHI keeps the distinct
 * order (pos[e] = e).  The
 * covariance and every other output keep the data-vector order whatever this
 * order is.  WLC_EINVAL for a null argument. */
int wlc_plan_gram_order(wlc_plan plan, int32_t *pos);

/* The plan's bin-averaging lists into HOST buffers (any may be NULL):
 *   off [n_cfg + 1]    entries off[c] .. off[c+1]-1 belong to configuration c
 *                      (ell-bins first, then triangles in data-vector order);
 *   legs [n_avg][3]    sub-bin index of each leg (bin b, sub-bin s -> b n_sub
 *                      + s; a P entry holds its leg twice, then -1);
 *   ell [n_ell_used * max(1, n_sub)] sub-bin centres;
 *   w [n_avg]          weights (sum 1 per configuration): see wlc_config.n_sub. */
int wlc_plan_averaging(wlc_plan plan, int32_t *off, int32_t *legs, double *ell, double *w);

/* Closed-form counts into HOST buffers (Sec. 3.2.2, App. B):
 *   n_modes [n_ell_used] = 2 l Delta_l f_sky;
 *   n_tri   [n_tri]      = Omega^2 l1 l2 l3 D1 D2 D3 / (2 pi^3 Lambda), the
 *                          continuum count at the bin centres. */
int wlc_counts_closed(wlc_plan plan, double *n_modes, double *n_tri);

/* Integer lattice counts into DEVICE buffers (Sec. 3.2.2 lattice, App. B
 * N_tri as a sum of the selection function): modes q != 0 of the lattice of
 * fundamental l_f = 2 pi / sqrt(Omega) with ceil((e_b/l_f)^2) <= |q|^2 <
 * ceil((e_{b+1}/l_f)^2) per ell-bin, and ordered pairs (q1, q2) with q1, q2,
 * q1 + q2 in the three bins of each triangle.  Bit-exact; asynchronous.
 * ws: DEVICE workspace of at least ws_run_bytes (only its index part is used);
 * modes [n_ell_used] and tris [n_tri] may each be NULL to skip. */
int wlc_lattice_counts(wlc_plan plan, void *ws, uint64_t *modes, uint64_t *tris, void *stream);

/* The hot path.  From the device tables, compute into DEVICE buffers:
 *   d [n_data]        data vector: Limber projections (eq. nProjection) of the
 *                     halo-model P (eq. PspHMtot2) and B (eqs. B1halo,
 *                     B2halos, first line of B3halos);
 *   r [n_data]        projected responses to a long mode (eqs. PowerHMResp,
 *                     BispHMResp, RespP, RespB);
 *   C [n_data][n_data] scaled covariance (FP64 if precision == WLC_FP64 else
 *                     FP32): Gaussian (eq. CovPPG and its bispectrum
 *                     analogue, App. B) + one-halo 4/5/6-point terms (eqs.
 *                     CovPPNG, Ins5P, Ins6P with eq. General1h) computed as the
 *                     Gram product A A^T over the flattened (chi, M) axis +
 *                     the super-sample term (eq. WLSSCflatskyLimber): sigma_b2
 *                     r r^T for a single long mode, or with WLC_FLAG_SSC_CHI
 *                     its line-of-sight form inside the Gram product;
 *   row_exp2 [n_data] the power-of-two scaling of C (see above).
 * ws: DEVICE workspace of at least ws_run_bytes, 256-byte aligned.
 * Unless WLC_FLAG_NOCHECK is set, validates the tables first and synchronises
 * the stream once (WLC_EINVAL / WLC_ERANGE); everything else is asynchronous. */
int wlc_run(wlc_plan plan, const wlc_tables *tables, void *ws, double *d, double *r, void *C,
            int32_t *row_exp2, void *stream);

/* sigma_W^2(chi_n) into DEVICE sw [n_chi]: the variance of the linear density
 * contrast averaged over the survey's disk at each chi node, the thin-shell
 * limit of the cylinder window of eq. Mask (App. B; definition after eq.
 * CovPP22, Sec. 3.2.3):
 *   sigma_W^2(chi) = 4 int d^2 eps / (2 pi)^2 [J1(x) / x]^2 P(eps, chi)
 *                  = (2 / pi) int eps^2 [J1(x) / x]^2 P(eps, chi) d ln eps,
 *   x = eps chi Theta, Theta the survey's angular radius:
 *   Omega = 4 pi f_sky = 2 pi (1 - cos Theta) (Sec. 3.2.2, after eq. PSest).
 * The integral runs over the k table [k_0, k_last] by the trapezoid rule in
 * ln eps on 16384 uniform nodes (end nodes: the table's own end values);
 * P(eps, chi) is read like every table value.  Only chi, k and P are read.
 * Asynchronous; no validation (the tables must satisfy wlc_run's rules). */
int wlc_sigma_w2(wlc_plan plan, const wlc_tables *tables, double *sw, void *stream);

/* (S/N)^2 = d^T C_true^-1 d (eq. SNprim) from wlc_run's outputs (DEVICE
 * C, row_exp2, d), by an FP64 Cholesky factorisation of the scaled matrix
 * bordered with the scaled data vector.  Result in *snr2_host.
 * ws: DEVICE workspace of at least ws_snr_bytes.  Synchronises the stream.
 * WLC_ENOTPD if a pivot is not positive. */
int wlc_snr2(wlc_plan plan, const void *C, const int32_t *row_exp2, const double *d, void *ws,
             double *snr2_host, void *stream);

/* wlc_snr2 without allocation and without synchronisation, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  The same FP64 bordered
 * Cholesky as wlc_snr2 (same kernels, same split-k choices, so the same
 * result bit for bit), with its workspace in a fixed device array of the
 * library: 64 MiB per device, held by every device the library has run this
 * entry point on until the process ends.  That bounds the data vector to
 * about 2300 rows: WLC_EINVAL (nothing enqueued) when wlc_snr2's workspace,
 * ws_snr_bytes, exceeds 64 MiB.
 * Inputs as wlc_snr2 (DEVICE C, row_exp2, d).  Outputs (DEVICE): snr2_dev[0]
 * = (S/N)^2, status_dev[0] = 0, or nonzero when a pivot was not positive
 * (then snr2_dev is meaningless).  Asynchronous on the stream; no host
 * synchronisation, no device allocation or free.  Every call on one device
 * shares the one array and keeps it until its work is done: calls on one
 * device whose work overlaps (different streams, or several host threads)
 * race; serialise them on one stream. */
int wlc_snr2_noalloc(wlc_plan plan, const void *C, const int32_t *row_exp2, const double *d, double *snr2_dev,
                     int32_t *status_dev, void *stream);

/* The cumulative (S/N)^2(ell_max) of eq. eq:SN: into snr2_host[n_ell_used]
 * (HOST), entry b is d^T C^-1 d over the rows whose legs all lie in ell-bins
 * 0..b, i.e. the data vector cut at an ell_max between bins b and b + 1; the
 * last entry is the full (S/N)^2.  The covariance of a cut vector is a
 * principal submatrix of C, so the rows are taken in ell_max order (stable
 * by their largest bin) and one bordered FP64 Cholesky gives every cut as a
 * prefix sum of y^2, y = L^-1 d.  Arguments, workspace (ws_snr_bytes) and
 * errors as wlc_snr2; synchronises the stream. */
int wlc_snr2_lmax(wlc_plan plan, const void *C, const int32_t *row_exp2, const double *d, void *ws,
                  double *snr2_host, void *stream);

/* Principal components of the joint covariance (Sec. 6): the eigen-
 * decomposition C_true = sum_a lambda_a S_a S_a^T (eq. SNPCA), the new
 * observables D^_a = S_a . d (eq. NewObs), their (S/N)^2_a = D^_a^2 /
 * lambda_a (eq. SNperEign) and the cumulative curve (eq. CumulSN).
 * The eigenvalues span tens of decades, so they come from one-sided Jacobi
 * on the graded Cholesky factor (C_true = G^T G, G = L^T 2^-t with L the
 * FP64 Cholesky factor of the scaled C), which keeps relative accuracy; the
 * rotations run in blocks of 32 columns on FP64 MFMA until no pair of
 * columns has |cos| above 8 sqrt(n_pad) eps, at most 40 sweeps.
 * Inputs as wlc_snr2 (DEVICE C, row_exp2, d).  Outputs (HOST, n_data each):
 *   lambda     eigenvalues of C_true, ascending;
 *   snr2_mode  (S/N)^2 of each mode, in the order of lambda;
 *   cum_desc   cumulative (S/N)^2 over the modes sorted by decreasing
 *              (S/N)^2 (its last entry is d^T C^-1 d);
 *   sweeps     (may be NULL) sweeps used.
 * S (DEVICE [n_data][n_data], may be NULL to skip the eigenvectors): row a
 * is the unit eigenvector of lambda[a], its largest entry in magnitude made
 * positive.  ws: DEVICE workspace of ws_pca_bytes.  Synchronises the stream
 * once per sweep.  WLC_ENOTPD if C is not positive definite, WLC_ENOCONV
 * without convergence, WLC_EINVAL if ws_pca_bytes is 0. */
int wlc_pca(wlc_plan plan, const void *C, const int32_t *row_exp2, const double *d, void *ws, double *lambda,
            double *snr2_mode, double *cum_desc, int32_t *sweeps, double *S, void *stream);

/* The same (S/N)^2 through the distinct rows, for PAPER tomography.
 * With C = C_G + E M E^T (C_G the Gaussian term, block-diagonal over
 * ell-configurations; E the map from data-vector rows to their distinct
 * rows; M the one-halo plus super-sample term on distinct rows) and d = E d_R:
 *   (S/N)^2 = u^T (I + L^T M L)^-1 u,  u = L^T d_R,  L L^T = E^T C_G^-1 E,
 * where E^T C_G^-1 E is block-diagonal with closed-form blocks (symmetrised
 * products of (P^s)^-1 per ell-bin).  The one large factorisation is an FP64
 * Cholesky on n_distinct rows instead of n_data (eqs. SNprim, eq:SN2, with
 * the Gaussian term of eq. CovPPG and App. B).
 * ws_run: the DEVICE workspace of a completed wlc_run with this plan (its
 *         Gram product, spectra, counts and row exponents are read; any
 *         precision, the result carries the Gram's precision);
 * ws:     DEVICE workspace of at least ws_snr_structured_bytes.
 * Synchronises the stream.  WLC_EINVAL for SORTED tomography (there
 * n_data = n_distinct and wlc_snr2 is the same computation), n_z > 32, or
 * WLC_FLAG_NGINS (its terms are not of the form E M E^T);
 * WLC_ENOTPD if a pivot is not positive. */
int wlc_snr2_structured(wlc_plan plan, const void *ws_run, void *ws, double *snr2_host, void *stream);

/* Tiles of the last run's one-halo product that took the split bf16 product
 * (WLC_BF16_AUTO: the tiles whose one-product error bound exceeds gram_tol;
 * all of them for WLC_BF16X3, none otherwise) and the number of tiles, into
 * HOST scalars.  ws_run: the DEVICE workspace of a completed wlc_run with
 * this plan; synchronises the device for the copy. */
int wlc_gram_split_tiles(wlc_plan plan, const void *ws_run, int64_t *split, int64_t *tiles);

/* ---- the one-halo Gram product of a caller's factor
 * The one-halo covariance of the distinct rows is (1/Omega) A A^T over the
 * flattened (chi, M) axis (eq. General1h with eqs. CovPPNG, Ins5P, Ins6P);
 * wlc_run builds A from the tables.  wlc_gram runs the same product kernels,
 * with the same tiles, split-K choice and summation order as wlc_run, on a
 * factor the caller supplies, and writes the lower triangle of A A^T (the
 * upper one is its mirror image).
 *   precision  WLC_BF16 (one product), WLC_BF16X3 (hi hi^T + hi lo^T +
 *              lo hi^T on every tile) or WLC_BF16_AUTO (per tile, see below);
 *              FP32 accumulation.
 *   n, k       rows and columns of A; n_pad = n rounded up to 256,
 *              k_pad = k rounded up to 64.
 *   a_hi, a_lo DEVICE, bf16 bit patterns of A (hi) and of its residue (lo)
 *              in the k-blocked layout: element (r, c) at
 *              ((c / 32) n_pad + r) 32 + c % 32, n_pad x k_pad elements,
 *              zero in the padding rows and columns.  a_lo is read by
 *              WLC_BF16X3 and WLC_BF16_AUTO (required there), ignored by
 *              WLC_BF16 (may be NULL).
 *   panel_f    WLC_BF16_AUTO: DEVICE, n_pad / 256 doubles F_I; the 256 x 256
 *              tile (I, J) takes the split product iff F_I F_J > lim, one
 *              product otherwise.  Ignored (may be NULL) for the others.
 *   panel_ext  DEVICE, n_pad / 256 int32 or NULL: the rows of panel I are
 *              zero from column 32 ext_I on (ext_I <= k_pad / 32), and tile
 *              (I, J) sums only the first 32 min(ext_I, ext_J) columns (the
 *              rest are zero products; A need not hold them).  NULL: all.
 *   g          DEVICE, FP32 [n_pad][n_pad], row-major: every entry (i, j)
 *              with i >= j is written; above the diagonal, the diagonal
 *              256 x 256 tiles hold partial or whole sums and the other tiles
 *              are left as they are.
 *   ws         DEVICE workspace of wlc_gram_ws_bytes bytes (the split-K
 *              partial products), 256-byte aligned; may be NULL when that is 0.
 * Asynchronous on stream.  WLC_EINVAL for another precision, n or k < 1 or
 * too large, a missing pointer or an unaligned workspace. */
int wlc_gram_ws_bytes(int precision, int64_t n, int64_t k, size_t *bytes);
int wlc_gram(int precision, int64_t n, int64_t k, const uint16_t *a_hi, const uint16_t *a_lo,
             const double *panel_f, double lim, const int32_t *panel_ext, float *g, void *ws, void *stream);

/* Work of the last run's one-halo product, into HOST doubles: flops counts
 * one product per tile over the columns it summed (2 x 256 x 256 per column
 * and tile I >= J for the bf16 products, 2 x 128 x 256 on the 128 x 256
 * tiles of the FP64 product, 2 x 128 x 128 on the FP32 product's tiles; each
 * stops where the shorter of its two 256-row panels' factors ends),
 * mfma_flops the same with the split tiles counted three times.
 * factor_bytes (may be NULL): the bytes of the factor A that
 * the product's operands need, over the distinct rows and the K columns (the
 * bf16 factors up to each panel's extent, with the lo half where a tile of
 * the panel can take the split product; FP32 and FP64 over all K).  All 0
 * for WLC_FP64_CHI.  ws_run: the DEVICE
 * workspace of a completed wlc_run with this plan; synchronises the device
 * for the copies. */
int wlc_gram_work(wlc_plan plan, const void *ws_run, double *flops, double *mfma_flops, double *factor_bytes);

/* ---- phase timing (per-plan HIP events; not for plans shared by concurrent runs)
 * With timing enabled, wlc_run and wlc_snr2 record a HIP event pair on their
 * stream around each phase; wlc_plan_timings synchronises on them and writes
 * the last recorded duration of every phase in milliseconds (0 if it did not
 * run) into ms[WLC_PHASE_COUNT] (HOST). */
enum {
  WLC_PHASE_TABLES = 0,  /* validation, staging, spectra, projection, Gram factor */
  WLC_PHASE_ABUILD = 1,  /* A rows in the Gram precision                           */
  WLC_PHASE_GRAM = 2,    /* one-halo Gram product (and its split-K reduction)      */
  WLC_PHASE_ASSEMBLE = 3,/* row exponents and covariance assembly                  */
  WLC_PHASE_SNR_PREP = 4,/* bordered FP64 matrix from C and d                      */
  WLC_PHASE_CHOL = 5,    /* blocked Cholesky and y^T y                             */
  WLC_PHASE_COUNT = 6
};
int wlc_plan_set_timing(wlc_plan plan, int enable);
int wlc_plan_timings(wlc_plan plan, float *ms);
/* Launch statistics of the Cholesky block-update kernel (k_update2 and its
 * split-k reduction) in the last timed wlc_snr2, into HOST scalars: summed
 * event time of the timed launches, number of launches, number timed (event
 * capacity permitting; the time covers only those), and the algorithmic
 * flops of all launches (2 k per updated lower-triangle entry).  Synchronises
 * on the events. */
int wlc_plan_kernel_stats(wlc_plan plan, double *ms_total, int64_t *launches, int64_t *timed, double *flops);

const char *wlc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* WLCOV_H */
