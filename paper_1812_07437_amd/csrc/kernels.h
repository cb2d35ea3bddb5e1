// Launch wrappers for the HIP kernels (host side, called by the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dev.h"
#include "wlcov.h"

namespace wlc {

// ---- tables and quadrature (k_tables.hip)
// Averaging list of the ell-configurations (the bin centres, or the sub-bins
// of bin averaging): entries off[c] .. off[c + 1] - 1 with legs leg[4 e + a]
// (indices into the staged ell values) and weights w[e] summing to one.
struct SubList {
  const int32_t *off, *leg;
  const double *w;
};
void launch_validate(const DevTables &T, const double *centres, int n_ell, double theta, int *flags, hipStream_t s);
void launch_stage(const DevTables &T, const double *centres, int n_ell, double *U, double *Pk, double *Ne,
                  hipStream_t s);
void launch_spectra(const DevTables &T, const int32_t *cfgT, int n_cfg, const SubList &sl, const double *U,
                    const double *Pk, const double *Ne, const double *centres, double *X, double *R, hipStream_t s);
void launch_project(const DevTables &T, const int32_t *rowR, const int32_t *cfgT, int64_t n_R, const double *X,
                    const double *R, double *dR, double *rR, hipStream_t s);
void launch_ps(const double *dR, double *Ps, int n_ell, int n_z, double noise, hipStream_t s);
// G [n_cfg][n_chi][n_mg]: n_mg = n_m, or n_m + 1 when sw != NULL, the last
// column then holding sqrt(Omega) chi_n sqrt(sigma_W^2(chi_n)) R[cfg][n] (the
// super-sample term resolved along chi as one more Gram column).
void launch_gfactor(const DevTables &T, const int32_t *cfgT, int n_cfg, const SubList &sl, const double *U,
                    const double *R, const double *sw, double sq_omega, int n_mg, double *G, double *Gmax,
                    hipStream_t s);
void launch_tfactor(const DevTables &T, const int32_t *rowR, const int32_t *cfgT, int64_t n_R, const double *Gmax,
                    double *Ts, int32_t *sexp, hipStream_t s);
// fmt: 0 = f64, 1 = bf16 (hi only), 2 = bf16 hi + lo, 3 = f32.  f64 and f32
// are row-major with row pitch lda; bf16 operands are k-blocked: element
// (r, k) at ((k / GRAM_KB) r_pad + r) GRAM_KB + k % GRAM_KB, so that the
// GRAM_KB columns of a run of rows (one Gram stage of a row panel) are one
// contiguous block (k_pad is a multiple of GRAM_KB).
constexpr int GRAM_KB = 32;
// panel_f, lim (fmt 2 only): write the lo half only for panels that can
// take the split product (WLC_BF16_AUTO); nullptr writes it everywhere.
// arow: the distinct row of each A-row (-1 past the distinct rows); ext
// (bf16 formats): the k-blocks each 256-row panel of A-rows needs (see
// launch_panel_ext), written only that far (the FP32 and FP64 formats write
// every k-block).  nullptr: A-row = distinct row, every k-block.
void launch_abuild(int fmt, const int32_t *rowR, const double *Ts, const double *G, int64_t n_R, int64_t r_pad,
                   int n_chi, int n_m, int64_t k_pad, int64_t lda, void *A0, void *A1, hipStream_t s,
                   const double *panel_f = nullptr, double lim = 0.0, const int32_t *arow = nullptr,
                   const int32_t *ext = nullptr);
// Per 256-row panel of A-rows, ext[P] = the 32-column k-blocks up to the last
// chi node where T (Ts [n_R][n_chi]) of one of its rows is nonzero: the
// factor of a row is zero beyond it (T carries the lensing kernels).
void launch_panel_ext(const double *Ts, const int32_t *arow, int64_t r_pad, int n_chi, int n_mg, int64_t k_pad,
                      int32_t *ext, hipStream_t s);

// Two-leg factors of the projected one-halo trispectrum (P.T term): G2
// [n2][n_chi][n_m] and Ts2 [rows][n_chi] for the n2 = n_ell (n_ell + 1) / 2
// ell-bin pairs p <= q (p = q first) and their bin rows.
void launch_twoleg(const DevTables &T, int n_ell, const double *U, double *G2, double *Ts2, hipStream_t s);

// ---- survey window (k_window.hip): sigma_W^2 at every chi node, the
// trapezoid rule in ln eps on WINDOW_NODES nodes over the k table
constexpr int WINDOW_NODES = 16384;
void launch_sigma_w2(const DevTables &T, double theta, double *sw, hipStream_t s);

// ---- Gram product (k_gram.hip): lower-triangle tiles of A A^T
struct GramShape {
  int64_t r_pad;   // padded rows (multiple of the tile)
  int64_t k_pad;   // padded contraction length
  int64_t ld_out;  // leading dimension of the output
  int64_t lda;     // row pitch of A in elements (>= k_pad); bf16 operands are k-blocked instead
};
size_t gram_partial_bytes(int prec, const GramShape &g);
// panel_f, split_lim: WLC_BF16_AUTO only (see k_gram.hip); ignored otherwise.
// panel_ext: per 256-row panel the 32-column k-blocks where its rows can be
// nonzero; a tile then sums only the first min over its two panels (the
// rest are zero products).  nullptr: every k-block.
void launch_gram(int prec, const GramShape &g, const void *A0, const void *A1, void *out, void *partial,
                 hipStream_t s, const double *panel_f = nullptr, double split_lim = 0.0,
                 const int32_t *panel_ext = nullptr);
// Batched bf16 Gram products (one persistent launch over the work items of
// several products, e.g. of the requests of a server).  A product in a
// batch computes exactly what launch_gram computes for it: the same tiles,
// k slices and partial buffer, followed by its own launch_gram_reduce.
struct GramJob {
  const void *A0, *A1;   // hi (and lo) operands, k-blocked
  void *out, *partial;   // FP32 output and split-K partials
  int64_t r_pad, k_pad, k_split, ld, part_stride;
  int64_t n_work;        // work items: tiles x n_split
  int64_t item0;         // first item of this product in the batch (set by the caller)
  const double *panel_f; // WLC_BF16_AUTO: per-panel largest one-halo share
  double split_lim;      // WLC_BF16_AUTO: split tile (I, J) iff panel_f[I] panel_f[J] > split_lim
  const int32_t *panel_ext;  // per panel the k-blocks that can be nonzero (nullptr: all)
  int32_t n_split, nt;
};
bool gram_batchable(int prec);  // the bf16 precisions
void gram_job(int prec, const GramShape &g, const void *A0, const void *A1, void *out, void *partial, GramJob &job,
              const double *panel_f = nullptr, double split_lim = 0.0, const int32_t *panel_ext = nullptr);
// counters: N_XCD x 16 uint32 of device scratch, cleared by the launch itself
constexpr int GRAM_BATCH_COUNTERS = 8 * 16;
int launch_gram_batch(int prec, const GramJob *jobs_dev, int n_jobs, int64_t total, uint32_t *counters,
                      hipStream_t s);
void launch_gram_reduce(int prec, const GramShape &g, void *out, void *partial, hipStream_t s);
// One-halo product through the chi factorisation (k_chifact.hip): H (scratch,
// n_cfg^2 n_chi doubles) from the configuration factors G, then the lower
// triangle of out[e][f] = sum_n Ts[e][n] Ts[f][n] H[c(e)][c(f)][n] over the
// distinct rows, grouped by configuration in blocks of sp (power spectrum)
// and sb (bispectrum) rows.
void launch_chifact(const double *Ts, const double *G, double *H, int n_cfg, int n_chi, int n_m, int nl, int sp,
                    int sb, int n_tri, double *out, int64_t ld, hipStream_t s);
// Copy the lower triangle of the first n rows/columns of G (row pitch ld,
// f32 or f64) onto the upper one, so that G is exactly symmetric.
void launch_gram_mirror(int f32, void *G, int64_t n, int64_t ld, hipStream_t s);
// G[e][f] = GP[pos[e]][pos[f]] for e, f < n (both triangles, f32 or f64,
// pitch ld): the product of the A-rows (GP, made symmetric first) back in the
// order of the distinct rows.
void launch_gram_unpermute(int f32, const void *GP, const int32_t *pos, int64_t n, int64_t ld, void *G,
                           hipStream_t s);
// Whether the FP64 product of this shape runs on 128 x 256 tiles (else on
// the 128 x 128 tiles of the FP32 product).
bool gram_f64_tiles(const GramShape &g);

// ---- assembly (k_assemble.hip)
struct AsmArgs {
  const int32_t *rowO;    // [n][8]: cfg, e, z0, z1, z2, l0, l1, l2
  const int32_t *cfgT;    // [n_cfg][4]: kind, l0, l1, l2
  const int32_t *sexp;    // [n_R] row exponents of A
  const void *Gm;         // [r_pad][r_pad], f64 or f32, symmetric on the first n_R rows
  int64_t ld_g;
  int gm_f32;
  const double *Ps;       // [n_ell][n_z][n_z]
  const double *nmodes;   // [n_ell]
  const double *ntri;     // [n_tri]
  const double *rR, *dR;  // [n_R]
  int n_z, n_ell;
  int64_t n;              // output rows
  double inv_omega, omega, sigma_b2;
  // B.B, P.T and P.B in-survey terms (eqs. CovBB, Covpb), when ngins != 0:
  int ngins;
  const double *T2;       // two-leg trispectrum, lower triangle, pitch ld_t2
  int64_t ld_t2;
};
void launch_rowexp(const AsmArgs &a, int32_t *row_exp2, double *d, double *r, hipStream_t s);
// WLC_BF16_AUTO: the largest one-halo share f_a = C1h_aa / C_aa of the data
// rows of every 256-row panel of distinct rows, into F [n_panels], and the
// largest of all into F[n_panels], from the
// Gram factors in FP64 before the product: S [n_cfg][n_chi] and gd [n_R]
// are scratch.  C_aa leaves out the in-survey terms (positive on the
// diagonal), so F errs on the large side.
// pos (nullptr: identity) maps a distinct row to its A-row, whose panel F holds.
void launch_split_plan(const AsmArgs &a, const int32_t *rowR, const double *Ts, const double *G, int64_t n_R,
                       int n_cfg, int n_chi, int n_mg, double *S, double *gd, double *F, int n_panels, hipStream_t s,
                       const int32_t *pos = nullptr);
// C in the type of the one-halo block Gm: FP32 when gm_f32, else FP64.
void launch_assemble(const AsmArgs &a, const int32_t *row_exp2, void *C, hipStream_t s);

// ---- signal-to-noise (k_chol.hip)
// perm (optional): row/column a of the bordered matrix is row perm[a] of C
void launch_chol_prep(const void *C, int c_f32, const int32_t *row_exp2, const double *d, int64_t n, int64_t ld,
                      double *Wm, hipStream_t s, const int32_t *perm = nullptr);
// Optional per-launch timing of the trailing-update kernel: event pairs are
// recorded around each launch while count < cap; flops accumulates the
// algorithmic flops of every launch.
struct KernelProbe {
  hipEvent_t *ev = nullptr;
  int cap = 0;
  int count = 0;
  int64_t launches = 0;
  double flops = 0.0;
};
int chol_factor(double *Wm, int64_t n, int64_t ld, double *scratch, int *flag, hipStream_t s,
                KernelProbe *probe = nullptr);
int64_t update2_max_slices(int64_t k_len);
size_t chol_scratch_bytes(int64_t n);
int64_t chol_part_rows(int64_t n);
// part: split-k scratch of part_rows x 256 doubles (NULL: no split)
void launch_update2(double *Wm, int64_t ld, int64_t c0, int64_t r1, int64_t c1, int64_t k0, int64_t k1,
                    double *part, int64_t part_rows, hipStream_t s, KernelProbe *probe = nullptr);
void launch_sumsq_row(const double *Wm, int64_t n, int64_t ld, double *out, hipStream_t s);
// out[g] = sum of y_j^2 over j < ends[g] (y: the last row of the bordered
// factor); part: ng doubles of scratch
void launch_sumsq_groups(const double *Wm, int64_t n, int64_t ld, const int32_t *ends, int ng, double *part,
                         double *out, hipStream_t s);

// ---- S/N through the distinct rows (k_woodbury.hip)
// Distinct rows are grouped by configuration: nl power-spectrum blocks of sp
// rows, then n_tri bispectrum blocks of sb rows.
struct BlockMap {
  int nl, n_tri, sp, sb;
  int64_t n_R;
  __host__ __device__ int blk(int64_t e) const {
    return e < (int64_t)nl * sp ? (int)(e / sp) : nl + (int)((e - (int64_t)nl * sp) / sb);
  }
  __host__ __device__ int64_t start(int c) const {
    return c < nl ? (int64_t)c * sp : (int64_t)nl * sp + (int64_t)(c - nl) * sb;
  }
  __host__ __device__ int size(int c) const { return c < nl ? sp : sb; }
  // offset of block c in a packed array of square blocks
  __host__ __device__ int64_t off(int c) const {
    return c < nl ? (int64_t)c * sp * sp : (int64_t)nl * sp * sp + (int64_t)(c - nl) * sb * sb;
  }
};
struct WoodArgs {
  BlockMap B;
  int n_ell, nz;                  // ell-bins used, redshift bins (nz <= 32)
  const double *Ps, *nmodes, *ntri, *dR, *rR;
  const int32_t *cfgT, *sexp;
  const void *Gm;                 // symmetric Gram of the run, pitch ld_g
  int gm_f32;
  int64_t ld_g;
  double omega, sigma_b2;
  double *Q;                      // [n_ell][nz][nz]
  double *Gb;                     // packed blocks of G
  double *rhat;                   // [n_R]
  int32_t *tau;                   // [n_R]
  double *T;                      // [n_R][ld_t]
  int64_t ld_t;
  double *W;                      // [n_R + 1][ld_w], bordered I + Z
  int64_t ld_w;
  int *flag;
};
constexpr int WOOD_NZ_MAX = 32;
void launch_woodbury(const WoodArgs &w, hipStream_t s);

// ---- principal components (k_pca.hip): one-sided block Jacobi on the rows
// of X (n_pad x n_pad, n_pad a multiple of 64 and at most 65535)
void launch_pca_init(const double *Wm, int64_t ld, const int32_t *t, int64_t n, int64_t n_pad, double *X, double *V,
                     double *y, hipStream_t s);
// one round r of the tournament; part: [pairs][pca_slices][64][64], Qg:
// [pairs][64][64] doubles, rot: [pairs] int32 of scratch
int pca_slices(int64_t n_pad);
void launch_pca_round(double *X, double *V, int64_t n_pad, int r, double tol, int max_inner, double *conv,
                      double *part, double *Qg, int32_t *rot, hipStream_t s);
void launch_pca_finish(const double *X, const double *y, const double *Vr, int64_t n, int64_t n_pad, double *lam,
                       double *snr2, int32_t *rank_lam, int32_t *rank_snr, double *lam_out, double *snr2_out,
                       double *desc, double *S, hipStream_t s);

// ---- lattice counts (k_lattice.hip); thr_max = largest threshold used
void launch_lattice(const int64_t *thr_dev, int64_t thr_max, int n_ell, const int32_t *tri, int n_tri,
                    uint64_t *modes, uint64_t *tris, hipStream_t s);

// ---- utilities (api.hip)
void launch_fill_i32(int32_t *p, int n, int32_t v, hipStream_t s);

}  // namespace wlc
