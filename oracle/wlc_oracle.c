/*
 * wlc_oracle.c -- plain, slow FP64 CPU oracle for the tomographic weak-lensing
 * power-spectrum / bispectrum data vector and joint covariance.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this file's library.  It shares no
 * code, header, table or constant generator with the HIP library; the two
 * meet only in the synthetic input tables.
 *
 * Every function below follows one passage of Rizzato, Benabed, Bernardeau &
 * Lacasa (2019), "Tomographic weak lensing bispectrum" (arXiv 1812.07437),
 * cited by section and equation label, and evaluates it literally in double
 * precision: no blocking, no factorisation of sums, no reordering beyond
 * what the equations state.  Values that depend only on a point (an
 * interpolated table value at one k, the 3-D spectrum at one (configuration,
 * chi) node) are tabulated once where they are needed many times; tabulation
 * calls the same function with the same arguments, so it changes no bit.
 *
 * Readings of points the paper leaves open (grids, interpolation, the
 * undefined B_G2, the super-sample form) are stated where they are used.
 *
 * Parity unpinned: the B_G2 term of the bispectrum response.  The paper uses
 * B_G2 without defining it; the tidal-kernel reading below is pinned only to
 * itself (its values at the equilateral and right-isosceles triangles), not
 * to anything the paper fixes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int n_z, n_chi, n_k, n_m;
  const double *chi, *w_chi; /* [n_chi] line-of-sight nodes and weights */
  const double *k;           /* [n_k] strictly increasing                 */
  const double *m, *w_m;     /* [n_m] masses and quadrature weights       */
  const double *W;           /* [n_z][n_chi] lensing kernels              */
  const double *P;           /* [n_chi][n_k] linear power at each chi     */
  const double *u;           /* [n_m][n_k] halo profile                   */
  const double *nmf;         /* [n_m] mass function n(M)                 */
  const double *b1, *b2;     /* [n_m] or NULL: b1 = 1, b2 = 0             */
  double rho;                /* comoving mean matter density              */
  double k_max;              /* hard cut on the line-of-sight integrand   */
} or_tables;

/* A data-vector row: kind 2 (power spectrum, one ell-bin used twice) or
 * kind 3 (bispectrum, a triangle of ell-bins); zbin[] are redshift bins. */
typedef struct {
  int kind;
  int lbin[3];
  int zbin[3];
} or_row;

static int g_range_error = 0; /* set when a needed k lies outside the table */

int or_range_error(void) { return g_range_error; }
void or_clear_error(void) { g_range_error = 0; }

/* --------------------------------------------------------------------
 * Table interpolation.  The paper evaluates analytic inputs; with tables
 * we read X(k) = exp(linear interpolation of ln X in ln k) between the two
 * bracketing nodes.  This is exact for power laws. */
static int bracket(const double *kg, int nk, double kk, int *j, double *t) {
  if (!(kk >= kg[0] && kk <= kg[nk - 1])) return -1;
  int lo = 0, hi = nk - 1; /* kg[lo] <= kk, and hi is past it or the end */
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (kg[mid] <= kk) lo = mid; else hi = mid;
  }
  if (lo == nk - 1) lo = nk - 2;
  *j = lo;
  *t = (log(kk) - log(kg[lo])) / (log(kg[lo + 1]) - log(kg[lo]));
  return 0;
}

double or_interp(const double *kg, const double *row, int nk, double kk) {
  int j; double t;
  if (bracket(kg, nk, kk, &j, &t)) { g_range_error = 1; return NAN; }
  return exp((1.0 - t) * log(row[j]) + t * log(row[j + 1]));
}

/* Logarithmic slope d ln P / d ln k: centred differences at the nodes
 * (one-sided at the two ends), then linear interpolation in ln k. */
static double node_slope(const double *kg, const double *row, int nk, int j) {
  int a = j > 0 ? j - 1 : 0;
  int b = j < nk - 1 ? j + 1 : nk - 1;
  return (log(row[b]) - log(row[a])) / (log(kg[b]) - log(kg[a]));
}

double or_neff(const double *kg, const double *row, int nk, double kk) {
  int j; double t;
  if (bracket(kg, nk, kk, &j, &t)) { g_range_error = 1; return NAN; }
  return (1.0 - t) * node_slope(kg, row, nk, j) + t * node_slope(kg, row, nk, j + 1);
}

/* --------------------------------------------------------------------
 * Halo-model mass integral I_mu^beta(k_1..k_mu), eq. ImunuHalos (Sec. 4.1):
 *   sum_m w_m b_beta(m) (m/rho)^mu n(m) prod_a u(m, k_a),  b_0 = 1.
 * No concentration scatter: u carries no c_v axis (model B of Sec. 5.4). */
static double bias(const or_tables *T, int beta, int mi) {
  if (beta == 0) return 1.0;
  if (beta == 1) return T->b1 ? T->b1[mi] : 1.0;
  return T->b2 ? T->b2[mi] : 0.0;
}

double or_halo_I(const or_tables *T, int mu, int beta, const double *ks) {
  double s = 0.0;
  for (int mi = 0; mi < T->n_m; ++mi) {
    double x = T->w_m[mi] * bias(T, beta, mi) * pow(T->m[mi] / T->rho, mu) * T->nmf[mi];
    for (int a = 0; a < mu; ++a) x *= or_interp(T->k, T->u + (size_t)mi * T->n_k, T->n_k, ks[a]);
    s += x;
  }
  return s;
}

/* Tree-level kernel F2 for two sides of a closed triangle whose third side is
 * kl; mu is the cosine between the two wavevectors (k_i + k_j = -k_l).  The
 * paper refers to the tree-level bispectrum without printing it; this is the
 * standard Einstein-de Sitter kernel. */
static double cosine(double ki, double kj, double kl) {
  return (kl * kl - ki * ki - kj * kj) / (2.0 * ki * kj);
}

double or_F2(double ki, double kj, double kl) {
  double mu = cosine(ki, kj, kl);
  return 5.0 / 7.0 + 0.5 * mu * (ki / kj + kj / ki) + 2.0 / 7.0 * mu * mu;
}

/* --------------------------------------------------------------------
 * 3-D spectra and their responses at one chi node n.
 *
 * kind 2 at k:  P_HM = I_2^0(k,k) + [I_1^1(k)]^2 P(k)          (eq. PspHMtot2)
 *               R_P  = [I_1^1]^2 (47/21 P - (1/3) dP/dlnk) + I_2^1(k,k)
 *                                                  (eqs. PowerHMResp, RespP)
 * kind 3 at (k1,k2,k3):
 *   B_HM = I_3^0 + sum_cyc I_1^1(k1) I_2^1(k2,k3) P(k1) + prod I_1^1 B_PT
 *          (eqs. B1halo, B2halos, first line of B3halos, BspHMtot)
 *   B_PT = sum over the three pairs of 2 F2(k_i,k_j) P_i P_j
 *   R_B  = prod I_1^1 [433/126 B_PT + 5/126 B_G2 - (1/3) sum_i dB_PT/dln k_i]
 *          + sum_cyc [I_1^1(k1) I_2^2(k2,k3) P(k1) + I_1^1(k1) I_2^1(k2,k3) R_lin(k1)]
 *          + I_3^1                                   (eqs. BispHMResp, RespB)
 * Readings: the mass-integral derivative raises the bias order (I_mu^{beta+1});
 * a bare "k" in the responses is the first leg; B_G2 = 2 sum_pairs
 * (mu_ij^2 - 1) P_i P_j; F2 depends only on ratios, so sum_i dB_PT/dln k_i =
 * sum_pairs 2 F2 P_i P_j (n_i + n_j) with n = dlnP/dlnk.
 * Returns 0 (and X = R = 0) when the largest k exceeds k_max (Sec. 4.4). */
int or_spectrum(const or_tables *T, int n, int kind, const double *kv, double *X, double *R) {
  const double *Pn = T->P + (size_t)n * T->n_k;
  double kmx = kv[0];
  for (int a = 1; a < kind; ++a) if (kv[a] > kmx) kmx = kv[a];
  if (kmx > T->k_max) { *X = 0.0; *R = 0.0; return 0; }
  if (kind == 2) {
    double k = kv[0];
    double kk[2] = {k, k};
    double I11 = or_halo_I(T, 1, 1, kk);
    double I20 = or_halo_I(T, 2, 0, kk);
    double I21 = or_halo_I(T, 2, 1, kk);
    double P = or_interp(T->k, Pn, T->n_k, k);
    double ne = or_neff(T->k, Pn, T->n_k, k);
    double Rlin = 47.0 / 21.0 * P - ne * P / 3.0;
    *X = I20 + I11 * I11 * P;
    *R = I11 * I11 * Rlin + I21;
    return 1;
  }
  double P[3], ne[3], I11[3], Rlin[3];
  for (int a = 0; a < 3; ++a) {
    double ka[1] = {kv[a]};
    P[a] = or_interp(T->k, Pn, T->n_k, kv[a]);
    ne[a] = or_neff(T->k, Pn, T->n_k, kv[a]);
    I11[a] = or_halo_I(T, 1, 1, ka);
    Rlin[a] = 47.0 / 21.0 * P[a] - ne[a] * P[a] / 3.0;
  }
  double I30 = or_halo_I(T, 3, 0, kv);
  double I31 = or_halo_I(T, 3, 1, kv);
  /* cyclic terms: leg a alone, the other two (b, c) inside one halo */
  double two_halo = 0.0, resp_cyc = 0.0;
  for (int a = 0; a < 3; ++a) {
    int b = (a + 1) % 3, c = (a + 2) % 3;
    double kbc[2] = {kv[b], kv[c]};
    double I21 = or_halo_I(T, 2, 1, kbc);
    double I22 = or_halo_I(T, 2, 2, kbc);
    two_halo += I11[a] * I21 * P[a];
    resp_cyc += I11[a] * I22 * P[a] + I11[a] * I21 * Rlin[a];
  }
  double Bpt = 0.0, Bg2 = 0.0, dil = 0.0;
  for (int a = 0; a < 3; ++a) {
    int i = a, j = (a + 1) % 3, l = (a + 2) % 3;
    double F = or_F2(kv[i], kv[j], kv[l]);
    double mu = cosine(kv[i], kv[j], kv[l]);
    Bpt += 2.0 * F * P[i] * P[j];
    Bg2 += 2.0 * (mu * mu - 1.0) * P[i] * P[j];
    dil += 2.0 * F * P[i] * P[j] * (ne[i] + ne[j]);
  }
  double I111 = I11[0] * I11[1] * I11[2];
  *X = I30 + two_halo + I111 * Bpt;
  *R = I111 * (433.0 / 126.0 * Bpt + 5.0 / 126.0 * Bg2 - dil / 3.0) + resp_cyc + I31;
  return 1;
}

/* Tabulate the 3-D spectra for a list of ell-configurations at every chi
 * node: cfg_kind[c] in {2,3}, cfg_ell[c][3] the ell values (sorted). */
void or_spectra_table(const or_tables *T, int n_cfg, const int *cfg_kind, const double *cfg_ell,
                      double *X, double *R) {
#pragma omp parallel for schedule(dynamic) collapse(2)
  for (int c = 0; c < n_cfg; ++c)
    for (int n = 0; n < T->n_chi; ++n) {
      double kv[3];
      for (int a = 0; a < cfg_kind[c]; ++a) kv[a] = cfg_ell[3 * c + a] / T->chi[n];
      or_spectrum(T, n, cfg_kind[c], kv, &X[(size_t)c * T->n_chi + n], &R[(size_t)c * T->n_chi + n]);
    }
}

/* --------------------------------------------------------------------
 * Limber projection, eq. nProjection (Sec. 3.1): the n-th order convergence
 * polyspectrum is int dchi chi^(2-2n) prod_i W_i(chi) P_3D(l_a/chi).  The
 * integral is the midpoint/trapezoid sum with the supplied weights.  The W
 * product runs over the bins sorted ascending (canonical order). */
static void sort_int(int *v, int n) {
  for (int a = 1; a < n; ++a)
    for (int b = a; b > 0 && v[b - 1] > v[b]; --b) { int t = v[b]; v[b] = v[b - 1]; v[b - 1] = t; }
}

/* d[r] and the response vector r[r] for n_rows rows; row_cfg[r] indexes the
 * tabulated spectra of its ell-configuration. */
void or_project(const or_tables *T, int n_rows, const int *row_kind, const int *row_z,
                const int *row_cfg, const double *X, const double *R, double *d, double *r) {
#pragma omp parallel for schedule(static)
  for (int a = 0; a < n_rows; ++a) {
    int p = row_kind[a];
    int z[3];
    for (int q = 0; q < p; ++q) z[q] = row_z[3 * a + q];
    sort_int(z, p);
    double sd = 0.0, sr = 0.0;
    for (int n = 0; n < T->n_chi; ++n) {
      double chi = T->chi[n];
      double tw = T->w_chi[n] * pow(chi, 2.0 - 2.0 * p);
      for (int q = 0; q < p; ++q) tw *= T->W[(size_t)z[q] * T->n_chi + n];
      sd += tw * X[(size_t)row_cfg[a] * T->n_chi + n];
      sr += tw * R[(size_t)row_cfg[a] * T->n_chi + n];
    }
    d[a] = sd;
    r[a] = sr;
  }
}

/* --------------------------------------------------------------------
 * One-halo (NGins) covariance between two rows, eqs. CovPPNG, Ins6P and
 * Ins5P with eq. General1h: (1/Omega) times the Limber projection of the
 * 1-halo (p_a+p_b)-point function I^0 at all legs of both rows:
 *   (1/Omega) sum_n w_n chi_n^(2-2(p_a+p_b)) prod W * sum_m w_m n_m
 *            (m/rho)^(p_a+p_b) prod_legs u(m, l/chi_n),
 * zero at nodes where any leg exceeds k_max.  A power-spectrum row brings
 * its ell twice (the pair l, -l).  Legs and bins are taken sorted.
 * U[(b*n_chi + n)*n_m + mi] holds u(m_mi, ell_b/chi_n) for every distinct
 * ell value b (tabulated by or_tab_u). */
void or_tab_u(const or_tables *T, int n_ell, const double *ell, double *U) {
#pragma omp parallel for collapse(2) schedule(static)
  for (int b = 0; b < n_ell; ++b)
    for (int n = 0; n < T->n_chi; ++n) {
      double kk = ell[b] / T->chi[n];
      for (int mi = 0; mi < T->n_m; ++mi)
        U[((size_t)b * T->n_chi + n) * T->n_m + mi] =
            kk > T->k_max ? 0.0 : or_interp(T->k, T->u + (size_t)mi * T->n_k, T->n_k, kk);
    }
}

/* mass weight w_m n_m (m/rho)^npt, tabulated for npt = 0..6 */
static double *mass_weights(const or_tables *T) {
  double *mw = (double *)malloc(sizeof(double) * 7 * (size_t)T->n_m);
  for (int p = 0; p < 7; ++p)
    for (int mi = 0; mi < T->n_m; ++mi)
      mw[(size_t)p * T->n_m + mi] = T->w_m[mi] * T->nmf[mi] * pow(T->m[mi] / T->rho, p);
  return mw;
}

static double cov1h(const or_tables *T, const double *ell, const double *U, const double *mw,
                    double omega, const int *ka, const int *la, const int *za,
                    const int *kb, const int *lb, const int *zb) {
  int z[6], legs[6];
  int nz = 0, nl = 0;
  for (int q = 0; q < *ka; ++q) z[nz++] = za[q];
  for (int q = 0; q < *kb; ++q) z[nz++] = zb[q];
  /* ell legs: a P row contributes its bin twice */
  if (*ka == 2) { legs[nl++] = la[0]; legs[nl++] = la[0]; }
  else for (int q = 0; q < 3; ++q) legs[nl++] = la[q];
  if (*kb == 2) { legs[nl++] = lb[0]; legs[nl++] = lb[0]; }
  else for (int q = 0; q < 3; ++q) legs[nl++] = lb[q];
  sort_int(z, nz);
  /* sort legs by their ell value (bins are ordered by ell) */
  sort_int(legs, nl);
  int npt = nl; /* order of the polyspectrum */
  double lmax = 0.0;
  for (int q = 0; q < nl; ++q) if (ell[legs[q]] > lmax) lmax = ell[legs[q]];
  double total = 0.0;
  for (int n = 0; n < T->n_chi; ++n) {
    double chi = T->chi[n];
    if (lmax / chi > T->k_max) continue;
    double tw = T->w_chi[n] * pow(chi, 2.0 - 2.0 * npt);
    for (int q = 0; q < nz; ++q) tw *= T->W[(size_t)z[q] * T->n_chi + n];
    double sm = 0.0;
    for (int mi = 0; mi < T->n_m; ++mi) {
      double x = mw[(size_t)npt * T->n_m + mi];
      for (int q = 0; q < nl; ++q) x *= U[((size_t)legs[q] * T->n_chi + n) * T->n_m + mi];
      sm += x;
    }
    total += tw * sm;
  }
  return total / omega;
}

/* rows are given as arrays kind[N], lbin[N][3], zbin[N][3] */
void or_cov1h_pairs(const or_tables *T, const double *ell, const double *U, double omega,
                    const int *kind, const int *lbin, const int *zbin,
                    int64_t n_pairs, const int64_t *pairs, double *out) {
  double *mw = mass_weights(T);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t q = 0; q < n_pairs; ++q) {
    int64_t a = pairs[2 * q], b = pairs[2 * q + 1];
    out[q] = cov1h(T, ell, U, mw, omega, &kind[a], &lbin[3 * a], &zbin[3 * a],
                   &kind[b], &lbin[3 * b], &zbin[3 * b]);
  }
  free(mw);
}

/* --------------------------------------------------------------------
 * Gaussian covariance.
 * Power spectrum, eq. CovPPG (Sec. 3.2.2):
 *   delta_{l l'} / N(l) [P^s_{ii'} P^s_{jj'} + P^s_{ij'} P^s_{ji'}],
 * bispectrum (App. B, Gauss term):
 *   (Omega / N_tri) sum over the 6 maps sigma of primed legs onto unprimed
 *   legs of prod_a P^s_{i_a i'_sigma(a)}(l_a) delta_K(l_a, l'_sigma(a)),
 * and no Gaussian power-spectrum / bispectrum cross term (eq. CovPBsynt).
 * Ps[(b*n_z + i)*n_z + j] is the shot-noise power (eq. ShotNoise) at the
 * centre of ell-bin b; nmodes[b] = N(l_b); ntri[t] = N_tri of triangle t
 * (row "cfg" for B rows is the triangle index). */
static const int PERM6[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

static double gauss(int n_z, const double *Ps, const double *nmodes, const double *ntri, double omega,
                    int ka, const int *la, const int *za, int ta,
                    int kb, const int *lb, const int *zb, int tb) {
#define PS(b, i, j) Ps[((size_t)(b) * n_z + (i)) * n_z + (j)]
  if (ka != kb) return 0.0;
  if (ka == 2) {
    if (la[0] != lb[0]) return 0.0;
    int b = la[0];
    return (PS(b, za[0], zb[0]) * PS(b, za[1], zb[1]) + PS(b, za[0], zb[1]) * PS(b, za[1], zb[0])) / nmodes[b];
  }
  if (ta != tb) return 0.0;
  double s = 0.0;
  for (int p = 0; p < 6; ++p) {
    const int *sg = PERM6[p];
    double term = 1.0;
    for (int a = 0; a < 3; ++a) {
      if (la[a] != lb[sg[a]]) { term = 0.0; break; }
      term *= PS(la[a], za[a], zb[sg[a]]);
    }
    s += term;
  }
  return omega / ntri[ta] * s;
#undef PS
}

void or_gauss_pairs(int n_z, const double *Ps, const double *nmodes, const double *ntri, double omega,
                    const int *kind, const int *lbin, const int *zbin, const int *tri,
                    int64_t n_pairs, const int64_t *pairs, double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < n_pairs; ++q) {
    int64_t a = pairs[2 * q], b = pairs[2 * q + 1];
    out[q] = gauss(n_z, Ps, nmodes, ntri, omega, kind[a], &lbin[3 * a], &zbin[3 * a], tri[a],
                   kind[b], &lbin[3 * b], &zbin[3 * b], tri[b]);
  }
}

/* --------------------------------------------------------------------
 * Full covariance on the lower triangle, mirrored:
 *   C = C_Gauss + C_1h + sigma_b^2 r r^T.
 * The last term is the super-sample covariance of eq. WLSSCflatskyLimber
 * read as a single coherent long mode of variance sigma_b^2 (rank one).
 * One-halo entries are computed for the canonical rows only (rows whose
 * value is fixed by the multiset of bins and legs; canon[a] names the row
 * holding the value for row a, c1h_canon is their [nc][nc] lower part). */
void or_cov_full(int n, const double *c1h_canon, int nc, const int *canon,
                 int n_z, const double *Ps, const double *nmodes, const double *ntri, double omega,
                 const int *kind, const int *lbin, const int *zbin, const int *tri,
                 const double *r, double sigma_b2, double *C) {
#pragma omp parallel for schedule(dynamic, 8)
  for (int a = 0; a < n; ++a)
    for (int b = 0; b <= a; ++b) {
      int ca = canon[a], cb = canon[b];
      int hi = ca > cb ? ca : cb, lo = ca > cb ? cb : ca;
      double g = gauss(n_z, Ps, nmodes, ntri, omega, kind[a], &lbin[3 * a], &zbin[3 * a], tri[a],
                       kind[b], &lbin[3 * b], &zbin[3 * b], tri[b]);
      double v = g + c1h_canon[(size_t)hi * nc + lo] + sigma_b2 * r[a] * r[b];
      C[(size_t)a * n + b] = v;
      C[(size_t)b * n + a] = v;
    }
}

/* Bin-averaged one-halo covariance (the average over the modes of each bin
 * that the paper replaces by the bin centres, Sec. 3.2.2 and the discussion
 * of Sec. 7): the one-halo term of eq. General1h averaged over the sub-bin
 * entries of both rows,
 *   sum_e sum_f w_e w_f C_1h(legs of entry e of row a, legs of entry f of row b),
 * entries off[c] .. off[c+1]-1 of the row's configuration c, each with three
 * legs leg[3 e + q] indexing ell_sub / U_sub and a weight w[e]. */
void or_cov1h_avg_pairs(const or_tables *T, const double *ell_sub, const double *U_sub, double omega,
                        const int *kind, const int *zbin, const int *cfg, const int *off, const int *leg,
                        const double *w, int64_t n_pairs, const int64_t *pairs, double *out) {
  double *mw = mass_weights(T);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t q = 0; q < n_pairs; ++q) {
    int64_t a = pairs[2 * q], b = pairs[2 * q + 1];
    int ca = cfg[a], cb = cfg[b];
    double s = 0.0;
    for (int e = off[ca]; e < off[ca + 1]; ++e)
      for (int f = off[cb]; f < off[cb + 1]; ++f)
        s += w[e] * w[f] * cov1h(T, ell_sub, U_sub, mw, omega, &kind[a], &leg[3 * e], &zbin[3 * a], &kind[b],
                                 &leg[3 * f], &zbin[3 * b]);
    out[q] = s;
  }
  free(mw);
}

/* --------------------------------------------------------------------
 * Projected one-halo trispectrum at four legs: the Limber projection of
 * eq. nProjection with n = 4 applied to I_4^0 of eq. ImunuHalos,
 *   sum_n w_n chi_n^-6 prod_q W_{z_q}(chi_n)
 *         sum_m w_m n_m (m/rho)^4 prod_q u(m, l_q / chi_n),
 * zero at nodes where a leg exceeds k_max (U is zero there).  legs[q] are
 * ell-bin indices, z[q] redshift bins. */
static double trispec(const or_tables *T, const double *ell, const double *U, const double *mw,
                      const int legs[4], const int z[4]) {
  double lmax = 0.0;
  for (int q = 0; q < 4; ++q) if (ell[legs[q]] > lmax) lmax = ell[legs[q]];
  double total = 0.0;
  for (int n = 0; n < T->n_chi; ++n) {
    double chi = T->chi[n];
    if (lmax / chi > T->k_max) continue;
    double tw = T->w_chi[n] * pow(chi, -6.0);
    for (int q = 0; q < 4; ++q) tw *= T->W[(size_t)z[q] * T->n_chi + n];
    double sm = 0.0;
    for (int mi = 0; mi < T->n_m; ++mi) {
      double x = mw[(size_t)4 * T->n_m + mi];
      for (int q = 0; q < 4; ++q) x *= U[((size_t)legs[q] * T->n_chi + n) * T->n_m + mi];
      sm += x;
    }
    total += tw * sm;
  }
  return total;
}

double or_trispec(const or_tables *T, const double *ell, const double *U, const int *legs, const int *z) {
  double *mw = mass_weights(T);
  double v = trispec(T, ell, U, mw, legs, z);
  free(mw);
  return v;
}

/* --------------------------------------------------------------------
 * The in-survey non-Gaussian terms of App. B built from lower-order
 * spectra: B.B and P.T between two bispectrum rows (eq. CovBB), P.B between
 * a power-spectrum and a bispectrum row (eq. Covpb).  Each term needs one leg
 * of the first row to lie in the same ell-bin as one leg of the second
 * (the Kronecker deltas), and carries 2 pi / (Omega l Delta l) = 1 / N(l)
 * for that bin.  Summing over the three legs a of the first row and the
 * three legs b of the second reproduces the printed bracket and its two
 * permutations:
 *   B.B: B[first row with bin z_a replaced by z'_b]
 *        * B[second row with bin z'_b replaced by z_a]
 *   P.T: P^s_{z_a z'_b}(l_a) * T(the two other legs of each row)
 *   P.B: for a power-spectrum row (l; i, j) and bispectrum leg b in bin l:
 *        P^s_{z'_b j}(l) B[z'_b replaced by i] + P^s_{i z'_b}(l) B[z'_b replaced by j].
 * Bfull[(t * n_z + i) * n_z^2 + j * n_z + k] is the projected bispectrum of
 * triangle t with bins (i, j, k) on its legs in order (the data vector
 * value of that multiset of bins); T the projected one-halo trispectrum
 * above.  Two power-spectrum rows get nothing here (their only term beyond
 * the Gaussian one is the one-halo trispectrum, eq. CovPPNG). */
static double ngins(const or_tables *T, const double *ell, const double *U, const double *mw, int n_z,
                    const double *Ps, const double *nmodes, const double *Bfull,
                    int ka, const int *la, const int *za, int ta, int kb, const int *lb, const int *zb, int tb) {
#define PS(b, i, j) Ps[((size_t)(b) * n_z + (i)) * n_z + (j)]
#define BF(t, z) Bfull[(((size_t)(t) * n_z + (z)[0]) * n_z + (z)[1]) * n_z + (z)[2]]
  if (ka == 2 && kb == 2) return 0.0;
  if (ka == 2 || kb == 2) {
    const int *lp = ka == 2 ? la : lb, *zp = ka == 2 ? za : zb;
    const int *lt = ka == 2 ? lb : la, *zt = ka == 2 ? zb : za;
    int tt = ka == 2 ? tb : ta;
    double s = 0.0;
    for (int b = 0; b < 3; ++b) {
      if (lt[b] != lp[0]) continue;
      int zi[3] = {zt[0], zt[1], zt[2]}, zj[3] = {zt[0], zt[1], zt[2]};
      zi[b] = zp[0];
      zj[b] = zp[1];
      s += (PS(lp[0], zt[b], zp[1]) * BF(tt, zi) + PS(lp[0], zp[0], zt[b]) * BF(tt, zj)) / nmodes[lp[0]];
    }
    return s;
  }
  double s = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      if (la[a] != lb[b]) continue;
      int z1[3] = {za[0], za[1], za[2]}, z2[3] = {zb[0], zb[1], zb[2]};
      z1[a] = zb[b];
      z2[b] = za[a];
      const double bb = BF(ta, z1) * BF(tb, z2);
      int legs[4], zz[4], q = 0;
      for (int x = 0; x < 3; ++x) if (x != a) { legs[q] = la[x]; zz[q] = za[x]; ++q; }
      for (int x = 0; x < 3; ++x) if (x != b) { legs[q] = lb[x]; zz[q] = zb[x]; ++q; }
      const double pt = PS(la[a], za[a], zb[b]) * trispec(T, ell, U, mw, legs, zz);
      s += (bb + pt) / nmodes[la[a]];
    }
  return s;
#undef BF
#undef PS
}

void or_ngins_pairs(const or_tables *T, const double *ell, const double *U, int n_z, const double *Ps,
                    const double *nmodes, const double *Bfull, const int *kind, const int *lbin, const int *zbin,
                    const int *tri, int64_t n_pairs, const int64_t *pairs, double *out) {
  double *mw = mass_weights(T);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t q = 0; q < n_pairs; ++q) {
    int64_t a = pairs[2 * q], b = pairs[2 * q + 1];
    out[q] = ngins(T, ell, U, mw, n_z, Ps, nmodes, Bfull, kind[a], &lbin[3 * a], &zbin[3 * a], tri[a], kind[b],
                   &lbin[3 * b], &zbin[3 * b], tri[b]);
  }
  free(mw);
}

void or_cov1h_canon(const or_tables *T, const double *ell, const double *U, double omega, int nc,
                    const int *kind, const int *lbin, const int *zbin, double *out) {
  double *mw = mass_weights(T);
#pragma omp parallel for schedule(dynamic, 4)
  for (int a = 0; a < nc; ++a)
    for (int b = 0; b <= a; ++b)
      out[(size_t)a * nc + b] = cov1h(T, ell, U, mw, omega, &kind[a], &lbin[3 * a], &zbin[3 * a],
                                      &kind[b], &lbin[3 * b], &zbin[3 * b]);
  free(mw);
}

/* --------------------------------------------------------------------
 * Super-sample covariance resolved along the line of sight.
 *
 * sigma_W^2(chi) is the variance of the linear density contrast averaged
 * over the survey's disk at distance chi: the delta_chi -> 0 limit of the
 * cylinder window of eq. Mask (App. B; the quantity is defined after eq.
 * CovPP22, Sec. 3.2.3).  In polar coordinates, d^2 eps = 2 pi eps d eps:
 *   sigma_W^2(chi) = 4 int d^2 eps / (2 pi)^2 [J1(x) / x]^2 P(eps, chi)
 *                  = (2 / pi) int eps^2 [J1(x) / x]^2 P(eps, chi) d ln eps,
 *   x = eps chi Theta.
 * Theta is the survey's angular radius, Omega = 2 pi (1 - cos Theta) (Sec.
 * 3.2.2, after eq. PSest).  Readings: the integral runs over the k table by
 * the trapezoid rule in ln eps on n_eps uniformly spaced nodes whose two end
 * nodes are the table's first and last k; P(eps, chi) is read like every
 * other table value; J1 is the C library's. */
#define OR_PI 3.14159265358979323846

void or_sigma_w2(const or_tables *T, double theta, int n_eps, double *out) {
  const double l0 = log(T->k[0]), l1 = log(T->k[T->n_k - 1]);
  const double h = (l1 - l0) / (n_eps - 1);
#pragma omp parallel for schedule(static)
  for (int n = 0; n < T->n_chi; ++n) {
    const double *Pn = T->P + (size_t)n * T->n_k;
    double s = 0.0;
    for (int j = 0; j < n_eps; ++j) {
      double eps = j == 0 ? T->k[0] : (j == n_eps - 1 ? T->k[T->n_k - 1] : exp(l0 + j * h));
      double x = eps * T->chi[n] * theta;
      double win = j1(x) / x;
      double w = (j == 0 || j == n_eps - 1) ? 0.5 * h : h;
      s += w * eps * eps * win * win * or_interp(T->k, Pn, T->n_k, eps);
    }
    out[n] = 2.0 / OR_PI * s;
  }
}

/* The super-sample term of eq. WLSSCflatskyLimber with this variance:
 *   C_ssc[a][b] = sum_n w_n sigma_W^2(chi_n) T_a(chi_n) R_a(chi_n) T_b(chi_n) R_b(chi_n),
 * T_a = chi^(2 - 2 p_a) prod_q W_{z_q} the projection function of eq.
 * nProjection and R_a the 3-D response of the row's ell-configuration at
 * chi_n (tabulated by or_spectra_table; zero above k_max). */
static double ssc_chi(const or_tables *T, const double *sw, const double *R, int ka, const int *za, int ca,
                      int kb, const int *zb, int cb) {
  double total = 0.0;
  for (int n = 0; n < T->n_chi; ++n) {
    double chi = T->chi[n];
    double ta = pow(chi, 2.0 - 2.0 * ka), tb = pow(chi, 2.0 - 2.0 * kb);
    for (int q = 0; q < ka; ++q) ta *= T->W[(size_t)za[q] * T->n_chi + n];
    for (int q = 0; q < kb; ++q) tb *= T->W[(size_t)zb[q] * T->n_chi + n];
    total += T->w_chi[n] * sw[n] * ta * R[(size_t)ca * T->n_chi + n] * tb * R[(size_t)cb * T->n_chi + n];
  }
  return total;
}

void or_ssc_chi_pairs(const or_tables *T, const double *sw, const double *R, const int *kind, const int *zbin,
                      const int *cfg, int64_t n_pairs, const int64_t *pairs, double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < n_pairs; ++q) {
    int64_t a = pairs[2 * q], b = pairs[2 * q + 1];
    out[q] = ssc_chi(T, sw, R, kind[a], &zbin[3 * a], cfg[a], kind[b], &zbin[3 * b], cfg[b]);
  }
}

/* --------------------------------------------------------------------
 * Signal-to-noise, eq. SNprim (Sec. 5): (S/N)^2 = D^T C^{-1} D, through the
 * Cholesky-Banachiewicz factorisation C = L L^T (row by row) and forward
 * substitution y = L^{-1} D, (S/N)^2 = y^T y.  or_chol_y returns y; both
 * return -1 if C is not positive definite. */
int or_chol_y(int n, const double *C, const double *D, double *y) {
  double *L = (double *)calloc((size_t)n * n, sizeof(double));
  if (!L) return -2;
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j <= i; ++j) {
      double s = 0.0;
#pragma omp parallel for reduction(+ : s) if (j > 512)
      for (int q = 0; q < j; ++q) s += L[(size_t)i * n + q] * L[(size_t)j * n + q];
      if (i == j) {
        double piv = C[(size_t)i * n + i] - s;
        if (!(piv > 0.0)) { free(L); return -1; }
        L[(size_t)i * n + i] = sqrt(piv);
      } else {
        L[(size_t)i * n + j] = (C[(size_t)i * n + j] - s) / L[(size_t)j * n + j];
      }
    }
  }
  for (int i = 0; i < n; ++i) {
    double s = D[i];
    for (int q = 0; q < i; ++q) s -= L[(size_t)i * n + q] * y[q];
    y[i] = s / L[(size_t)i * n + i];
  }
  free(L);
  return 0;
}

int or_snr2(int n, const double *C, const double *D, double *snr2) {
  double *y = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  if (!y) return -2;
  int rc = or_chol_y(n, C, D, y);
  double acc = 0.0;
  if (rc == 0)
    for (int i = 0; i < n; ++i) acc += y[i] * y[i];
  free(y);
  *snr2 = acc;
  return rc;
}

/* --------------------------------------------------------------------
 * Lattice counts (Sec. 3.2.2 mode lattice and App. B triangle count N_tri):
 * modes are integer vectors q != 0 of the survey lattice; a mode is in a bin
 * when T_lo <= |q|^2 < T_hi (thresholds in units of the fundamental mode).
 * The triangle count is the number of ordered pairs (q1, q2) with q1 in bin
 * 1, q2 in bin 2 and q1 + q2 in bin 3, counted one pair at a time. */
uint64_t or_lattice_modes(int64_t tlo, int64_t thi) {
  int64_t R = (int64_t)sqrt((double)thi) + 2;
  uint64_t c = 0;
  for (int64_t x = -R; x <= R; ++x)
    for (int64_t y = -R; y <= R; ++y) {
      int64_t s = x * x + y * y;
      if (s > 0 && s >= tlo && s < thi) ++c;
    }
  return c;
}

/* Sum over the modes of a bin of |q|^(2 p) (for averages of a power of
 * |q| over the bin's modes). */
double or_lattice_mode_moment(int64_t tlo, int64_t thi, int p) {
  int64_t R = (int64_t)sqrt((double)thi) + 2;
  double acc = 0.0;
  for (int64_t x = -R; x <= R; ++x)
    for (int64_t y = -R; y <= R; ++y) {
      int64_t s = x * x + y * y;
      if (s > 0 && s >= tlo && s < thi) acc += pow((double)s, p);
    }
  return acc;
}

/* Over the ordered pairs (q1, q2) of a triangle bin: the pair count (return
 * value) and, in *moment, the sum of (|q1|^2 |q2|^2 |q1 + q2|^2)^p. */
double or_lattice_triangle_moment(int64_t tlo1, int64_t thi1, int64_t tlo2, int64_t thi2, int64_t tlo3,
                                  int64_t thi3, int p, double *moment) {
  int64_t R1 = (int64_t)sqrt((double)thi1) + 2, R2 = (int64_t)sqrt((double)thi2) + 2;
  double count = 0.0, acc = 0.0;
#pragma omp parallel for reduction(+ : count, acc) collapse(2) schedule(dynamic, 4)
  for (int64_t x1 = -R1; x1 <= R1; ++x1)
    for (int64_t y1 = -R1; y1 <= R1; ++y1) {
      int64_t s1 = x1 * x1 + y1 * y1;
      if (!(s1 > 0 && s1 >= tlo1 && s1 < thi1)) continue;
      for (int64_t x2 = -R2; x2 <= R2; ++x2)
        for (int64_t y2 = -R2; y2 <= R2; ++y2) {
          int64_t s2 = x2 * x2 + y2 * y2;
          if (!(s2 > 0 && s2 >= tlo2 && s2 < thi2)) continue;
          int64_t x = x1 + x2, y = y1 + y2, s3 = x * x + y * y;
          if (!(s3 > 0 && s3 >= tlo3 && s3 < thi3)) continue;
          count += 1.0;
          acc += pow((double)s1 * (double)s2 * (double)s3, p);
        }
    }
  *moment = acc;
  return count;
}

uint64_t or_lattice_triangles(int64_t tlo1, int64_t thi1, int64_t tlo2, int64_t thi2,
                              int64_t tlo3, int64_t thi3) {
  /* list the modes of bins 1 and 2, then test every pair */
  int64_t R1 = (int64_t)sqrt((double)thi1) + 2, R2 = (int64_t)sqrt((double)thi2) + 2;
  size_t cap1 = (size_t)(2 * R1 + 1) * (2 * R1 + 1), cap2 = (size_t)(2 * R2 + 1) * (2 * R2 + 1);
  int32_t *q1 = (int32_t *)malloc(sizeof(int32_t) * 2 * cap1);
  int32_t *q2 = (int32_t *)malloc(sizeof(int32_t) * 2 * cap2);
  size_t n1 = 0, n2 = 0;
  for (int64_t x = -R1; x <= R1; ++x)
    for (int64_t y = -R1; y <= R1; ++y) {
      int64_t s = x * x + y * y;
      if (s > 0 && s >= tlo1 && s < thi1) { q1[2 * n1] = (int32_t)x; q1[2 * n1 + 1] = (int32_t)y; ++n1; }
    }
  for (int64_t x = -R2; x <= R2; ++x)
    for (int64_t y = -R2; y <= R2; ++y) {
      int64_t s = x * x + y * y;
      if (s > 0 && s >= tlo2 && s < thi2) { q2[2 * n2] = (int32_t)x; q2[2 * n2 + 1] = (int32_t)y; ++n2; }
    }
  uint64_t total = 0;
#pragma omp parallel for reduction(+ : total) schedule(dynamic, 64)
  for (size_t a = 0; a < n1; ++a) {
    uint64_t c = 0;
    for (size_t b = 0; b < n2; ++b) {
      int64_t x = (int64_t)q1[2 * a] + q2[2 * b], y = (int64_t)q1[2 * a + 1] + q2[2 * b + 1];
      int64_t s = x * x + y * y;
      if (s > 0 && s >= tlo3 && s < thi3) ++c;
    }
    total += c;
  }
  free(q1);
  free(q2);
  return total;
}
