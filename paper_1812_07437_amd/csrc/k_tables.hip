// Table staging, halo-model quadrature, Limber projection and the Gram factor.
//
// Rizzato et al. (2019), arXiv 1812.07437:
//   halo mass integrals I_mu^beta ............ eq. ImunuHalos (Sec. 4.1)
//   P_HM, B_HM ............................... eqs. PspHMtot2, B1halo, B2halos, B3halos (first line)
//   responses to a long mode ................. eqs. PowerHMResp, BispHMResp, RespP, RespB (Sec. 4.3)
//   Limber projection ........................ eq. nProjection (Sec. 3.1)
//   one-halo n-point function ................ eq. General1h (Sec. 4.2)
//   k_max cut of the line-of-sight integrand . Sec. 4.4
// Tables are read by linear interpolation of ln X in ln k between the
// bracketing nodes; d ln P / d ln k uses centred node differences (one-sided
// at the ends) interpolated linearly in ln k.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace wlc {

// ------------------------------------------------------------- validation
// flags[0]: a bad value; flags[1]: some ell/chi below k_max off the k table;
// flags[2]: theta > 0 and k_0 chi_max theta > 0.1 (the table starts above the
// scale of the survey window at the farthest node).
__global__ void k_validate(DevTables T, const double *centres, int n_ell, double theta, int *flags) {
  const int64_t nP = (int64_t)T.n_chi * T.n_k, nU = (int64_t)T.n_m_pts * T.n_k, nW = (int64_t)T.n_z * T.n_chi;
  const int64_t nM = T.n_m_pts, nC = T.n_chi, nK = T.n_k, nCov = (int64_t)n_ell * T.n_chi;
  const int64_t total = nP + nU + nW + nM + nC + nK + nCov;
  int bad = 0, range = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    int64_t q = i;
    if (q < nP) { double v = T.P[q]; bad |= !(isfinite(v) && v > 0.0); continue; }
    q -= nP;
    if (q < nU) { double v = T.u[q]; bad |= !(isfinite(v) && v > 0.0); continue; }
    q -= nU;
    if (q < nW) { double v = T.W[q]; bad |= !(isfinite(v) && v >= 0.0); continue; }
    q -= nW;
    if (q < nM) {
      bad |= !(isfinite(T.n_m[q]) && T.n_m[q] > 0.0);
      bad |= !(isfinite(T.m[q]) && T.m[q] > 0.0);
      bad |= !(isfinite(T.w_m[q]) && T.w_m[q] >= 0.0);
      if (T.b1) bad |= !isfinite(T.b1[q]);
      if (T.b2) bad |= !isfinite(T.b2[q]);
      continue;
    }
    q -= nM;
    if (q < nC) {
      bad |= !(isfinite(T.chi[q]) && T.chi[q] > 0.0 && isfinite(T.w_chi[q]) && T.w_chi[q] >= 0.0);
      if (q > 0) bad |= !(T.chi[q] > T.chi[q - 1]);
      continue;
    }
    q -= nC;
    if (q < nK) {
      bad |= !(isfinite(T.k[q]) && T.k[q] > 0.0);
      if (q > 0) bad |= !(T.k[q] > T.k[q - 1]);
      continue;
    }
    q -= nK;
    {
      const int b = (int)(q / T.n_chi), n = (int)(q % T.n_chi);
      const double kk = centres[b] / T.chi[n];
      if (kk <= T.k_max && !(kk >= T.k[0] && kk <= T.k[T.n_k - 1])) range = 1;
    }
  }
  if (bad) atomicOr(&flags[0], 1);
  if (range) atomicOr(&flags[1], 1);
  if (theta > 0.0 && blockIdx.x == 0 && threadIdx.x == 0 && !(T.k[0] * T.chi[T.n_chi - 1] * theta <= 0.1))
    atomicOr(&flags[2], 1);
}

void launch_validate(const DevTables &T, const double *centres, int n_ell, double theta, int *flags,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_validate, dim3(512), dim3(256), 0, s, T, centres, n_ell, theta, flags);
}

// ------------------------------------------------------------- staging
// U[b][n][m] = u(m, c_b / chi_n) (0 above k_max); Pk, Ne [b][n] = P and its
// logarithmic slope at c_b / chi_n.
__global__ void k_stage_u(DevTables T, const double *centres, int n_ell, double *U) {
  const int64_t total = (int64_t)n_ell * T.n_chi * T.n_m_pts;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int mi = (int)(i % T.n_m_pts);
    const int64_t bn = i / T.n_m_pts;
    const int n = (int)(bn % T.n_chi), b = (int)(bn / T.n_chi);
    const double kk = centres[b] / T.chi[n];
    double v = 0.0;
    int j; double t;
    if (kk <= T.k_max && bracket_lnk(T.k, T.n_k, kk, j, t)) {
      const double *row = T.u + (int64_t)mi * T.n_k;
      v = exp((1.0 - t) * log(row[j]) + t * log(row[j + 1]));
    }
    U[i] = v;
  }
}

__device__ __forceinline__ double node_slope(const double *kg, const double *row, int nk, int j) {
  const int a = j > 0 ? j - 1 : 0, b = j < nk - 1 ? j + 1 : nk - 1;
  return (log(row[b]) - log(row[a])) / (log(kg[b]) - log(kg[a]));
}

__global__ void k_stage_p(DevTables T, const double *centres, int n_ell, double *Pk, double *Ne) {
  const int64_t total = (int64_t)n_ell * T.n_chi;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int n = (int)(i % T.n_chi), b = (int)(i / T.n_chi);
    const double kk = centres[b] / T.chi[n];
    double pv = 0.0, nv = 0.0;
    int j; double t;
    if (kk <= T.k_max && bracket_lnk(T.k, T.n_k, kk, j, t)) {
      const double *row = T.P + (int64_t)n * T.n_k;
      pv = exp((1.0 - t) * log(row[j]) + t * log(row[j + 1]));
      nv = (1.0 - t) * node_slope(T.k, row, T.n_k, j) + t * node_slope(T.k, row, T.n_k, j + 1);
    }
    Pk[i] = pv;
    Ne[i] = nv;
  }
}

void launch_stage(const DevTables &T, const double *centres, int n_ell, double *U, double *Pk, double *Ne,
                  hipStream_t s) {
  const int64_t tu = (int64_t)n_ell * T.n_chi * T.n_m_pts;
  const int gu = (int)std::min<int64_t>((tu + 255) / 256, 65536);
  hipLaunchKernelGGL(k_stage_u, dim3(gu), dim3(256), 0, s, T, centres, n_ell, U);
  const int64_t tp = (int64_t)n_ell * T.n_chi;
  const int gp = (int)std::min<int64_t>((tp + 255) / 256, 65536);
  hipLaunchKernelGGL(k_stage_p, dim3(gp), dim3(256), 0, s, T, centres, n_ell, Pk, Ne);
}

// ------------------------------------------------------------- 3-D spectra
// One wavefront per (configuration, chi node): for each entry of the
// configuration's averaging list (its bin centres, or its sub-bins), lanes
// stride over the mass nodes, a wavefront reduction gives every mass
// integral, and lane 0 adds the entry's weighted X and R.
__device__ __forceinline__ double cosine3(double ki, double kj, double kl) {
  return (kl * kl - ki * ki - kj * kj) / (2.0 * ki * kj);
}

// X and R at one ell-triple (kind 3) or ell (kind 2) and chi node; valid on
// lane 0.  l0, l1, l2 index the staged ell values.
__device__ void spectrum_at(const DevTables &T, int kind, int l0, int l1, int l2, int n, const double *U,
                            const double *Pk, const double *Ne, const double *centres, int lane, double &X,
                            double &R) {
  const double chi = T.chi[n];
  double lmax = centres[l0];
  if (kind == 3) lmax = fmax(lmax, fmax(centres[l1], centres[l2]));
  X = R = 0.0;
  if (lmax / chi > T.k_max) return;
  const int nm = T.n_m_pts;
  const double inv_rho = 1.0 / T.rho;
  if (kind == 2) {
    const double *Ub = U + ((size_t)l0 * T.n_chi + n) * nm;
    double I11 = 0.0, I20 = 0.0, I21 = 0.0;
    for (int mi = lane; mi < nm; mi += WAVE) {
      const double x = T.m[mi] * inv_rho;
      const double wn = T.w_m[mi] * T.n_m[mi];
      const double b1 = T.b1 ? T.b1[mi] : 1.0;
      const double uu = Ub[mi];
      I11 += wn * b1 * x * uu;
      I20 += wn * x * x * uu * uu;
      I21 += wn * b1 * x * x * uu * uu;
    }
    I11 = wave_sum(I11); I20 = wave_sum(I20); I21 = wave_sum(I21);
    if (lane == 0) {
      const double P = Pk[(size_t)l0 * T.n_chi + n], ne = Ne[(size_t)l0 * T.n_chi + n];
      const double Rlin = 47.0 / 21.0 * P - ne * P / 3.0;
      X = I20 + I11 * I11 * P;
      R = I11 * I11 * Rlin + I21;
    }
    return;
  }
  const int lg[3] = {l0, l1, l2};
  const double *Ua = U + ((size_t)l0 * T.n_chi + n) * nm;
  const double *Ub = U + ((size_t)l1 * T.n_chi + n) * nm;
  const double *Uc = U + ((size_t)l2 * T.n_chi + n) * nm;
  double I11[3] = {0, 0, 0}, I21[3] = {0, 0, 0}, I22[3] = {0, 0, 0}, I30 = 0.0, I31 = 0.0;
  for (int mi = lane; mi < nm; mi += WAVE) {
    const double x = T.m[mi] * inv_rho;
    const double wn = T.w_m[mi] * T.n_m[mi];
    const double b1 = T.b1 ? T.b1[mi] : 1.0;
    const double b2 = T.b2 ? T.b2[mi] : 0.0;
    const double u[3] = {Ua[mi], Ub[mi], Uc[mi]};
    const double w1 = wn * x, w2 = wn * x * x, w3 = wn * x * x * x;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double ubc = u[(a + 1) % 3] * u[(a + 2) % 3];
      I11[a] += w1 * b1 * u[a];
      I21[a] += w2 * b1 * ubc;
      I22[a] += w2 * b2 * ubc;
    }
    const double u3 = u[0] * u[1] * u[2];
    I30 += w3 * u3;
    I31 += w3 * b1 * u3;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) { I11[a] = wave_sum(I11[a]); I21[a] = wave_sum(I21[a]); I22[a] = wave_sum(I22[a]); }
  I30 = wave_sum(I30);
  I31 = wave_sum(I31);
  if (lane == 0) {
    double P[3], ne[3], kv[3], Rlin[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      P[a] = Pk[(size_t)lg[a] * T.n_chi + n];
      ne[a] = Ne[(size_t)lg[a] * T.n_chi + n];
      kv[a] = centres[lg[a]] / chi;
      Rlin[a] = 47.0 / 21.0 * P[a] - ne[a] * P[a] / 3.0;
    }
    double two_halo = 0.0, resp_cyc = 0.0, Bpt = 0.0, Bg2 = 0.0, dil = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      two_halo += I11[a] * I21[a] * P[a];
      resp_cyc += I11[a] * I22[a] * P[a] + I11[a] * I21[a] * Rlin[a];
      const int i = a, j = (a + 1) % 3, l = (a + 2) % 3;
      const double mu = cosine3(kv[i], kv[j], kv[l]);
      const double F = 5.0 / 7.0 + 0.5 * mu * (kv[i] / kv[j] + kv[j] / kv[i]) + 2.0 / 7.0 * mu * mu;
      Bpt += 2.0 * F * P[i] * P[j];
      Bg2 += 2.0 * (mu * mu - 1.0) * P[i] * P[j];
      dil += 2.0 * F * P[i] * P[j] * (ne[i] + ne[j]);
    }
    const double I111 = I11[0] * I11[1] * I11[2];
    X = I30 + two_halo + I111 * Bpt;
    R = I111 * (433.0 / 126.0 * Bpt + 5.0 / 126.0 * Bg2 - dil / 3.0) + resp_cyc + I31;
  }
}

__global__ void k_spectra(DevTables T, const int32_t *cfgT, int n_cfg, SubList sl, const double *U,
                          const double *Pk, const double *Ne, const double *centres, double *X, double *R) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t item = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  if (item >= (int64_t)n_cfg * T.n_chi) return;
  const int c = (int)(item / T.n_chi), n = (int)(item % T.n_chi);
  const int kind = cfgT[4 * c];
  double xs = 0.0, rs = 0.0;
  for (int e = sl.off[c]; e < sl.off[c + 1]; ++e) {
    double xe, re;
    spectrum_at(T, kind, sl.leg[4 * e], sl.leg[4 * e + 1], sl.leg[4 * e + 2], n, U, Pk, Ne, centres, lane, xe,
                re);
    xs += sl.w[e] * xe;
    rs += sl.w[e] * re;
  }
  if (lane == 0) {
    X[item] = xs;
    R[item] = rs;
  }
}

void launch_spectra(const DevTables &T, const int32_t *cfgT, int n_cfg, const SubList &sl, const double *U,
                    const double *Pk, const double *Ne, const double *centres, double *X, double *R, hipStream_t s) {
  const int64_t items = (int64_t)n_cfg * T.n_chi;
  const int g = (int)((items + 3) / 4);
  hipLaunchKernelGGL(k_spectra, dim3(g), dim3(256), 0, s, T, cfgT, n_cfg, sl, U, Pk, Ne, centres, X, R);
}

// ------------------------------------------------------------- projection
// One wavefront per distinct row: lanes stride over chi, then reduce.
__global__ void k_project(DevTables T, const int32_t *rowR, const int32_t *cfgT, int64_t n_R, const double *X,
                          const double *R, double *dR, double *rR) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  if (row >= n_R) return;
  const int c = rowR[4 * row];
  const int p = cfgT[4 * c];
  int z[3] = {rowR[4 * row + 1], rowR[4 * row + 2], rowR[4 * row + 3]};
  double sd = 0.0, sr = 0.0;
  for (int n = lane; n < T.n_chi; n += WAVE) {
    const double chi = T.chi[n];
    double tw = T.w_chi[n] * pow(chi, 2.0 - 2.0 * p);
    for (int q = 0; q < p; ++q) tw *= T.W[(size_t)z[q] * T.n_chi + n];
    sd += tw * X[(size_t)c * T.n_chi + n];
    sr += tw * R[(size_t)c * T.n_chi + n];
  }
  sd = wave_sum(sd);
  sr = wave_sum(sr);
  if (lane == 0) { dR[row] = sd; rR[row] = sr; }
}

void launch_project(const DevTables &T, const int32_t *rowR, const int32_t *cfgT, int64_t n_R, const double *X,
                    const double *R, double *dR, double *rR, hipStream_t s) {
  const int g = (int)((n_R + 3) / 4);
  hipLaunchKernelGGL(k_project, dim3(g), dim3(256), 0, s, T, rowR, cfgT, n_R, X, R, dR, rR);
}

// Shot-noise power P^s_ij(l_b) = P_ij(l_b) + delta_ij sigma_eps^2 / n_i
// (eq. ShotNoise); the power-spectrum rows lead the distinct rows.
__global__ void k_ps(const double *dR, double *Ps, int n_ell, int n_z, double noise) {
  const int total = n_ell * n_z * n_z;
  const int npair = n_z * (n_z + 1) / 2;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < total; q += gridDim.x * blockDim.x) {
    const int j = q % n_z, i = (q / n_z) % n_z, b = q / (n_z * n_z);
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    const int rank = lo * n_z - lo * (lo - 1) / 2 + (hi - lo);
    Ps[q] = dR[(size_t)b * npair + rank] + (i == j ? noise : 0.0);
  }
}

void launch_ps(const double *dR, double *Ps, int n_ell, int n_z, double noise, hipStream_t s) {
  const int total = n_ell * n_z * n_z;
  hipLaunchKernelGGL(k_ps, dim3((total + 255) / 256), dim3(256), 0, s, dR, Ps, n_ell, n_z, noise);
}

// ------------------------------------------------------------- Gram factor
// The one-halo (p_a + p_b)-point function factorises over the legs of each
// row (eq. General1h), so
//   A[row][(n, m)] = sqrt(w_n) chi_n^-(2p-1) prod_i W_i(chi_n)        (= T[row][n])
//                  * sqrt(w_m n_m) (m/rho)^p prod_legs u(m, l/chi_n)   (= G[cfg][n][m])
// and (1/Omega) A A^T is the one-halo covariance of eqs. CovPPNG, Ins5P, Ins6P.
// With sw, one more column per chi node carries the super-sample term of eq.
// WLSSCflatskyLimber resolved along chi,
//   sum_n w_n sigma_W^2(chi_n) chi_n^(2-2p) prod W R_cfg(chi_n) (same for b),
// as G[cfg][n][n_m] = sqrt(Omega) chi_n sqrt(sigma_W^2(chi_n)) R[cfg][n].
__global__ void k_gfactor(DevTables T, const int32_t *cfgT, int n_cfg, SubList sl, const double *U,
                          const double *R, const double *sw, double sq_omega, int n_mg, double *G, double *Gmax) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t item = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  if (item >= (int64_t)n_cfg * T.n_chi) return;
  const int c = (int)(item / T.n_chi), n = (int)(item % T.n_chi);
  const int kind = cfgT[4 * c];
  const int nm = T.n_m_pts;
  const double inv_rho = 1.0 / T.rho;
  const int e0 = sl.off[c], e1 = sl.off[c + 1];
  double mx = 0.0;
  double *Gout = G + (size_t)item * n_mg;
  for (int mi = lane; mi < nm; mi += WAVE) {
    const double x = T.m[mi] * inv_rho;
    double g = 0.0;
    // the average over the configuration's entries (one entry of weight 1
    // at the bin centres)
    for (int e = e0; e < e1; ++e) {
      const double *U0 = U + ((size_t)sl.leg[4 * e] * T.n_chi + n) * nm;
      const double *U1 = kind == 3 ? U + ((size_t)sl.leg[4 * e + 1] * T.n_chi + n) * nm : U0;
      double ge = sqrt(T.w_m[mi] * T.n_m[mi]) * x * x * U0[mi] * U1[mi];
      if (kind == 3) ge *= x * U[((size_t)sl.leg[4 * e + 2] * T.n_chi + n) * nm + mi];
      g += sl.w[e] * ge;
    }
    Gout[mi] = g;
    mx = fmax(mx, fabs(g));
  }
  if (sw && lane == 0) {
    const double g = sq_omega * T.chi[n] * sqrt(sw[n]) * R[item];
    Gout[nm] = g;
    mx = fmax(mx, fabs(g));
  }
  mx = wave_max(mx);
  if (lane == 0) Gmax[item] = mx;
}

void launch_gfactor(const DevTables &T, const int32_t *cfgT, int n_cfg, const SubList &sl, const double *U,
                    const double *R, const double *sw, double sq_omega, int n_mg, double *G, double *Gmax,
                    hipStream_t s) {
  const int64_t items = (int64_t)n_cfg * T.n_chi;
  hipLaunchKernelGGL(k_gfactor, dim3((int)((items + 3) / 4)), dim3(256), 0, s, T, cfgT, n_cfg, sl, U, R, sw,
                     sq_omega, n_mg, G, Gmax);
}

// Per distinct row: T[n] and the row exponent s = -e with
// max_k |A[row][k]| = f 2^e, f in [0.5, 1); Ts[row][n] = 2^s T[n].
__global__ void k_tfactor(DevTables T, const int32_t *rowR, const int32_t *cfgT, int64_t n_R, const double *Gmax,
                          double *Ts, int32_t *sexp) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  if (row >= n_R) return;
  const int c = rowR[4 * row];
  const int p = cfgT[4 * c];
  const int z[3] = {rowR[4 * row + 1], rowR[4 * row + 2], rowR[4 * row + 3]};
  double mx = 0.0;
  for (int n = lane; n < T.n_chi; n += WAVE) {
    const double chi = T.chi[n];
    double t = sqrt(T.w_chi[n]) * pow(chi, 1.0 - 2.0 * p);
    for (int q = 0; q < p; ++q) t *= T.W[(size_t)z[q] * T.n_chi + n];
    mx = fmax(mx, fabs(t) * Gmax[(size_t)c * T.n_chi + n]);
  }
  mx = wave_max(mx);
  const int s = -exp2_of(mx);
  for (int n = lane; n < T.n_chi; n += WAVE) {
    const double chi = T.chi[n];
    double t = sqrt(T.w_chi[n]) * pow(chi, 1.0 - 2.0 * p);
    for (int q = 0; q < p; ++q) t *= T.W[(size_t)z[q] * T.n_chi + n];
    Ts[(size_t)row * T.n_chi + n] = ldexp(t, s);
  }
  if (lane == 0) sexp[row] = s;
}

void launch_tfactor(const DevTables &T, const int32_t *rowR, const int32_t *cfgT, int64_t n_R, const double *Gmax,
                    double *Ts, int32_t *sexp, hipStream_t s) {
  hipLaunchKernelGGL(k_tfactor, dim3((int)((n_R + 3) / 4)), dim3(256), 0, s, T, rowR, cfgT, n_R, Gmax, Ts, sexp);
}

// ------------------------------------------------------------- two-leg factors
// The projected one-halo trispectrum that enters the P.T term of eq. CovBB
// at the two remaining legs of each of two triangles factorises like the
// one-halo covariance: for a two-leg configuration (ell-bins p <= q) and
// bins (j at p, k at q),
//   T[(pq, jk)][(p'q', j'k')] = sum_n Ts2[(pq, jk)][n] Ts2[(p'q', j'k')][n]
//                               * sum_m G2[pq][n][m] G2[p'q'][n][m],
//   Ts2 = sqrt(w_n) chi_n^-3 W_j(chi_n) W_k(chi_n),
//   G2  = sqrt(w_m n_m) (m/rho)^2 u(m, l_p/chi_n) u(m, l_q/chi_n)
// (eq. nProjection with n = 4, I_4^0 of eq. ImunuHalos).  Configurations:
// p = q first (index p), then p < q in lexicographic order; rows: pairs
// j <= k for p = q, all n_z^2 ordered pairs (j, k) for p < q.
__global__ void k_g2factor(DevTables T, int n_ell, const double *U, double *G2) {
  const int n2 = n_ell + n_ell * (n_ell - 1) / 2;
  const int64_t total = (int64_t)n2 * T.n_chi * T.n_m_pts;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int mi = (int)(i % T.n_m_pts);
    const int64_t cn = i / T.n_m_pts;
    const int n = (int)(cn % T.n_chi), c = (int)(cn / T.n_chi);
    int p, q;
    if (c < n_ell) {
      p = q = c;
    } else {
      int r = c - n_ell;
      for (p = 0; r >= n_ell - 1 - p; ++p) r -= n_ell - 1 - p;
      q = p + 1 + r;
    }
    const double x = T.m[mi] / T.rho;
    G2[i] = sqrt(T.w_m[mi] * T.n_m[mi]) * x * x * U[((size_t)p * T.n_chi + n) * T.n_m_pts + mi] *
            U[((size_t)q * T.n_chi + n) * T.n_m_pts + mi];
  }
}

__global__ void k_t2factor(DevTables T, int n_ell, int64_t rows, double *Ts2) {
  const int nz = T.n_z, sp = nz * (nz + 1) / 2;
  const int64_t total = rows * T.n_chi;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int n = (int)(i % T.n_chi);
    const int64_t row = i / T.n_chi;
    int j, k;
    if (row < (int64_t)n_ell * sp) {
      int w = (int)(row % sp);
      for (j = 0; w >= nz - j; ++j) w -= nz - j;
      k = j + w;
    } else {
      const int w = (int)((row - (int64_t)n_ell * sp) % (nz * nz));
      j = w / nz;
      k = w % nz;
    }
    const double chi = T.chi[n];
    Ts2[i] = sqrt(T.w_chi[n]) / (chi * chi * chi) * T.W[(size_t)j * T.n_chi + n] * T.W[(size_t)k * T.n_chi + n];
  }
}

void launch_twoleg(const DevTables &T, int n_ell, const double *U, double *G2, double *Ts2, hipStream_t s) {
  const int n2 = n_ell + n_ell * (n_ell - 1) / 2;
  const int nz = T.n_z;
  const int64_t rows = (int64_t)n_ell * (nz * (nz + 1) / 2) + (int64_t)(n2 - n_ell) * nz * nz;
  const int64_t tg = (int64_t)n2 * T.n_chi * T.n_m_pts, tt = rows * T.n_chi;
  hipLaunchKernelGGL(k_g2factor, dim3((unsigned)std::min<int64_t>((tg + 255) / 256, 65536)), dim3(256), 0, s, T,
                     n_ell, U, G2);
  hipLaunchKernelGGL(k_t2factor, dim3((unsigned)std::min<int64_t>((tt + 255) / 256, 65536)), dim3(256), 0, s, T,
                     n_ell, rows, Ts2);
}

// ------------------------------------------------------------- A build
// A[row][k], k = n * n_m + m; rows >= n_R and k >= n_chi * n_m are zero.  A
// row of A is T_row(chi_n) G_cfg(chi_n, M_m).  The write traffic is the
// kernel's whole HBM cost.
//
// Row-major f64 / f32 ([r_pad][lda]): consecutive rows mostly share their
// configuration, so each block holds 8 consecutive k of G_cfg per thread in
// registers and writes them, times T_row, for AB_ROWS consecutive rows,
// reloading G only where the configuration changes.  With arow, row r of A
// is the distinct row arow[r] (zero where it is negative); every k is
// written.
constexpr int AB_ROWS = 16;

template <int FMT>
__global__ __launch_bounds__(256) void k_abuild(const int32_t *__restrict__ rowR, const double *__restrict__ Ts,
                                               const double *__restrict__ G, int64_t n_R, int n_chi, int n_m,
                                               int64_t k_pad, int64_t lda, void *A0, void *A1,
                                               const int32_t *__restrict__ arow) {
  const int64_t k0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 8;
  if (k0 >= k_pad) return;
  const int64_t k_len = (int64_t)n_chi * n_m;
  int nq[8];
  {
    int n = (int)(k0 / n_m), m = (int)(k0 % n_m);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      nq[q] = k0 + q < k_len ? n : -1;
      if (++m == n_m) { m = 0; ++n; }
    }
  }
  double g[8];
  int cc = -1;
  const int64_t r0 = (int64_t)blockIdx.y * AB_ROWS;
  for (int rr = 0; rr < AB_ROWS; ++rr) {
    const int64_t row = r0 + rr;
    const int64_t e = arow ? (int64_t)arow[row] : (row < n_R ? row : -1);  // its distinct row
    double v[8];
    if (e >= 0) {
      const int c = rowR[4 * e];
      if (c != cc) {
        cc = c;
        const double *Gc = G + (size_t)c * k_len + k0;
        if (k0 + 8 <= k_len && (k_len & 1) == 0) {  // 16-byte aligned pairs
#pragma unroll
          for (int q = 0; q < 8; q += 2) {
            const double2 t = *(const double2 *)(Gc + q);
            g[q] = t.x;
            g[q + 1] = t.y;
          }
        } else {
#pragma unroll
          for (int q = 0; q < 8; ++q) g[q] = nq[q] >= 0 ? Gc[q] : 0.0;
        }
      }
      const double *Tr = Ts + (size_t)e * n_chi;
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = nq[q] >= 0 ? Tr[nq[q]] * g[q] : 0.0;
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = 0.0;
    }
    const size_t off = (size_t)row * lda + k0;
    if constexpr (FMT == 0) {
      double *o = (double *)A0 + off;
#pragma unroll
      for (int q = 0; q < 8; q += 2) *(double2 *)(o + q) = make_double2(v[q], v[q + 1]);
    } else if constexpr (FMT == 3) {
      float *o = (float *)A0 + off;
      *(float4 *)o = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
      *(float4 *)(o + 4) = make_float4((float)v[4], (float)v[5], (float)v[6], (float)v[7]);
    }
  }
}

// k-blocked bf16 (fmt 1: hi only; fmt 2: hi and lo; see launch_abuild): a 256-thread
// block covers 64 rows and AB_KB consecutive 32-column k-blocks.  Each
// wavefront takes every fourth k-block of the block; in one, lane l converts
// 8 consecutive k (chunk l % 4) of the rows l / 4 + 16 j, j < AB_RW, so that
// each of its stores writes 16 whole rows of the k-block, 1 KB contiguous
// (non-temporal: at large10 1.55 -> 1.3 ms with hi, 2.2 -> 1.6 ms with lo).
// Rows of one configuration are consecutive (in the A-row order of the bf16
// products, those of one lowest redshift bin), so a lane's 8 values of G
// serve all its rows of one configuration, and T is taken once per row and
// chi node.  When N_M is a multiple of 8 a chunk lies in one chi
// node, and T of the workgroup's rows and G of its configurations (at most
// AB_GC of them) are staged in LDS with coalesced loads; otherwise the values
// are taken one by one from global memory.
constexpr int AB_KB = 32;
constexpr int AB_RW = 4;
// chi nodes of T a workgroup stages in LDS: its AB_KB k-blocks span
// AB_KB 32 / N_M + 1 nodes at most (33 for N_M >= 32); more go to global memory
constexpr int AB_TN = 40;
// configurations whose G a workgroup stages in LDS, pass by pass (a pass is
// the four k-blocks the wavefronts convert together): in the A-row order at
// n_z = 10, 64 rows of one lowest bin z span at most eight configurations
// for z <= 6 (10 or more rows each); wider spans take the global path
// (measured at large10: 1.58 ms with 6 or 8, 1.63 with 3, 1.82 with 12)
constexpr int AB_GC = 8;

// Two floats to packed bf16, rounded to nearest even (v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint32_t pack_bf16_rne(float a, float b) {
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2{a, b}), bf16x2));
}

// With panel_f (the per-tile precision of WLC_BF16_AUTO: per 256-row panel
// the largest one-halo share, then the largest of all), the lo half of a
// panel is written only if some tile of its row or column can take the split
// product, F_P F_max > lim; the product never reads it otherwise.
template <int FMT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FMT == 1 ? 5 : 4))) void k_abuild_blk(const int32_t *__restrict__ rowR, const double *__restrict__ Ts,
                                                   const double *__restrict__ G, int64_t n_R, int n_chi, int n_m,
                                                   int64_t k_pad, int64_t r_pad, uint16_t *__restrict__ A0,
                                                   uint16_t *__restrict__ A1, const double *__restrict__ panel_f,
                                                   double lim, const int32_t *__restrict__ arow,
                                                   const int32_t *__restrict__ ext) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int chunk = lane & 3;
  const int64_t row0 = (int64_t)blockIdx.y * 64 + (lane >> 2);  // A-rows row0 + 16 j
  // a workgroup's 64 rows lie in one 256-row panel; with ext the panel's rows
  // are zero from k-block ext[panel] on, and no product reads them there
  const int panel = blockIdx.y / 4;
  const int n_kb =
      (int)min((int64_t)AB_KB, (ext ? (int64_t)ext[panel] : k_pad / GRAM_KB) - (int64_t)blockIdx.x * AB_KB);
  if (n_kb <= 0) return;  // workgroup-uniform, before any barrier
  const bool need_lo = FMT == 2 && (panel_f == nullptr || panel_f[panel] * panel_f[r_pad / 256] > lim);
  const int64_t k_len = (int64_t)n_chi * n_m;
  const bool whole = (n_m & 7) == 0;  // a chunk of 8 k lies in one chi node
  // the distinct row of an A-row (-1 for padding)
  auto distinct = [&](int64_t r) -> int { return arow ? arow[r] : (r < n_R ? (int)r : -1); };
  int cfg[AB_RW];
  const double *Tr[AB_RW];
#pragma unroll
  for (int j = 0; j < AB_RW; ++j) {
    const int e = distinct(row0 + 16 * j);
    cfg[j] = e >= 0 ? rowR[4 * e] : -1;
    Tr[j] = Ts + (size_t)(e >= 0 ? e : 0) * n_chi;
  }
  // T of the workgroup's 64 rows at the chi nodes of its k range, staged in
  // LDS with coalesced loads (a lane would otherwise gather T of its rows
  // from 16 rows n_chi apart at every node change)
  __shared__ double Tl[64][AB_TN + 1];
  __shared__ int c_rng[2];  // smallest and largest configuration of the workgroup's rows
  const int64_t kbeg = (int64_t)blockIdx.x * AB_KB * GRAM_KB;
  const int n_lo = kbeg < k_len ? (int)(kbeg / n_m) : 0;
  const int n_hi = kbeg < k_len ? (int)((min(kbeg + (int64_t)n_kb * GRAM_KB, k_len) - 1) / n_m) : 0;
  const int nodes = n_hi - n_lo + 1;
  const bool staged = whole && kbeg < k_len && nodes <= AB_TN;  // workgroup-uniform
  if (staged) {
    if (threadIdx.x == 0) c_rng[0] = 0x7FFFFFFF, c_rng[1] = -1;
    __syncthreads();
    if (threadIdx.x < 64) {
      const int e = distinct((int64_t)blockIdx.y * 64 + threadIdx.x);
      if (e >= 0) {
        atomicMin(&c_rng[0], rowR[4 * e]);
        atomicMax(&c_rng[1], rowR[4 * e]);
      }
    }
    for (int idx = threadIdx.x; idx < 64 * nodes; idx += 256) {
      const int r = idx / nodes, q = idx % nodes;
      const int e = distinct((int64_t)blockIdx.y * 64 + r);
      Tl[r][q] = e >= 0 ? Ts[(int64_t)e * n_chi + n_lo + q] : 0.0;
    }
    __syncthreads();
  }
  // G of the workgroup's configurations for the four k-blocks of a pass, in
  // two alternating buffers: the barrier after filling one for pass p also
  // ends every wavefront's reads of pass p - 1, whose buffer pass p + 1 fills
  __shared__ double Gl[2][AB_GC][4 * GRAM_KB];
  const int c_first = staged ? c_rng[0] : 0, c_last = staged ? c_rng[1] : -1;
  const bool gstaged = staged && c_last >= c_first && c_last - c_first < AB_GC;  // workgroup-uniform
  int node[AB_RW];
  double tn[AB_RW];
#pragma unroll
  for (int j = 0; j < AB_RW; ++j) node[j] = -1, tn[j] = 0.0;
  for (int pass = 0; pass < (n_kb + 3) / 4; ++pass) {
    const int q = 4 * pass + wave;
    if (gstaged) {
      const int64_t kp = kbeg + (int64_t)pass * 4 * GRAM_KB;
      for (int idx = threadIdx.x; idx < AB_GC * 2 * GRAM_KB; idx += 256) {
        const int ci = idx / (2 * GRAM_KB), e = 2 * (idx % (2 * GRAM_KB));
        const int64_t k = kp + e;  // even, and k_len is a multiple of 8: k + 1 < k_len with k
        double2 v = make_double2(0.0, 0.0);
        if (ci <= c_last - c_first && k < k_len) v = *(const double2 *)(G + (size_t)(c_first + ci) * k_len + k);
        *(double2 *)&Gl[pass & 1][ci][e] = v;
      }
      __syncthreads();
    }
    if (q >= n_kb) continue;  // past the panel's k-blocks (later passes' barriers still to come: no break)
    const int64_t kblk = (int64_t)blockIdx.x * AB_KB + q;
    const int64_t k0 = kblk * GRAM_KB + 8 * chunk;
    const int n = k0 < k_len ? (int)(k0 / n_m) : 0;
    double g[8];
    int gc = -1;
#pragma unroll
    for (int j = 0; j < AB_RW; ++j) {
      const int64_t row = row0 + 16 * j;
      float x[8];
      if (whole && cfg[j] >= 0 && k0 < k_len) {
        if (cfg[j] != gc) {
          if (gstaged) {
            const double *Gs = &Gl[pass & 1][cfg[j] - c_first][wave * GRAM_KB + 8 * chunk];
#pragma unroll
            for (int e = 0; e < 8; ++e) g[e] = Gs[e];
          } else {
            const double *Gc = G + (size_t)cfg[j] * k_len + k0;
#pragma unroll
            for (int e = 0; e < 8; e += 2) {
              const double2 t = *(const double2 *)(Gc + e);
              g[e] = t.x;
              g[e + 1] = t.y;
            }
          }
          gc = cfg[j];
        }
        if (node[j] != n) {
          node[j] = n;
          tn[j] = staged ? Tl[(lane >> 2) + 16 * j][n - n_lo] : Tr[j][n];
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = (float)(tn[j] * g[e]);
      } else {
        // one by one, stepping across the chi node edges (k0 = n N_M + m)
        const double *Gc = G + (size_t)(cfg[j] >= 0 ? cfg[j] : 0) * k_len;
        int nn = n, mm = (int)(k0 - (int64_t)n * n_m);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int64_t k = k0 + e;
          x[e] = cfg[j] >= 0 && k < k_len ? (float)(Tr[j][nn] * Gc[k]) : 0.0f;
          if (++mm == n_m) mm = 0, ++nn;
        }
      }
      uint32_t hi[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) hi[e] = pack_bf16_rne(x[2 * e], x[2 * e + 1]);
      const size_t off = ((size_t)kblk * r_pad + row) * GRAM_KB + 8 * chunk;
      __builtin_nontemporal_store(u32x4{hi[0], hi[1], hi[2], hi[3]}, (u32x4 *)(A0 + off));
      if (need_lo) {
        uint32_t lo[4];
#pragma unroll
        for (int e = 0; e < 4; ++e)
          lo[e] = pack_bf16_rne(x[2 * e] - __uint_as_float(hi[e] << 16),
                                x[2 * e + 1] - __uint_as_float(hi[e] & 0xFFFF0000u));
        __builtin_nontemporal_store(u32x4{lo[0], lo[1], lo[2], lo[3]}, (u32x4 *)(A1 + off));
      }
    }
  }
}

// One workgroup per 256-row panel of A-rows: each thread scans its row's T
// back from the last chi node to the last nonzero one; the panel keeps the
// largest count of k-blocks (the k of node n are n N_M .. n N_M + N_M - 1).
__global__ __launch_bounds__(256) void k_panel_ext(const double *__restrict__ Ts, const int32_t *__restrict__ arow,
                                                  int n_chi, int n_mg, int64_t k_pad, int32_t *__restrict__ ext) {
  __shared__ int32_t best;
  if (threadIdx.x == 0) best = 0;
  __syncthreads();
  const int e = arow[(int64_t)blockIdx.x * 256 + threadIdx.x];
  int last = -1;
  if (e >= 0) {
    const double *t = Ts + (size_t)e * n_chi;
    for (int n = n_chi - 1; n >= 0; --n)
      if (t[n] != 0.0) {
        last = n;
        break;
      }
  }
  const int64_t kb = min(((int64_t)(last + 1) * n_mg + GRAM_KB - 1) / GRAM_KB, k_pad / GRAM_KB);
  if (kb > 0) atomicMax(&best, (int32_t)kb);
  __syncthreads();
  if (threadIdx.x == 0) ext[blockIdx.x] = best;
}

void launch_panel_ext(const double *Ts, const int32_t *arow, int64_t r_pad, int n_chi, int n_mg, int64_t k_pad,
                      int32_t *ext, hipStream_t s) {
  hipLaunchKernelGGL(k_panel_ext, dim3((unsigned)(r_pad / 256)), dim3(256), 0, s, Ts, arow, n_chi, n_mg, k_pad, ext);
}

void launch_abuild(int fmt, const int32_t *rowR, const double *Ts, const double *G, int64_t n_R, int64_t r_pad,
                   int n_chi, int n_m, int64_t k_pad, int64_t lda, void *A0, void *A1, hipStream_t s,
                   const double *panel_f, double lim, const int32_t *arow, const int32_t *ext) {
  if (fmt == 1 || fmt == 2) {
    // r_pad is a multiple of 64 and k_pad of GRAM_KB (rows are padded to the
    // Gram tile, columns to 64)
    const dim3 grid((unsigned)((k_pad / GRAM_KB + AB_KB - 1) / AB_KB), (unsigned)(r_pad / 64));
    if (fmt == 1)
      hipLaunchKernelGGL(k_abuild_blk<1>, grid, dim3(256), 0, s, rowR, Ts, G, n_R, n_chi, n_m, k_pad, r_pad,
                         (uint16_t *)A0, (uint16_t *)A1, nullptr, 0.0, arow, ext);
    else
      hipLaunchKernelGGL(k_abuild_blk<2>, grid, dim3(256), 0, s, rowR, Ts, G, n_R, n_chi, n_m, k_pad, r_pad,
                         (uint16_t *)A0, (uint16_t *)A1, panel_f, lim, arow, ext);
    return;
  }
  // r_pad is a multiple of AB_ROWS (rows are padded to the Gram tile)
  const dim3 grid((unsigned)((k_pad / 8 + 255) / 256), (unsigned)((r_pad + AB_ROWS - 1) / AB_ROWS));
  if (fmt == 0)
    hipLaunchKernelGGL(k_abuild<0>, grid, dim3(256), 0, s, rowR, Ts, G, n_R, n_chi, n_m, k_pad, lda, A0, A1, arow);
  else
    hipLaunchKernelGGL(k_abuild<3>, grid, dim3(256), 0, s, rowR, Ts, G, n_R, n_chi, n_m, k_pad, lda, A0, A1, arow);
}

}  // namespace wlc
