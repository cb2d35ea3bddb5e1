// Assembly of the joint P+B covariance (Rizzato et al. 2019, eq. eq:SN2):
//   C = C_Gauss + E (G / Omega) E^T + sigma_b^2 r r^T,
// with E the map from data-vector rows to distinct rows, G the Gram product of
// the one-halo factor, and the Gaussian blocks
//   P-P: delta_{l l'} / N(l) [P^s_ii' P^s_jj' + P^s_ij' P^s_ji']       (eq. CovPPG)
//   B-B: Omega / N_tri sum over the 6 maps sigma of primed onto unprimed legs of
//        prod_a P^s_{i_a i'_sigma(a)}(l_a) delta_K(l_a, l'_sigma(a))     (App. B, Gauss term)
//   P-B: none                                                          (eq. CovPBsynt)
// The result is written scaled, C~[a][b] = 2^(t_a + t_b) C[a][b], with t
// chosen so that every C~[a][a] lies in [1, 4).  Each unordered pair (a, b)
// is evaluated once and written to both halves, so C~ is exactly symmetric.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace wlc {

__device__ __forceinline__ double gauss_entry(const AsmArgs &A, const int32_t *ra, const int32_t *rb) {
  if (ra[0] != rb[0]) return 0.0;  // different ell-configuration
  const int nz = A.n_z;
  const double *Ps = A.Ps;
  const int kind = A.cfgT[4 * ra[0]];
  if (kind == 2) {
    const int b = ra[5];
    const double *P = Ps + (size_t)b * nz * nz;
    return (P[ra[2] * nz + rb[2]] * P[ra[3] * nz + rb[3]] + P[ra[2] * nz + rb[3]] * P[ra[3] * nz + rb[2]]) /
           A.nmodes[b];
  }
  const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  double s = 0.0;
#pragma unroll
  for (int p = 0; p < 6; ++p) {
    double term = 1.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int sa = perm[p][a];
      if (ra[5 + a] != rb[5 + sa]) { term = 0.0; break; }
      term *= Ps[((size_t)ra[5 + a] * nz + ra[2 + a]) * nz + rb[2 + sa]];
    }
    s += term;
  }
  return A.omega / A.ntri[ra[0] - A.n_ell] * s;
}

// ---- in-survey terms beyond the one-halo functions (eqs. CovBB, Covpb)
// Index of the distinct row of a bin multiset: pairs i <= j and triples
// i <= j <= k are ranked in the plan's order (first index slowest).
__device__ __forceinline__ int pair_rank(int i, int j, int nz) {
  if (i > j) { const int t = i; i = j; j = t; }
  return i * nz - i * (i - 1) / 2 + (j - i);
}

__device__ __forceinline__ int trip_rank(int a, int b, int c, int nz) {
  // sort three values
  if (a > b) { const int t = a; a = b; b = t; }
  if (b > c) { const int t = b; b = c; c = t; }
  if (a > b) { const int t = a; a = b; b = t; }
  int r = 0;
  for (int x = 0; x < a; ++x) r += (nz - x) * (nz - x + 1) / 2;
  for (int y = a; y < b; ++y) r += nz - y;
  return r + (c - b);
}

// Row of the two-leg trispectrum for legs p <= q (ell-bins) carrying bins
// (j on p, k on q).
__device__ __forceinline__ int64_t twoleg_row(int p, int q, int j, int k, int nl, int nz) {
  const int sp = nz * (nz + 1) / 2;
  if (p == q) return (int64_t)p * sp + pair_rank(j, k, nz);
  const int r = p * (nl - 1) - p * (p - 1) / 2 + (q - p - 1);
  return (int64_t)nl * sp + (int64_t)r * nz * nz + j * nz + k;
}

__device__ __forceinline__ double ngins_entry(const AsmArgs &A, const int32_t *ra, const int32_t *rb) {
  const int nz = A.n_z, nl = A.n_ell;
  const int kind_a = A.cfgT[4 * ra[0]], kind_b = A.cfgT[4 * rb[0]];
  if (kind_a == 2 && kind_b == 2) return 0.0;
  const int sp = nz * (nz + 1) / 2, st = nz * (nz + 1) * (nz + 2) / 6;
  const int64_t np = (int64_t)nl * sp;  // first distinct bispectrum row
  const double *Ps = A.Ps;
  auto ps = [&](int b, int i, int j) { return Ps[((size_t)b * nz + i) * nz + j]; };
  auto bval = [&](int cfg, int z0, int z1, int z2) {
    return A.dR[np + (int64_t)(cfg - nl) * st + trip_rank(z0, z1, z2, nz)];
  };
  if (kind_a == 2 || kind_b == 2) {
    const int32_t *rp = kind_a == 2 ? ra : rb, *rt = kind_a == 2 ? rb : ra;
    const int l = rp[5], i = rp[2], j = rp[3];
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (rt[5 + b] != l) continue;
      int zi[3] = {rt[2], rt[3], rt[4]}, zj[3] = {rt[2], rt[3], rt[4]};
      zi[b] = i;
      zj[b] = j;
      s += (ps(l, rt[2 + b], j) * bval(rt[0], zi[0], zi[1], zi[2]) +
            ps(l, i, rt[2 + b]) * bval(rt[0], zj[0], zj[1], zj[2])) / A.nmodes[l];
    }
    return s;
  }
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const int l = ra[5 + a];
      if (l != rb[5 + b]) continue;
      int z1[3] = {ra[2], ra[3], ra[4]}, z2[3] = {rb[2], rb[3], rb[4]};
      z1[a] = rb[2 + b];
      z2[b] = ra[2 + a];
      const double bb = bval(ra[0], z1[0], z1[1], z1[2]) * bval(rb[0], z2[0], z2[1], z2[2]);
      // the two other legs of each row, in leg order (ell-bins non-decreasing)
      const int ax = a == 0 ? 1 : 0, ay = a == 2 ? 1 : 2, bx = b == 0 ? 1 : 0, by = b == 2 ? 1 : 2;
      const int64_t ta = twoleg_row(ra[5 + ax], ra[5 + ay], ra[2 + ax], ra[2 + ay], nl, nz);
      const int64_t tb = twoleg_row(rb[5 + bx], rb[5 + by], rb[2 + bx], rb[2 + by], nl, nz);
      const double t4 = ta >= tb ? A.T2[ta * A.ld_t2 + tb] : A.T2[tb * A.ld_t2 + ta];
      s += (bb + ps(l, ra[2 + a], rb[2 + b]) * t4) / A.nmodes[l];
    }
  return s;
}

// G has been mirrored to exact symmetry, so it is read along rows: for the
// 64 consecutive data rows b of a wavefront the distinct rows e(b) are
// clustered, and the reads touch few cache lines.
__device__ __forceinline__ double gram_at(const AsmArgs &A, int64_t ea, int64_t eb) {
  return A.gm_f32 ? (double)((const float *)A.Gm)[ea * A.ld_g + eb] : ((const double *)A.Gm)[ea * A.ld_g + eb];
}

// Diagonal first: row exponents t_a, and the expanded d, r.
__global__ void k_rowexp(AsmArgs A, int32_t *row_exp2, double *d, double *r) {
  const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (a >= A.n) return;
  const int32_t *ra = A.rowO + 8 * a;
  const int64_t e = ra[1];
  const double g = gram_at(A, e, e);
  const double rr = A.rR[e];
  double c = ldexp(g, -2 * A.sexp[e]) * A.inv_omega + gauss_entry(A, ra, ra) + A.sigma_b2 * rr * rr;
  if (A.ngins) c += ngins_entry(A, ra, ra);
  int t = 0;
  if (c > 0.0 && isfinite(c)) {
    const int E = exp2_of(c);
    const int q = E - 1;
    t = -(q >= 0 ? q / 2 : -((1 - q) / 2));  // -floor((E - 1) / 2)
  }
  row_exp2[a] = t;
  d[a] = A.dR[e];
  r[a] = rr;
}

void launch_rowexp(const AsmArgs &a, int32_t *row_exp2, double *d, double *r, hipStream_t s) {
  hipLaunchKernelGGL(k_rowexp, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a, row_exp2, d, r);
}

// ---- per-tile precision of the bf16 Gram (WLC_BF16_AUTO)
// The one-halo diagonal of distinct row e in FP64 from its factors,
//   G_ee = sum_n Ts[e][n]^2 S[c(e)][n],  S[c][n] = sum_m G[c][n][m]^2
// (the row of A is Ts[e][n] G[c][n][m] over k = (n, m)), then for every data
// row a the share f_a = C1h_aa / C_aa, C_aa = C1h_aa + Gaussian + super-sample
// as in k_rowexp, and per panel of 256 distinct rows the largest f_a.
constexpr int SPLIT_PANEL = 256;  // rows per panel: the bf16 Gram tile

__global__ void k_gsq(const double *__restrict__ G, int64_t items, int n_mg, double *__restrict__ S) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t item = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  if (item >= items) return;
  const double *g = G + item * n_mg;
  double acc = 0.0;
  for (int m = lane; m < n_mg; m += WAVE) acc += g[m] * g[m];
  acc = wave_sum(acc);
  if (lane == 0) S[item] = acc;
}

__global__ void k_gdiag(const int32_t *__restrict__ rowR, const double *__restrict__ Ts, const double *__restrict__ S,
                        int64_t n_R, int n_chi, double *__restrict__ gd) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  if (row >= n_R) return;
  const int c = rowR[4 * row];
  const double *t = Ts + row * n_chi;
  const double *sc = S + (int64_t)c * n_chi;
  double acc = 0.0;
  for (int n = lane; n < n_chi; n += WAVE) acc += t[n] * t[n] * sc[n];
  acc = wave_sum(acc);
  if (lane == 0) gd[row] = acc;
}

__global__ void k_zero_f64(double *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

__global__ void k_split_share(AsmArgs A, const double *__restrict__ gd, double *__restrict__ F,
                              const int32_t *__restrict__ pos) {
  const int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (a >= A.n) return;
  const int32_t *ra = A.rowO + 8 * a;
  const int64_t e = ra[1];
  const double c1h = ldexp(gd[e], -2 * A.sexp[e]) * A.inv_omega;
  const double rr = A.rR[e];
  const double c = c1h + gauss_entry(A, ra, ra) + A.sigma_b2 * rr * rr;
  // a share of 1 (no other term) for a row whose diagonal is not positive
  const double f = c > 0.0 && isfinite(c) ? c1h / c : 1.0;
  // non-negative doubles order like their bit patterns
  const unsigned long long bits = (unsigned long long)__double_as_longlong(f);
  atomicMax((unsigned long long *)&F[(pos ? pos[e] : e) / SPLIT_PANEL], bits);  // the panel of its A-row
  atomicMax((unsigned long long *)&F[A.ld_g / SPLIT_PANEL], bits);  // the largest of all panels
}

void launch_split_plan(const AsmArgs &a, const int32_t *rowR, const double *Ts, const double *G, int64_t n_R,
                       int n_cfg, int n_chi, int n_mg, double *S, double *gd, double *F, int n_panels, hipStream_t s,
                       const int32_t *pos) {
  const int64_t items = (int64_t)n_cfg * n_chi;
  hipLaunchKernelGGL(k_gsq, dim3((unsigned)((items + 3) / 4)), dim3(256), 0, s, G, items, n_mg, S);
  hipLaunchKernelGGL(k_gdiag, dim3((unsigned)((n_R + 3) / 4)), dim3(256), 0, s, rowR, Ts, S, n_R, n_chi, gd);
  hipLaunchKernelGGL(k_zero_f64, dim3((n_panels + 256) / 256), dim3(256), 0, s, F, n_panels + 1);
  hipLaunchKernelGGL(k_split_share, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a, gd, F, pos);
}

// 64 x 64 output tiles (I >= J); each thread computes 16 entries of one
// column, the transposed copy goes through LDS so both halves are written
// with contiguous rows.  Tiles are numbered row-major over the triangle and
// each XCD (workgroup b runs on XCD b mod 8, each XCD has its own L2) takes
// a contiguous run of them, so the one-halo rows of a tile row are fetched
// into one L2 instead of all eight.  A tile's loads form two rounds: the
// row records and output exponents, then (all depending only on the
// records) the one-halo values and the distinct rows' exponents and
// responses, so a workgroup waits on global memory twice before it writes.
constexpr int AT = 64;
constexpr int ASM_XCD = 8;

template <typename OutT>
__global__ __launch_bounds__(256) void k_assemble(AsmArgs A, const int32_t *__restrict__ row_exp2,
                                                  OutT *__restrict__ C, int64_t n_tiles) {
  __shared__ OutT tileT[AT][AT + 1];
  __shared__ int32_t rowA[AT][8], rowB[AT][8];
  __shared__ int32_t tA[AT], tB[AT], sA[AT], sB[AT];
  __shared__ double rA[AT], rB[AT];
  const int64_t per = (int64_t)gridDim.x / ASM_XCD;
  const int64_t t = (int64_t)(blockIdx.x % ASM_XCD) * per + blockIdx.x / ASM_XCD;
  if (t >= n_tiles) return;  // grid padding (whole workgroup)
  int64_t i = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  const int64_t I = i, J = t - i * (i + 1) / 2;
  const int64_t a0 = I * AT, b0 = J * AT;
  const int tid = threadIdx.x;
  for (int q = tid; q < AT * 8; q += 256) {
    const int r = q / 8, c = q % 8;
    rowA[r][c] = a0 + r < A.n ? A.rowO[(a0 + r) * 8 + c] : 0;
    rowB[r][c] = b0 + r < A.n ? A.rowO[(b0 + r) * 8 + c] : 0;
  }
  if (tid < AT) {
    tA[tid] = a0 + tid < A.n ? row_exp2[a0 + tid] : 0;
  } else if (tid < 2 * AT) {
    tB[tid - AT] = b0 + tid - AT < A.n ? row_exp2[b0 + tid - AT] : 0;
  }
  __syncthreads();
  const int cb = tid & 63;          // column within the tile
  const int rbase = (tid >> 6) * 16;
  const int64_t b = b0 + cb;
  // the 16 one-halo values, all loads in flight together with those of the
  // exponents and responses (padding rows map to distinct row 0, so every
  // index is valid)
  // (the one-halo block has the output's type: FP32 for the mixed modes)
  OutT gv[16];
  const int64_t eb = rowB[cb][1];
  const OutT *G = (const OutT *)A.Gm;
#pragma unroll
  for (int q = 0; q < 16; ++q) gv[q] = G[rowA[rbase + q][1] * A.ld_g + eb];
  if (tid < AT) {
    const bool live = a0 + tid < A.n;
    sA[tid] = live ? A.sexp[rowA[tid][1]] : 0;
    rA[tid] = live ? A.rR[rowA[tid][1]] : 0.0;
  } else if (tid < 2 * AT) {
    const int q = tid - AT;
    const bool live = b0 + q < A.n;
    sB[q] = live ? A.sexp[rowB[q][1]] : 0;
    rB[q] = live ? A.rR[rowB[q][1]] : 0.0;
  }
  __syncthreads();
#pragma unroll 4
  for (int q = 0; q < 16; ++q) {
    const int ra = rbase + q;
    const int64_t a = a0 + ra;
    OutT v = 0;
    const bool live = a < A.n && b < A.n && a >= b;
    if (live) {
      const int tt = tA[ra] + tB[cb];
      const double g = (double)gv[q];
      double rest = A.sigma_b2 * rA[ra] * rB[cb] + gauss_entry(A, rowA[ra], rowB[cb]);
      if (A.ngins) rest += ngins_entry(A, rowA[ra], rowB[cb]);
      v = (OutT)(ldexp(g * A.inv_omega, tt - sA[ra] - sB[cb]) + ldexp(rest, tt));
      C[a * A.n + b] = v;
    }
    tileT[ra][cb] = v;
  }
  __syncthreads();
  // transposed half: C[b][a] for the same pairs, rows of the output contiguous,
  // with non-temporal stores (measured 1 ms faster at N = 82575; both halves
  // non-temporal was 2 ms slower)
#pragma unroll 4
  for (int q = 0; q < 16; ++q) {
    const int rb = rbase + q;  // row of the transposed tile (b index)
    const int ca = cb;         // column (a index)
    const int64_t bb = b0 + rb, aa = a0 + ca;
    if (aa < A.n && bb < A.n && aa > bb) __builtin_nontemporal_store(tileT[ca][rb], &C[bb * A.n + aa]);
  }
}

void launch_assemble(const AsmArgs &a, const int32_t *row_exp2, void *C, hipStream_t s) {
  const int64_t nt = (a.n + AT - 1) / AT;
  const int64_t tiles = nt * (nt + 1) / 2;
  const dim3 grid((unsigned)((tiles + ASM_XCD - 1) / ASM_XCD * ASM_XCD));
  if (a.gm_f32)
    hipLaunchKernelGGL(k_assemble<float>, grid, dim3(256), 0, s, a, row_exp2, (float *)C, tiles);
  else
    hipLaunchKernelGGL(k_assemble<double>, grid, dim3(256), 0, s, a, row_exp2, (double *)C, tiles);
}

}  // namespace wlc
