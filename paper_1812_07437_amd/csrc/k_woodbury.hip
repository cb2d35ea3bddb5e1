// Signal-to-noise (eq. SNprim) through the distinct rows.
//
// The joint covariance is C = C_G + E M E^T: C_G the Gaussian term, zero
// between different ell-configurations (eqs. CovPPG, CovPBsynt and the
// Gaussian term of App. B); E the map from data-vector rows to distinct rows
// (the Limber kernels are symmetric in the bins, so the one-halo term, the
// response and d itself depend only on the multiset of bins); and
// M = C_1h + sigma_b^2 r r^T on the distinct rows.  Since d = E d_R,
//   (S/N)^2 = d_R^T (G^-1 + M)^-1 d_R = u^T (I + Z)^-1 u,
//   G = E^T C_G^-1 E = L L^T,  u = L^T d_R,  Z = L^T M L,
// an identity with no cancellation; the one large factorisation is that of
// I + Z (N_R rows instead of N), done by the bordered Cholesky.
//
// G is block-diagonal over configurations and each block has a closed form
// in Q_b = (P^s_b)^-1.  On the data-vector rows of one configuration the
// Gaussian block is
//   P rows (pairs i <= j):        S2(P_b) / N(l_b)
//   scalene triangle:             (Omega / N_tri) P_1 (x) P_2 (x) P_3
//   l1 = l2 < l3 (rows i <= j, k): (Omega / N_tri) S2(P_1) (x) P_3
//   l1 < l2 = l3 (rows i, j <= k): (Omega / N_tri) P_1 (x) S2(P_2)
//   equilateral (rows i <= j <= k): (Omega / N_tri) S3(P_b)
// with S2(P)[(ij)(kl)] = P_ik P_jl + P_il P_jk and S3(P) the sum over the six
// leg permutations.  These products are symmetric under the permutations of
// equal legs, and on the symmetric subspace their inverses are
//   S2(P)^-1 = (nu nu^T / 4) o S2(Q),  S3(P)^-1 = (mu mu^T / 36) o S3(Q),
// nu and mu counting the distinct orderings of the bins.  G then sums the
// inverse over the rows that share a multiset of bins.
//
// Rows are scaled by powers of two throughout (G by D = diag(2^tau) so that
// its diagonal lies in [1, 4), M by D^-1), so that every factor stays near
// unit size; the scaling is exact.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace wlc {

// ------------------------------------------------------------------ Q
constexpr int QMAX = WOOD_NZ_MAX;

// Q_b = (P^s_b)^-1 for every ell-bin, one thread per bin (n_z <= QMAX).
__global__ void k_qinv(const double *__restrict__ Ps, int n_ell, int nz, double *__restrict__ Q,
                       int *__restrict__ flag) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_ell) return;
  double L[QMAX][QMAX];
  const double *P = Ps + (size_t)b * nz * nz;
  bool bad = false;
  for (int j = 0; j < nz; ++j) {
    double s = P[j * nz + j];
    for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
    if (!(s > 0.0)) {
      bad = true;
      s = 1.0;
    }
    L[j][j] = sqrt(s);
    for (int i = j + 1; i < nz; ++i) {
      double t = P[i * nz + j];
      for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
      L[i][j] = t / L[j][j];
    }
  }
  // X = L^-1 in the upper part of L (X[i][j] for i >= j stored at L[j][i])
  for (int j = 0; j < nz; ++j) {
    L[j][j] = 1.0 / L[j][j];
    for (int i = j + 1; i < nz; ++i) {
      double t = 0.0;
      for (int k = j; k < i; ++k) t -= L[i][k] * (k == j ? L[j][j] : L[j][k]);
      L[j][i] = t / L[i][i];
    }
  }
  // Q = X^T X
  for (int i = 0; i < nz; ++i)
    for (int j = 0; j < nz; ++j) {
      double t = 0.0;
      for (int k = (i > j ? i : j); k < nz; ++k) {
        const double xi = k == i ? L[i][i] : L[i][k];  // X[k][i]
        const double xj = k == j ? L[j][j] : L[j][k];
        t += xi * xj;
      }
      Q[((size_t)b * nz + i) * nz + j] = t;
    }
  if (bad) atomicOr(flag, 1);
}

// ------------------------------------------------------------------ G
__device__ __forceinline__ void decode_pair(int m, int nz, int &i, int &j) {
  for (i = 0; i < nz; ++i) {
    const int cnt = nz - i;
    if (m < cnt) {
      j = i + m;
      return;
    }
    m -= cnt;
  }
}

__device__ __forceinline__ void decode_trip(int m, int nz, int &i, int &j, int &k) {
  for (i = 0; i < nz; ++i)
    for (j = i; j < nz; ++j) {
      const int cnt = nz - j;
      if (m < cnt) {
        k = j + m;
        return;
      }
      m -= cnt;
    }
}

struct Qv {
  const double *Q;
  int nz;
  __device__ double operator()(int b, int x, int y) const { return Q[((size_t)b * nz + x) * nz + y]; }
};

__device__ __forceinline__ double s2(const Qv &q, int b, int i, int j, int k, int l) {
  return q(b, i, k) * q(b, j, l) + q(b, i, l) * q(b, j, k);
}

// distinct orderings of a sorted triple; returns their number
__device__ __forceinline__ int orderings(const int m[3], int out[6][3]) {
  const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  int n = 0;
  for (int p = 0; p < 6; ++p) {
    const int a = m[perm[p][0]], b = m[perm[p][1]], c = m[perm[p][2]];
    bool dup = false;
    for (int q = 0; q < n; ++q) dup |= (out[q][0] == a && out[q][1] == b && out[q][2] == c);
    if (!dup) {
      out[n][0] = a;
      out[n][1] = b;
      out[n][2] = c;
      ++n;
    }
  }
  return n;
}

// For a triangle with two equal legs, the data-vector rows of multiset m:
// the bin on the odd leg is one of the distinct values of m and the other two
// are sorted.  Returns the count; odd[q] is the odd leg's bin, (lo, hi) the pair.
__device__ __forceinline__ int odd_leg_rows(const int m[3], int odd[3], int lo[3], int hi[3]) {
  int n = 0;
  for (int q = 0; q < 3; ++q) {
    if (q > 0 && m[q] == m[q - 1]) continue;
    const int a = q == 0 ? m[1] : m[0], b = q == 2 ? m[1] : m[2];
    odd[n] = m[q];
    lo[n] = a;
    hi[n] = b;
    ++n;
  }
  return n;
}

__global__ void k_gblock(BlockMap B, const int32_t *__restrict__ cfgT, Qv q, const double *__restrict__ nmodes,
                         const double *__restrict__ ntri, double omega, double *__restrict__ Gb) {
  const int c = blockIdx.y;
  const int s = B.size(c);
  const int nz = q.nz;
  double *G = Gb + B.off(c);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)s * s;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int mi = (int)(e / s), mj = (int)(e % s);
    if (mj > mi) continue;
    double v = 0.0;
    if (c < B.nl) {
      int i, j, k, l;
      decode_pair(mi, nz, i, j);
      decode_pair(mj, nz, k, l);
      const double nu = (i == j ? 1.0 : 2.0) * (k == l ? 1.0 : 2.0);
      v = nmodes[c] * nu * 0.25 * s2(q, c, i, j, k, l);
    } else {
      const int l1 = cfgT[4 * c + 1], l2 = cfgT[4 * c + 2], l3 = cfgT[4 * c + 3];
      int m[3], mp[3];
      decode_trip(mi, nz, m[0], m[1], m[2]);
      decode_trip(mj, nz, mp[0], mp[1], mp[2]);
      if (l1 == l2 && l2 == l3) {
        int oa[6][3], ob[6][3];
        const int na = orderings(m, oa), nb = orderings(mp, ob);
        double t = 0.0;
        for (int p = 0; p < nb; ++p) t += q(l1, m[0], ob[p][0]) * q(l1, m[1], ob[p][1]) * q(l1, m[2], ob[p][2]);
        // the six leg permutations visit each distinct ordering 6 / nb times
        v = (double)(na * nb) / 36.0 * (6.0 / nb) * t;
      } else if (l1 == l2 || l2 == l3) {
        int oa[3], la[3], ha[3], ob[3], lb[3], hb[3];
        const int na = odd_leg_rows(m, oa, la, ha), nb = odd_leg_rows(mp, ob, lb, hb);
        const int lp = l1 == l2 ? l1 : l2, lodd = l1 == l2 ? l3 : l1;
        for (int x = 0; x < na; ++x)
          for (int y = 0; y < nb; ++y) {
            const double nu = (la[x] == ha[x] ? 1.0 : 2.0) * (lb[y] == hb[y] ? 1.0 : 2.0);
            v += nu * 0.25 * s2(q, lp, la[x], ha[x], lb[y], hb[y]) * q(lodd, oa[x], ob[y]);
          }
      } else {
        int oa[6][3], ob[6][3];
        const int na = orderings(m, oa), nb = orderings(mp, ob);
        for (int x = 0; x < na; ++x)
          for (int y = 0; y < nb; ++y) v += q(l1, oa[x][0], ob[y][0]) * q(l2, oa[x][1], ob[y][1]) * q(l3, oa[x][2], ob[y][2]);
      }
      v *= ntri[c - B.nl] / omega;
    }
    G[(int64_t)mi * s + mj] = v;
  }
}

// ------------------------------------------------------------------ blocks
// Per block (one workgroup): row scales tau with G_ee 2^(2 tau) in [1, 4),
// the scaled block factored in place (lower), u = L^T D^-1 d_R into the
// border row, and r scaled by D^-1.
__global__ __launch_bounds__(256) void k_gchol(BlockMap B, double *__restrict__ Gb, const double *__restrict__ dR,
                                               const double *__restrict__ rR, int32_t *__restrict__ tau,
                                               double *__restrict__ rhat, double *__restrict__ urow,
                                               int *__restrict__ flag) {
  __shared__ double piv;
  __shared__ int bad;
  const int c = blockIdx.x;
  const int s = B.size(c);
  const int64_t b0 = B.start(c);
  double *A = Gb + B.off(c);
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  for (int e = tid; e < s; e += 256) {
    const double g = A[(int64_t)e * s + e];
    int t = 0;
    if (g > 0.0 && isfinite(g)) {
      const int q = exp2_of(g) - 1;
      t = -(q >= 0 ? q / 2 : -((1 - q) / 2));  // -floor((E - 1) / 2)
    }
    tau[b0 + e] = t;
    rhat[b0 + e] = ldexp(rR[b0 + e], -t);
  }
  __syncthreads();
  for (int64_t e = tid; e < (int64_t)s * s; e += 256) {
    const int i = (int)(e / s), j = (int)(e % s);
    if (j <= i) A[e] = ldexp(A[e], tau[b0 + i] + tau[b0 + j]);
  }
  __syncthreads();
  for (int k = 0; k < s; ++k) {
    if (tid == 0) {
      const double v = A[(int64_t)k * s + k];
      if (!(v > 0.0)) bad = 1;
      piv = sqrt(v > 0.0 ? v : 1.0);
      A[(int64_t)k * s + k] = piv;
    }
    __syncthreads();
    const double rp = 1.0 / piv;
    for (int i = k + 1 + tid; i < s; i += 256) A[(int64_t)i * s + k] *= rp;
    __syncthreads();
    const int m = s - 1 - k;
    for (int e = tid; e < m * m; e += 256) {
      const int i = k + 1 + e / m, j = k + 1 + e % m;
      if (j <= i) A[(int64_t)i * s + j] -= A[(int64_t)i * s + k] * A[(int64_t)j * s + k];
    }
    __syncthreads();
  }
  for (int e = tid; e < s; e += 256) {
    double u = 0.0;
    for (int f = e; f < s; ++f) u += A[(int64_t)f * s + e] * ldexp(dR[b0 + f], -tau[b0 + f]);
    urow[b0 + e] = u;
  }
  if (tid == 0 && bad) atomicOr(flag, 1);
}

// ------------------------------------------------------------------ products
// MODE 0:  T[e][g] = sum_{h in block(e), h >= e} L[h][e] Mhat[g][h]   (all tiles)
// MODE 1:  W[e][f] = delta_ef + sum_{g in block(f), g >= f} T[e][g] L[g][f]   (e >= f)
// with Mhat[g][h] = 2^-(s_g + s_h + tau_g + tau_h) Gm[g][h] / Omega
//                  + sigma_b^2 rhat_g rhat_h,
// Gm the mirrored (symmetric) Gram output.  64 x 64 tiles on
// v_mfma_f64_16x16x4 (four wavefronts of 32 x 32); the contraction runs over
// the configuration blocks that the tile's rows (MODE 0) or columns (MODE 1)
// touch, in LDS stages of 16.
struct WbArgs {
  BlockMap B;
  const double *Gb;        // factored blocks
  const void *Gm;          // symmetric Gram, f32 or f64, pitch ld_g
  int gm_f32;
  int64_t ld_g;
  const int32_t *sexp;     // Gram row exponents
  const int32_t *tau;
  const double *rhat;
  double inv_omega, sigma_b2;
  double *T;               // [n_R][ld_t]
  int64_t ld_t;
  double *W;               // [n_R + 1][ld_w]
  int64_t ld_w;
};

constexpr int WK = 16;
constexpr int WLD = WK + 1;

template <int MODE>
__global__ __launch_bounds__(256) void k_wb_prod(WbArgs a) {
  __shared__ double lds[2][64 * WLD];
  const int64_t nR = a.B.n_R;
  const int64_t nt = (nR + 63) / 64;
  int64_t ti, tj;
  if (MODE == 0) {
    ti = blockIdx.x / nt;
    tj = blockIdx.x % nt;
  } else {
    const int64_t t = blockIdx.x;
    int64_t i = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    while (i * (i + 1) / 2 > t) --i;
    ti = i;
    tj = t - i * (i + 1) / 2;
  }
  const int64_t e0 = ti * 64, f0 = tj * 64;
  // contraction range: the blocks spanned by the rows (MODE 0) or columns (MODE 1)
  const int64_t s0 = MODE == 0 ? e0 : f0;
  const int64_t s1 = min(nR, s0 + 64) - 1;
  const int cb0 = a.B.blk(s0), cb1 = a.B.blk(s1);
  const int64_t k0 = a.B.start(cb0), k1 = a.B.start(cb1) + a.B.size(cb1);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  f64x4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = f64x4{0.0, 0.0, 0.0, 0.0};
  // Per loaded element j of this thread: its row r = q / WK of the tile is
  // fixed, so the block facts of the L row (e in MODE 0, f in MODE 1) and
  // the scale of the Mhat row f (MODE 0) are taken once here, and the k
  // loop does no index division.
  double pa[4], pb[4];
  int64_t lb0[4], lb1[4], lbase[4];  // block [lb0, lb1) holding the L row, Gb index of L[lb0][row]
  int lsz[4];
  double fscale[4], frh[4];          // MODE 0: 2^-(s_f + tau_f) / Omega and sigma_b^2 rhat_f
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int r = (tid + 256 * j) / WK;
    const int64_t lr = (MODE == 0 ? e0 : f0) + r;  // the row whose L column is read
    lb0[j] = lb1[j] = lbase[j] = 0;
    lsz[j] = 0;
    if (lr < nR) {
      const int c = a.B.blk(lr);
      lb0[j] = a.B.start(c);
      lsz[j] = a.B.size(c);
      lb1[j] = lb0[j] + lsz[j];
      lbase[j] = a.B.off(c) + (lr - lb0[j]);
    }
    fscale[j] = frh[j] = 0.0;
    if (MODE == 0 && f0 + r < nR) {
      const int64_t f = f0 + r;
      fscale[j] = ldexp(a.inv_omega, -(a.sexp[f] + a.tau[f]));
      frh[j] = a.sigma_b2 * a.rhat[f];
    }
  }
  auto gload = [&](int64_t kq) {
    // every element of this thread sits in column k = kq + tid % WK of the
    // stage, so the column's Mhat factors are loaded once.  All loads are
    // unconditional, from indices clamped into range, and masked afterwards
    // by multiplication (the values are finite), so they are in flight
    // together instead of one branch and wait each.
    const int64_t k = kq + tid % WK;
    const bool kin = k < k1;
    const int64_t kc = kin ? k : k1 - 1;
    int sk = 0;
    double rk = 0.0;
    if (MODE == 0) {
      sk = a.sexp[kc] + a.tau[kc];
      rk = a.rhat[kc];
    }
    double lw[4], gw[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t lr = (MODE == 0 ? e0 : f0) + (tid + 256 * j) / WK;
      // L[k][lr]: nonzero only inside lr's block, on or below its diagonal;
      // elsewhere the block's diagonal entry L[lr][lr] is read instead
      const bool lin = k >= lr && k < lb1[j];
      lw[j] = a.Gb[lbase[j] + ((lin ? k : lr) - lb0[j]) * lsz[j]];
    }
    if (MODE == 0) {
      if (a.gm_f32) {
        float gf[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          gf[j] = ((const float *)a.Gm)[min(f0 + (tid + 256 * j) / WK, nR - 1) * a.ld_g + kc];
#pragma unroll
        for (int j = 0; j < 4; ++j) gw[j] = (double)gf[j];
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) gw[j] = ((const double *)a.Gm)[min(f0 + (tid + 256 * j) / WK, nR - 1) * a.ld_g + kc];
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) gw[j] = a.T[min(e0 + (tid + 256 * j) / WK, nR - 1) * a.ld_t + kc];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = (tid + 256 * j) / WK;
      const int64_t e = e0 + r, f = f0 + r;
      const int64_t lr = MODE == 0 ? e : f;
      const double lv = lw[j] * ((k >= lr && k < lb1[j]) ? 1.0 : 0.0);
      const double in = kin ? 1.0 : 0.0;
      if (MODE == 0) {
        pa[j] = lv * in;
        pb[j] = (ldexp(gw[j] * fscale[j], -sk) + frh[j] * rk) * ((f < nR && kin) ? 1.0 : 0.0);
      } else {
        pa[j] = gw[j] * ((e < nR && kin) ? 1.0 : 0.0);
        pb[j] = lv * in;
      }
    }
  };
  gload(k0);
  for (int64_t kq = k0; kq < k1; kq += WK) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = tid + 256 * j;
      lds[0][(q / WK) * WLD + q % WK] = pa[j];
      lds[1][(q / WK) * WLD + q % WK] = pb[j];
    }
    __syncthreads();
    if (kq + WK < k1) gload(kq + WK);
#pragma unroll
    for (int kk = 0; kk < WK; kk += 4) {
      const int kc = kk + (lane >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        av[x] = lds[0][(wr + x * 16 + (lane & 15)) * WLD + kc];
        bv[x] = lds[1][(wc + x * 16 + (lane & 15)) * WLD + kc];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x], bv[y], acc[x][y], 0, 0, 0);
    }
  }
  // accumulator value v of lane l: row l / 16 + 4 v, column l % 16; W goes
  // out non-temporal (fewer dirty lines under the kernels after it)
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t e = e0 + wr + x * 16 + (lane >> 4) + 4 * v;
        const int64_t f = f0 + wc + y * 16 + (lane & 15);
        if (e >= nR || f >= nR) continue;
        if (MODE == 0) a.T[e * a.ld_t + f] = acc[x][y][v];
        else if (e >= f) __builtin_nontemporal_store(acc[x][y][v] + (e == f ? 1.0 : 0.0), &a.W[e * a.ld_w + f]);
      }
}

// ------------------------------------------------------------------ driver
void launch_woodbury(const WoodArgs &w, hipStream_t s) {
  const BlockMap &B = w.B;
  const int n_cfg = B.nl + B.n_tri;
  hipLaunchKernelGGL(k_qinv, dim3((w.n_ell + 63) / 64), dim3(64), 0, s, w.Ps, w.n_ell, w.nz, w.Q, w.flag);
  const int smax = B.sb > B.sp ? B.sb : B.sp;
  const unsigned gx = (unsigned)((smax * smax + 255) / 256);
  hipLaunchKernelGGL(k_gblock, dim3(gx, (unsigned)n_cfg), dim3(256), 0, s, B, w.cfgT, Qv{w.Q, w.nz}, w.nmodes,
                     w.ntri, w.omega, w.Gb);
  hipLaunchKernelGGL(k_gchol, dim3((unsigned)n_cfg), dim3(256), 0, s, B, w.Gb, w.dR, w.rR, w.tau, w.rhat,
                     w.W + B.n_R * w.ld_w, w.flag);
  WbArgs a{B, w.Gb, w.Gm, w.gm_f32, w.ld_g, w.sexp, w.tau, w.rhat, 1.0 / w.omega, w.sigma_b2, w.T, w.ld_t, w.W,
           w.ld_w};
  const int64_t nt = (B.n_R + 63) / 64;
  hipLaunchKernelGGL(k_wb_prod<0>, dim3((unsigned)(nt * nt)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_wb_prod<1>, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(256), 0, s, a);
}

}  // namespace wlc
