// One-halo covariance through its factorisation along the line of sight.
//
// A row of the flattened one-halo factor is A[row][(n, m)] = T_row(chi_n)
// G_c(chi_n, M_m), c the row's ell-configuration (eq. General1h with the
// Limber kernel of eq. nProjection), so
//   (A A^T)[a][b] = sum_n T_a(n) T_b(n) H_n[c(a)][c(b)],
//   H_n[c][c'] = sum_m G_c(n, m) G_c'(n, m).
// H is small (configurations x configurations x chi nodes), and the second
// sum is a product over the chi nodes only: N_M times fewer operations than
// the flattened Gram, and computed here in FP64 from the same factors T
// (which carry the rows' power-of-two scales) and G.
//
// Distinct rows are grouped by configuration with uniform block sizes
// (sp rows per power-spectrum configuration, sb per triangle).  Blocks are
// cut into sub-tiles of 64 rows; sub-tile rows are numbered configuration
// by configuration, so a pair of sub-tile rows R >= R' covers configurations
// c >= c' and one weight vector h = H[c][c'][.] applies to the whole pair:
// each pair is a 64 x 64 FP64 MFMA product over n with one operand scaled
// by h.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace wlc {

// ------------------------------------------------------------------ H
// H[c][c'][n] = sum_m G[c][n][m] G[c'][n][m]; block (n, group of 16 c).
constexpr int HG = 16;
constexpr int HM = 256;

__global__ __launch_bounds__(256) void k_hfactor(const double *__restrict__ G, int n_cfg, int n_chi, int n_m,
                                                 double *__restrict__ H) {
  __shared__ double Gs[HG][HM];
  const int n = blockIdx.x, c0 = blockIdx.y * HG;
  const int tid = threadIdx.x;
  for (int cp = tid; cp < ((n_cfg + 255) / 256) * 256; cp += 256) {
    double acc[HG];
#pragma unroll
    for (int i = 0; i < HG; ++i) acc[i] = 0.0;
    for (int m0 = 0; m0 < n_m; m0 += HM) {
      const int mlen = min(HM, n_m - m0);
      __syncthreads();
      for (int q = tid; q < HG * HM; q += 256) {
        const int i = q / HM, m = q % HM;
        Gs[i][m] = (c0 + i < n_cfg && m < mlen) ? G[((size_t)(c0 + i) * n_chi + n) * n_m + m0 + m] : 0.0;
      }
      __syncthreads();
      if (cp < n_cfg) {
        const double *g = G + ((size_t)cp * n_chi + n) * n_m + m0;
        for (int m = 0; m < mlen; ++m) {
          const double v = g[m];
#pragma unroll
          for (int i = 0; i < HG; ++i) acc[i] += Gs[i][m] * v;
        }
      }
    }
    if (cp < n_cfg) {
#pragma unroll
      for (int i = 0; i < HG; ++i)
        if (c0 + i < n_cfg) H[((size_t)(c0 + i) * n_cfg + cp) * n_chi + n] = acc[i];
    }
  }
}

// ------------------------------------------------------------------ C_1h
struct SubRow {
  int c;       // configuration
  int64_t e0;  // first distinct row
  int cnt;     // rows in this sub-tile (<= 64)
};

__device__ __forceinline__ SubRow sub_row(int64_t R, int nl, int sp, int sb, int tp, int tb) {
  SubRow s;
  if (R < (int64_t)nl * tp) {
    const int c = (int)(R / tp), ti = (int)(R % tp);
    s.c = c;
    s.e0 = (int64_t)c * sp + ti * 64;
    s.cnt = min(64, sp - ti * 64);
  } else {
    const int64_t q = R - (int64_t)nl * tp;
    const int t = (int)(q / tb), ti = (int)(q % tb);
    s.c = nl + t;
    s.e0 = (int64_t)nl * sp + (int64_t)t * sb + ti * 64;
    s.cnt = min(64, sb - ti * 64);
  }
  return s;
}

constexpr int CK = 16;        // chi nodes per LDS stage
constexpr int CLD = CK + 1;   // padded row

__global__ __launch_bounds__(256) void k_chifact(const double *__restrict__ Ts, const double *__restrict__ H,
                                                 int n_cfg, int n_chi, int nl, int sp, int sb, int tp, int tb,
                                                 double *__restrict__ out, int64_t ld) {
  __shared__ double lds[2][64 * CLD];  // [A' rows, B rows][64][CK]
  int64_t R, Rp;
  {
    const int64_t t = blockIdx.x;
    int64_t i = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    while (i * (i + 1) / 2 > t) --i;
    R = i;
    Rp = t - i * (i + 1) / 2;
  }
  const SubRow A = sub_row(R, nl, sp, sb, tp, tb), B = sub_row(Rp, nl, sp, sb, tp, tb);
  const double *h = H + ((size_t)A.c * n_cfg + B.c) * n_chi;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  f64x4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = f64x4{0.0, 0.0, 0.0, 0.0};

  // staging: 64 rows x CK nodes per side, 4 per thread; element q is row
  // q / CK, node q % CK
  double pa[4], pb[4];
  // (loads unconditional, from indices clamped into range, and masked by
  // multiplication afterwards: the factors are finite, and all 12 loads of
  // a thread are in flight together)
  auto gload = [&](int n0) {
    double ta[4], tb[4], hv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = tid + 256 * j;
      const int r = q / CK, n = min(n0 + q % CK, n_chi - 1);
      ta[j] = Ts[(size_t)(A.e0 + min(r, A.cnt - 1)) * n_chi + n];
      tb[j] = Ts[(size_t)(B.e0 + min(r, B.cnt - 1)) * n_chi + n];
      hv[j] = h[n];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = tid + 256 * j;
      const int r = q / CK, n = n0 + q % CK;
      const bool kin = n < n_chi;
      pa[j] = ta[j] * hv[j] * ((kin && r < A.cnt) ? 1.0 : 0.0);
      pb[j] = tb[j] * ((kin && r < B.cnt) ? 1.0 : 0.0);
    }
  };
  gload(0);
  for (int n0 = 0; n0 < n_chi; n0 += CK) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = tid + 256 * j;
      lds[0][(q / CK) * CLD + q % CK] = pa[j];
      lds[1][(q / CK) * CLD + q % CK] = pb[j];
    }
    __syncthreads();
    if (n0 + CK < n_chi) gload(n0 + CK);
#pragma unroll
    for (int kk = 0; kk < CK; kk += 4) {
      const int kc = kk + (lane >> 4);
      double a[2], b[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        a[x] = lds[0][(wr + x * 16 + (lane & 15)) * CLD + kc];
        b[x] = lds[1][(wc + x * 16 + (lane & 15)) * CLD + kc];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
    }
  }
  // accumulator value v of lane l: row l / 16 + 4 v, column l % 16; the
  // product is written non-temporal (the later kernels then run 2.6 ms faster
  // at large10: fewer dirty lines left to write back under them)
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = wr + x * 16 + (lane >> 4) + 4 * v;
        const int c = wc + y * 16 + (lane & 15);
        if (r < A.cnt && c < B.cnt) __builtin_nontemporal_store(acc[x][y][v], &out[(A.e0 + r) * ld + B.e0 + c]);
      }
}

void launch_chifact(const double *Ts, const double *G, double *H, int n_cfg, int n_chi, int n_m, int nl, int sp,
                    int sb, int n_tri, double *out, int64_t ld, hipStream_t s) {
  hipLaunchKernelGGL(k_hfactor, dim3((unsigned)n_chi, (unsigned)((n_cfg + HG - 1) / HG)), dim3(256), 0, s, G, n_cfg,
                     n_chi, n_m, H);
  const int tp = (sp + 63) / 64, tb = sb > 0 ? (sb + 63) / 64 : 1;
  const int64_t ns = (int64_t)nl * tp + (int64_t)n_tri * tb;
  const int64_t items = ns * (ns + 1) / 2;
  if (items > 0)
    hipLaunchKernelGGL(k_chifact, dim3((unsigned)items), dim3(256), 0, s, Ts, H, n_cfg, n_chi, nl, sp, sb, tp, tb,
                       out, ld);
}

}  // namespace wlc
