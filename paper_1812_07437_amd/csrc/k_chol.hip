// (S/N)^2 = D^T C^-1 D (Rizzato et al. 2019, eq. SNprim) by an FP64 Cholesky
// factorisation of the bordered matrix
//     M = [ C~    d~ ]        C~ = 2^t C 2^t,  d~ = 2^t d,
//         [ d~^T   . ]
// Factoring the first n columns of M leaves y = L^-1 d~ in its last row, and
// (S/N)^2 = y^T y.  Right-looking blocked algorithm on the lower triangle:
// 64-wide panels (diagonal block factored and inverted in LDS, panel solved by
// multiplication with that inverse), trailing updates on f64 MFMA with up to
// 256-wide slices of the factored panel.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace wlc {

constexpr int NB = 64;       // inner panel width
constexpr int NB_OUT = 256;  // outer panel width

// ------------------------------------------------------------- prepare
// Lower triangle of M from the scaled covariance (f32 or f64) and d.
template <typename InT>
__global__ void k_chol_prep(const InT *__restrict__ C, const int32_t *__restrict__ t, const double *__restrict__ d,
                            int64_t n, int64_t ld, int64_t row_off, double *__restrict__ Wm) {
  const int64_t i = row_off + blockIdx.y;  // row of M, 0..n
  if (i > n) return;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j <= i && j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    Wm[i * ld + j] = i < n ? (double)C[i * n + j] : ldexp(d[j], t[j]);
  }
}

void launch_chol_prep(const void *C, int c_f32, const int32_t *row_exp2, const double *d, int64_t n, int64_t ld,
                      double *Wm, hipStream_t s) {
  for (int64_t r0 = 0; r0 <= n; r0 += 65535) {
    const int64_t rows = std::min<int64_t>(65535, n + 1 - r0);
    const dim3 grid((unsigned)std::min<int64_t>((n + 255) / 256, 512), (unsigned)rows);
    if (c_f32)
      hipLaunchKernelGGL(k_chol_prep<float>, grid, dim3(256), 0, s, (const float *)C, row_exp2, d, n, ld, r0, Wm);
    else
      hipLaunchKernelGGL(k_chol_prep<double>, grid, dim3(256), 0, s, (const double *)C, row_exp2, d, n, ld, r0, Wm);
  }
}

// ------------------------------------------------------------- diagonal block
// Factor the jb x jb diagonal block at j0 in LDS (column by column), write L
// back and its inverse Linv (lower triangular, row-major jb x NB) to global.
__global__ __launch_bounds__(256) void k_potrf_diag(double *__restrict__ Wm, int64_t ld, int64_t j0, int jb,
                                                    double *__restrict__ Linv, int *__restrict__ flag) {
  __shared__ double L[NB][NB + 1];
  __shared__ double X[NB][NB + 1];
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  for (int q = tid; q < NB * NB; q += 256) {
    const int r = q / NB, c = q % NB;
    L[r][c] = (r < jb && c <= r) ? Wm[(j0 + r) * ld + j0 + c] : 0.0;
    X[r][c] = 0.0;
  }
  __syncthreads();
  for (int k = 0; k < jb; ++k) {
    if (tid == 0) {
      const double p = L[k][k];
      if (!(p > 0.0)) bad = 1;
      L[k][k] = sqrt(fabs(p) > 0.0 ? fabs(p) : 1.0);
    }
    __syncthreads();
    const double dk = L[k][k];
    for (int r = k + 1 + tid; r < jb; r += 256) L[r][k] /= dk;
    __syncthreads();
    // trailing update of the block: rows r > k, columns c in (k, r]
    const int m = jb - k - 1;
    for (int q = tid; q < m * m; q += 256) {
      const int r = k + 1 + q / m, c = k + 1 + q % m;
      if (c <= r) L[r][c] -= L[r][k] * L[c][k];
    }
    __syncthreads();
  }
  // inverse of the lower-triangular factor, one column per thread group:
  // X L = I solved column by column of the identity
  for (int c = tid; c < jb; c += 256) {
    for (int r = c; r < jb; ++r) {
      double s = (r == c) ? 1.0 : 0.0;
      for (int q = c; q < r; ++q) s -= L[r][q] * X[q][c];
      X[r][c] = s / L[r][r];
    }
  }
  __syncthreads();
  for (int q = tid; q < jb * jb; q += 256) {
    const int r = q / jb, c = q % jb;
    if (c <= r) Wm[(j0 + r) * ld + j0 + c] = L[r][c];
    Linv[r * NB + c] = c <= r ? X[r][c] : 0.0;
  }
  if (tid == 0 && bad) atomicOr(flag, 1);
}

// ------------------------------------------------------------- panel solve
// Rows [r0, r1) of columns [j0, j0 + jb): X = B Linv^T, 64 rows per workgroup.
__global__ __launch_bounds__(256) void k_trsm(double *__restrict__ Wm, int64_t ld, int64_t j0, int jb, int64_t r0,
                                              int64_t r1, const double *__restrict__ Linv) {
  __shared__ double Li[NB][NB + 1];
  __shared__ double B[NB][NB + 1];
  const int tid = threadIdx.x;
  const int64_t rb = r0 + (int64_t)blockIdx.x * NB;
  for (int q = tid; q < NB * NB; q += 256) {
    const int r = q / NB, c = q % NB;
    Li[r][c] = (r < jb && c < jb) ? Linv[r * NB + c] : 0.0;
    B[r][c] = (rb + r < r1 && c < jb) ? Wm[(rb + r) * ld + j0 + c] : 0.0;
  }
  __syncthreads();
  const int r = tid & 63;
  const int cbase = (tid >> 6) * 16;
  double out[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int c = cbase + q;
    double s = 0.0;
    for (int k = 0; k <= c; ++k) s += B[r][k] * Li[c][k];
    out[q] = s;
  }
  if (rb + r < r1) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int c = cbase + q;
      if (c < jb) Wm[(rb + r) * ld + j0 + c] = out[q];
    }
  }
}

// ------------------------------------------------------------- trailing update
// W[i][j] -= sum_{q in [k0, k1)} W[i][q] W[j][q] for i in [c0, r1), j in
// [c0, c1), i >= j.  64 x 64 tiles, four wavefronts of 32 x 32 each on
// v_mfma_f64_16x16x4 (lane l holds row l % 16 and k l / 16 of each operand;
// accumulator value v of lane l is row l / 16 + 4 v, column l % 16).
constexpr int UT = 64;
constexpr int UK = 16;

__global__ __launch_bounds__(256) void k_update(double *__restrict__ Wm, int64_t ld, int64_t c0, int64_t r1, int64_t c1,
                                                int64_t k0, int64_t k1) {
  __shared__ double Sa[UT][UK + 1], Sb[UT][UK + 1];
  const int64_t ti = blockIdx.y, tj = blockIdx.x;
  const int64_t i0 = c0 + ti * UT, j0 = c0 + tj * UT;
  if (j0 > i0 + UT - 1) return;  // tile entirely above the diagonal
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int64_t kq = k0; kq < k1; kq += UK) {
    __syncthreads();
    for (int q = tid; q < UT * UK; q += 256) {
      const int r = q / UK, c = q % UK;
      const int64_t k = kq + c;
      Sa[r][c] = (i0 + r < r1 && k < k1) ? Wm[(i0 + r) * ld + k] : 0.0;
      Sb[r][c] = (j0 + r < c1 && k < k1) ? Wm[(j0 + r) * ld + k] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < UK; kk += 4) {
      const int kc = kk + (lane >> 4);
      double a[2], b[2];
#pragma unroll
      for (int blk = 0; blk < 2; ++blk) {
        a[blk] = Sa[wr + blk * 16 + (lane & 15)][kc];
        b[blk] = Sb[wc + blk * 16 + (lane & 15)][kc];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
    }
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = i0 + wr + x * 16 + (lane >> 4) + 4 * v;
        const int64_t j = j0 + wc + y * 16 + (lane & 15);
        if (i < r1 && j < c1 && i >= j) Wm[i * ld + j] -= acc[x][y][v];
      }
}

static void launch_update(double *Wm, int64_t ld, int64_t c0, int64_t r1, int64_t c1, int64_t k0, int64_t k1,
                          hipStream_t s) {
  if (c0 >= c1 || c0 >= r1 || k0 >= k1) return;
  const int64_t tr = (r1 - c0 + UT - 1) / UT, tc = (c1 - c0 + UT - 1) / UT;
  // grid y is bounded by 65535 tiles (4.2M rows)
  hipLaunchKernelGGL(k_update, dim3((unsigned)tc, (unsigned)tr), dim3(256), 0, s, Wm, ld, c0, r1, c1, k0, k1);
}

// Factor columns [0, n) of M (n + 1 rows).  Returns 0; the pivot flag is
// checked by the caller after synchronisation.
int chol_factor(double *Wm, int64_t n, int64_t ld, double *Linv, int *flag, hipStream_t s) {
  const int64_t rows = n + 1;
  for (int64_t J0 = 0; J0 < n; J0 += NB_OUT) {
    const int64_t Jend = std::min<int64_t>(J0 + NB_OUT, n);
    for (int64_t j0 = J0; j0 < Jend; j0 += NB) {
      const int jb = (int)std::min<int64_t>(NB, Jend - j0);
      hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, s, Wm, ld, j0, jb, Linv, flag);
      const int64_t r0 = j0 + jb;
      if (r0 < rows) {
        const int64_t nblk = (rows - r0 + NB - 1) / NB;
        hipLaunchKernelGGL(k_trsm, dim3((unsigned)nblk), dim3(256), 0, s, Wm, ld, j0, jb, r0, rows, Linv);
      }
      // update the rest of this outer panel with the freshly solved columns
      launch_update(Wm, ld, j0 + jb, rows, Jend, j0, j0 + jb, s);
    }
    // trailing matrix with the whole outer panel
    launch_update(Wm, ld, Jend, rows, n, J0, Jend, s);
  }
  return 0;
}

// ------------------------------------------------------------- y^T y
__global__ void k_sumsq_row(const double *__restrict__ Wm, int64_t n, int64_t ld, double *__restrict__ out) {
  __shared__ double part[256];
  const double *y = Wm + n * ld;
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < n; j += 256) s += y[j] * y[j];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = part[0];
}

void launch_sumsq_row(const double *Wm, int64_t n, int64_t ld, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_sumsq_row, dim3(1), dim3(256), 0, s, Wm, n, ld, out);
}

}  // namespace wlc
