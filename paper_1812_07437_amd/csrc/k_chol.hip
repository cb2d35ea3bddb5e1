// (S/N)^2 = D^T C^-1 D (Rizzato et al. 2019, eq. SNprim) by an FP64 Cholesky
// factorisation of the bordered matrix
//     M = [ C~    d~ ]        C~ = 2^t C 2^t,  d~ = 2^t d,
//         [ d~^T   . ]
// Factoring the first n columns of M leaves y = L^-1 d~ in its last row, and
// (S/N)^2 = y^T y.
//
// Left-looking over 256-wide panels: each panel first receives the update
// from every column to its left in one long-k MFMA product (k_update.hip),
// then is factored right-looking in 64-wide steps: the 64 x 64 diagonal block
// factored and inverted by one wavefront, the rows below multiplied by the
// inverse on MFMA, and the rest of the panel updated with a short product.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace wlc {

constexpr int NB = 64;       // inner panel width
constexpr int NB_OUT = 256;  // outer panel width
constexpr int64_t PART_ROWS = 524288;  // split-k scratch: slices x rows of 256 doubles

// ------------------------------------------------------------- prepare
// Lower triangle of M from the scaled covariance (f32 or f64) and d: one
// block per row and PREP_COLS columns, blocks right of the row's end exit.
// M is written with non-temporal stores (it is far larger than the caches).
constexpr int PREP_COLS = 2048;
template <typename InT>
__global__ void k_chol_prep(const InT *__restrict__ C, const int32_t *__restrict__ t, const double *__restrict__ d,
                            const int32_t *__restrict__ perm, int64_t n, int64_t ld, int64_t row_off,
                            double *__restrict__ Wm) {
  const int64_t i = row_off + blockIdx.y;  // row of M, 0..n
  const int64_t jb = (int64_t)blockIdx.x * PREP_COLS;
  if (i > n || jb > i) return;  // the block lies right of the row's last entry
  const int64_t pi = perm && i < n ? perm[i] : i;
#pragma unroll
  for (int q = 0; q < PREP_COLS / 256; ++q) {
    const int64_t j = jb + q * 256 + threadIdx.x;
    if (j <= i && j < n) {
      const int64_t pj = perm ? perm[j] : j;
      __builtin_nontemporal_store(i < n ? (double)C[pi * n + pj] : ldexp(d[pj], t[pj]), &Wm[i * ld + j]);
    }
  }
}

void launch_chol_prep(const void *C, int c_f32, const int32_t *row_exp2, const double *d, int64_t n, int64_t ld,
                      double *Wm, hipStream_t s, const int32_t *perm) {
  for (int64_t r0 = 0; r0 <= n; r0 += 65535) {
    const int64_t rows = std::min<int64_t>(65535, n + 1 - r0);
    const dim3 grid((unsigned)((n + PREP_COLS - 1) / PREP_COLS), (unsigned)rows);
    if (c_f32)
      hipLaunchKernelGGL(k_chol_prep<float>, grid, dim3(256), 0, s, (const float *)C, row_exp2, d, perm, n, ld, r0,
                         Wm);
    else
      hipLaunchKernelGGL(k_chol_prep<double>, grid, dim3(256), 0, s, (const double *)C, row_exp2, d, perm, n, ld,
                         r0, Wm);
  }
}

// ------------------------------------------------------------- diagonal block
// One workgroup of 256 threads on the jb x jb diagonal block at j0 (rows
// beyond jb padded with the identity), held in registers: thread
// t = 16 tj + ti owns rows 4 ti .. 4 ti + 3 and columns 4 tj .. 4 tj + 3.
// The factorisation runs square-root free, as A = U D U^T with U unit lower,
// and inverts U in the same pass: at step k the owners of column k publish
// it in LDS as it stands (the Schur complement column, d_k = its diagonal
// entry, U[i][k] = a[i][k] / d_k), the owners of row k of V publish that
// row (final after step k - 1), and after one barrier every thread applies
// -a[i][k] a[j][k] / d_k to its block of A and -U[i][k] V[k][j] to its block
// of V (V = I at the start, V = U^-1 at the end: forward substitution with
// a unit diagonal).  Each step is one chain of dependent instructions with
// no square root and one division; the updates mask the broadcast factors
// rather than each product, and entries above the diagonal of a thread's
// block take harmless updates that are never read.  The published vectors
// alternate between two LDS buffers, so one barrier per step suffices.
// Afterwards d_k is the diagonal of A, and in one parallel pass
// L = U D^1/2 (L[i][k] = a[i][k] / sqrt(d_k)) goes back to the matrix and
// X = L^-1 = D^-1/2 V to Linv (row-major, NB columns).
__device__ __forceinline__ double pick4(const double (&v)[4], int c) {
  return c == 0 ? v[0] : c == 1 ? v[1] : c == 2 ? v[2] : v[3];
}

__global__ __launch_bounds__(256) void k_potrf_diag(double *__restrict__ Wm, int64_t ld, int64_t j0, int jb,
                                                    double *__restrict__ Linv, int *__restrict__ flag) {
  __shared__ double vcol[2][NB];  // column k of the Schur complement
  __shared__ double vrow[2][NB];  // row k of V
  __shared__ double dsq[NB], dinv[NB];  // sqrt(d_k) and its reciprocal
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int ti = tid & 15, tj = tid >> 4;
  const int i0 = 4 * ti, c0 = 4 * tj;
  double a[4][4], x[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      // every load unconditional, from the block's lower triangle (the
      // mirror position above the diagonal, clamped to the block), and
      // masked arithmetically, so all are in flight at once
      const int i = i0 + r, j = c0 + c;
      const double w = Wm[(j0 + min(max(i, j), jb - 1)) * ld + j0 + min(min(i, j), jb - 1)];
      a[r][c] = w * ((i < jb && j <= i) ? 1.0 : 0.0) + ((i >= jb && i == j) ? 1.0 : 0.0);
      x[r][c] = i == j ? 1.0 : 0.0;
    }
  if (tid == 0) bad = 0;
  // unrolled by four so that the column within a thread's block is a constant
#pragma unroll 4
  for (int k = 0; k < NB; ++k) {
    const int kb = k >> 2, kc = k & 3, buf = k & 1;
    if (tj == kb) {
#pragma unroll
      for (int r = 0; r < 4; ++r) vcol[buf][i0 + r] = pick4(a[r], kc);
    }
    if (ti == kb) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double col[4] = {x[0][c], x[1][c], x[2][c], x[3][c]};
        vrow[buf][c0 + c] = pick4(col, kc);
      }
    }
    __syncthreads();
    // all reads first and unconditionally (masked afterwards), so that
    // they overlap one another and the division
    const double dk = vcol[buf][k];
    double ci[4], cj[4], vk[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ci[q] = vcol[buf][i0 + q];
      cj[q] = vcol[buf][c0 + q];
      vk[q] = vrow[buf][c0 + q];
    }
    const double rd = dk > 0.0 ? 1.0 / dk : 0.0;
    double li[4], lj[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      li[q] = i0 + q > k ? ci[q] : 0.0;
      lj[q] = c0 + q > k ? cj[q] * rd : 0.0;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double u = li[r] * rd;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        a[r][c] -= li[r] * lj[c];
        x[r][c] -= u * vk[c];
      }
    }
  }
  if (ti == tj) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double dk = a[r][r];
      if (!(dk > 0.0)) bad = 1;
      const double sq = sqrt(dk > 0.0 ? dk : 1.0);
      dsq[i0 + r] = sq;
      dinv[i0 + r] = 1.0 / sq;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = i0 + r, j = c0 + c;
      if (i < jb && j <= i) Wm[(j0 + i) * ld + j0 + j] = j < i ? a[r][c] * dinv[j] : dsq[j];
      Linv[i * NB + j] = j <= i ? x[r][c] * dinv[i] : 0.0;
    }
  if (tid == 0 && bad) atomicOr(flag, 1);
}

// ------------------------------------------------------------- panel solve
// Rows [r0, r1) of columns [j0, j0 + jb): X = B L^-T, 64 rows per
// workgroup; four wavefronts each compute a 32 x 32 quadrant on
// v_mfma_f64_16x16x4 (accumulator rows l / 16 + 4 v, columns l % 16).
__global__ __launch_bounds__(256) void k_trsm(double *__restrict__ Wm, int64_t ld, int64_t j0, int jb, int64_t r0,
                                              int64_t r1, const double *__restrict__ Linv) {
  __shared__ double Li[NB][NB + 1];
  __shared__ double B[NB][NB + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t rb = r0 + (int64_t)blockIdx.x * NB;
  // all 32 loads of a thread in flight together: unconditional, from
  // addresses clamped into the panel (entries below the diagonal block,
  // finite), masked arithmetically afterwards
  double lv[NB * NB / 256], bv[NB * NB / 256];
#pragma unroll
  for (int m = 0; m < NB * NB / 256; ++m) {
    const int q = tid + 256 * m, i = q / NB, c = q % NB;
    lv[m] = Linv[q];
    const double w = Wm[min(rb + i, r1 - 1) * ld + j0 + min(c, jb - 1)];
    bv[m] = w * ((rb + i < r1 && c < jb) ? 1.0 : 0.0);
  }
#pragma unroll
  for (int m = 0; m < NB * NB / 256; ++m) {
    const int q = tid + 256 * m;
    Li[q / NB][q % NB] = lv[m];
    B[q / NB][q % NB] = bv[m];
  }
  __syncthreads();
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < NB; kk += 4) {
    const int kc = kk + (lane >> 4);
    double a[2], b[2];
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
      a[blk] = B[wr + blk * 16 + (lane & 15)][kc];
      b[blk] = Li[wc + blk * 16 + (lane & 15)][kc];  // (L^-T)[k][j] = Linv[j][k]
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = wr + x * 16 + (lane >> 4) + 4 * v;
        const int c = wc + y * 16 + (lane & 15);
        if (rb + i < r1 && c < jb) Wm[(rb + i) * ld + j0 + c] = acc[x][y][v];
      }
}

// Factor columns [0, n) of M (n + 1 rows).  scratch: the 64 x 64 inverse of
// the current diagonal block, then the split-k buffer of the panel updates.
// The pivot flag is checked by the caller after synchronisation.
int chol_factor(double *Wm, int64_t n, int64_t ld, double *scratch, int *flag, hipStream_t s,
                KernelProbe *probe) {
  const int64_t rows = n + 1;
  double *Linv = scratch;
  double *part = scratch + NB * NB;
  for (int64_t J0 = 0; J0 < n; J0 += NB_OUT) {
    const int64_t Jend = std::min<int64_t>(J0 + NB_OUT, n);
    // everything left of the panel, in one product over k = [0, J0)
    launch_update2(Wm, ld, J0, rows, Jend, 0, J0, part, chol_part_rows(n), s, probe);
    for (int64_t j0 = J0; j0 < Jend; j0 += NB) {
      const int jb = (int)std::min<int64_t>(NB, Jend - j0);
      hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, s, Wm, ld, j0, jb, Linv, flag);
      const int64_t r0 = j0 + jb;
      if (r0 < rows) {
        const int64_t nblk = (rows - r0 + NB - 1) / NB;
        hipLaunchKernelGGL(k_trsm, dim3((unsigned)nblk), dim3(256), 0, s, Wm, ld, j0, jb, r0, rows, Linv);
      }
      // the rest of this panel with the freshly solved columns
      launch_update2(Wm, ld, j0 + jb, rows, Jend, j0, j0 + jb, nullptr, 0, s, probe);
    }
  }
  return 0;
}

// Split-k scratch rows for an n x n factorisation: the long panel updates
// have k ranges below n, so they take at most update2_max_slices(n) slices
// of at most n + 1 rows each; small matrices reserve little.  The reserve
// never binds the split choice below PART_ROWS, so it does not change it.
int64_t chol_part_rows(int64_t n) { return std::min<int64_t>(PART_ROWS, update2_max_slices(n) * (n + 1)); }
size_t chol_scratch_bytes(int64_t n) { return (size_t)NB * NB * 8 + (size_t)chol_part_rows(n) * NB_OUT * 8; }

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

// Prefix sums of y^2 (the last row of the bordered factor) at the group ends
// ends[0] <= ... <= ends[ng-1] = n: one block sums each group, then one
// thread accumulates the groups in order.
__global__ void k_sumsq_groups(const double *__restrict__ Wm, int64_t n, int64_t ld, const int32_t *__restrict__ ends,
                               double *__restrict__ part) {
  __shared__ double red[256];
  const int g = blockIdx.x;
  const int64_t lo = g == 0 ? 0 : ends[g - 1], hi = ends[g];
  const double *y = Wm + n * ld;
  double s = 0.0;
  for (int64_t j = lo + threadIdx.x; j < hi; j += 256) s += y[j] * y[j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[g] = red[0];
}

__global__ void k_prefix(const double *__restrict__ part, int ng, double *__restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int g = 0; g < ng; ++g) {
    s += part[g];
    out[g] = s;
  }
}

void launch_sumsq_groups(const double *Wm, int64_t n, int64_t ld, const int32_t *ends, int ng, double *part,
                         double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_sumsq_groups, dim3((unsigned)ng), dim3(256), 0, s, Wm, n, ld, ends, part);
  hipLaunchKernelGGL(k_prefix, dim3(1), dim3(64), 0, s, part, ng, out);
}

}  // namespace wlc
