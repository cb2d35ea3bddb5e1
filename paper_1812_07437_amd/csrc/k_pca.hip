// Principal components of the joint covariance (Rizzato et al. 2019, arXiv
// 1812.07437, Sec. 6): C = sum_a lambda_a S_a S_a^T (eq. SNPCA), the new
// observables D^_a = S_a . D (eq. NewObs) and their (S/N)^2_a = D^_a^2 /
// lambda_a (eq. SNperEign), with the cumulative curve of eq. CumulSN.
//
// The eigenvalues span tens of decades.  A tridiagonal eigensolver resolves
// only those above about 1e-16 of the largest, so this path uses one-sided
// (Hestenes) Jacobi, which keeps relative accuracy on graded matrices
// (Demmel and Veselic 1992): with C = Delta C^ Delta (Delta = 2^-t, the
// row scaling of the covariance) and C^ = L L^T from the bordered Cholesky,
// C = G^T G for G = L^T Delta.  Column rotations G -> G Q make the columns
// w_a of G Q orthogonal; then lambda_a = |w_a|^2, the eigenvectors are the
// columns of the accumulated Q, and since d = G^T y (y = L^-1 2^t d, the
// Cholesky's own forward substitution), D^_a = w_a . y.
//
// Storage: the columns of G are the rows of X (row j = 2^-t_j times row j of
// L, zero-padded to n_pad), and the columns of Q the rows of V, so every
// vector the method touches is a contiguous row.  Rows are grouped in blocks
// of 32; each round pairs all blocks (a round-robin tournament over n_blk =
// n_pad / 32 blocks, n_blk - 1 rounds per sweep); for each pair (p, q) the
// 64 x 64 Gram matrix of its rows is formed on FP64 MFMA, rotated towards
// diagonal form by cyclic two-sided Jacobi in LDS (relative accuracy again:
// rotations are driven by |M_jl| / sqrt(M_jj M_ll)), and the 64 x 64
// rotation is applied to its rows of X and V on FP64 MFMA.  Sweeps repeat
// until no pair has a scaled off-diagonal entry above tol.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace wlc {

constexpr int PB = 32;        // rows per block
constexpr int PR = 2 * PB;    // rows per pair
constexpr int PLD = PR + 1;   // padded LDS row

// Round-robin tournament: position 0 is fixed, the others rotate by r.
__device__ __forceinline__ int rr_at(int pos, int r, int n) { return pos == 0 ? 0 : 1 + (pos - 1 + r) % (n - 1); }

// X from the bordered factor Wm (rows 0..n-1: L in the lower triangle, row n:
// y): X[j][k] = 2^-t_j Wm[j][k] for k <= j < n, else 0; y_pad = row n of Wm;
// V = I when given.  One block row per blockIdx.y.
__global__ void k_pca_init(const double *__restrict__ Wm, int64_t ld, const int32_t *__restrict__ t, int64_t n,
                           int64_t n_pad, double *__restrict__ X, double *__restrict__ V, double *__restrict__ y) {
  const int64_t j = blockIdx.y;
  const double sc = j < n ? ldexp(1.0, -t[j]) : 0.0;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n_pad; k += (int64_t)gridDim.x * blockDim.x) {
    X[j * n_pad + k] = (j < n && k <= j) ? sc * Wm[j * ld + k] : 0.0;
    if (V) V[j * n_pad + k] = j == k ? 1.0 : 0.0;
    if (j == 0) y[k] = k < n ? Wm[n * ld + k] : 0.0;
  }
}

__device__ __forceinline__ void atomic_max_nonneg(double *addr, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax(reinterpret_cast<unsigned long long *>(addr), (unsigned long long)__double_as_longlong(v));
}

// A round is three launches.  (a) k_pca_gram: partial 64 x 64 Gram matrices
// of each block pair over KS column slices (FP64 MFMA); (b) k_pca_rot, one
// workgroup per pair: sum the slices in fixed order, measure the largest
// scaled off-diagonal entry, and unless it is below tol run Jacobi sweeps on
// M in LDS and store Q (reordering the rotated columns by norm, as in
// de Rijk's sorting, was measured to break the convergence of the cyclic
// tournament here);
// (c) k_pca_apply: rows of X (and V) <- Q^T rows, 64 columns per workgroup,
// skipped for pairs that did not rotate.
__device__ __forceinline__ int64_t pair_row(int bp, int bq, int j) {
  return j < PB ? (int64_t)bp * PB + j : (int64_t)bq * PB + (j - PB);
}

// Gram of a pair, with the pair's 64 rows
// are copied one 64-column chunk ahead into two LDS buffers of [64 rows][64
// doubles], unpadded, with the 16-byte chunk s of row l at slot s ^ (l & 15),
// so the 16 consecutive rows one MFMA operand read touches at one column
// fall on 16 distinct bank groups.  A wavefront copy fills two rows.
__device__ __forceinline__ int gram_slot(int l, int k) { return l * PR + 2 * ((k >> 1) ^ (l & 15)) + (k & 1); }

__global__ __launch_bounds__(256) void k_pca_gram(const double *__restrict__ X, int64_t n_pad, int n_blk, int r,
                                                    int64_t cols, double *__restrict__ part) {
  __shared__ __attribute__((aligned(16))) double st0[PR * PR];
  __shared__ __attribute__((aligned(16))) double st1[PR * PR];
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int pi = blockIdx.x, ks = blockIdx.y;
  const int bp = rr_at(pi, r, n_blk), bq = rr_at(n_blk - 1 - pi, r, n_blk);
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int64_t c0 = (int64_t)ks * cols;
  const int nch = (int)(cols / PR);
  // copy i of this wavefront: rows l0 = 2 (4 i + w) and l0 + 1 of the pair
  // (one 32-row block, so consecutive rows of X), one descriptor per copy
  const double *rows[8];
  uint32_t off[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int l0 = 2 * (i * 4 + wave), l = l0 + (lane >> 5);
    rows[i] = X + pair_row(bp, bq, l0) * n_pad;
    off[i] = (uint32_t)(((lane >> 5) * n_pad + 2 * ((lane & 31) ^ (l & 15))) * 8);
  }
  auto issue = [&](int ci, double *buf) {
#pragma unroll
    for (int i = 0; i < 8; ++i)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          __builtin_amdgcn_make_buffer_rsrc((void *)rows[i], 0, (int)(2 * n_pad * 8), 0x00020000),
          (__attribute__((address_space(3))) void *)(buf + (i * 4 + wave) * 2 * PR), 16, off[i],
          (int)((c0 + (int64_t)ci * PR) * 8), 0, 0);
    __builtin_amdgcn_sched_barrier(0);
  };
  f64x4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int z = 0; z < 2; ++z) acc[x][z] = f64x4{0.0, 0.0, 0.0, 0.0};
  auto compute = [&](const double *buf) {
#pragma unroll
    for (int kk = 0; kk < PR; kk += 4) {
      const int k = kk + (lane >> 4);
      double a[2], b[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        a[x] = buf[gram_slot(wr + x * 16 + (lane & 15), k)];
        b[x] = buf[gram_slot(wc + x * 16 + (lane & 15), k)];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int z = 0; z < 2; ++z) acc[x][z] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[z], acc[x][z], 0, 0, 0);
    }
  };
  if (nch > 0) issue(0, st0);
  int ci = 0;
  for (; ci + 1 < nch; ci += 2) {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wavefront's copy of chunk ci
    __syncthreads();
    issue(ci + 1, st1);
    compute(st0);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    if (ci + 2 < nch) issue(ci + 2, st0);
    compute(st1);
  }
  if (ci < nch) {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    compute(st0);
  }
  // accumulator value v of lane l: row l / 16 + 4 v, column l % 16
  double *P = part + ((int64_t)pi * gridDim.y + ks) * PR * PR;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int z = 0; z < 2; ++z)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        P[(wr + x * 16 + (lane >> 4) + 4 * v) * PR + wc + z * 16 + (lane & 15)] = acc[x][z][v];
}

constexpr int RT = 1024;  // threads of the rotation kernel: one 2 x 2 block each per inner step

__global__ __launch_bounds__(RT) void k_pca_rot(const double *__restrict__ part, int n_ks, double tol, int max_inner,
                                                 double *__restrict__ Qg, int32_t *__restrict__ rot,
                                                 double *__restrict__ conv) {
  __shared__ double M[PR * PLD];
  __shared__ double Q[PR * PLD];
  __shared__ double cs_c[PR], cs_s[PR], cs_t[PR];
    __shared__ double red[RT];
  const int tid = threadIdx.x, pi = blockIdx.x;
  for (int e = tid; e < PR * PR; e += RT) {
    const double *P = part + (int64_t)pi * n_ks * PR * PR + e;
    double v = 0.0;
    for (int k = 0; k < n_ks; ++k) v += P[(int64_t)k * PR * PR];
    M[(e / PR) * PLD + e % PR] = v;
    Q[(e / PR) * PLD + e % PR] = (e / PR == e % PR) ? 1.0 : 0.0;
  }
  __syncthreads();
  // symmetrise from the lower triangle and measure the largest scaled
  // off-diagonal entry
  double off = 0.0;
  for (int e = tid; e < PR * PR; e += RT) {
    const int j = e / PR, l = e % PR;
    if (l < j) {
      const double mjl = M[j * PLD + l];
      M[l * PLD + j] = mjl;
      const double den = sqrt(M[j * PLD + j] * M[l * PLD + l]);
      if (den > 0.0) off = fmax(off, fabs(mjl) / den);
    }
  }
  red[tid] = off;
  __syncthreads();
  for (int w = RT / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
    __syncthreads();
  }
  const double off0 = red[0];
  if (tid == 0) {
    atomic_max_nonneg(conv, off0);
    rot[pi] = off0 > tol ? 1 : 0;
  }
  if (!(off0 > tol)) return;  // this pair is already orthogonal
  __syncthreads();

  // cyclic two-sided Jacobi on M (in place), Q accumulates the rotations
  for (int sweep = 0; sweep < max_inner; ++sweep) {
    double inner = 0.0;
    for (int ir = 0; ir < PR - 1; ++ir) {
      if (tid < PR / 2) {
        const int j = rr_at(tid, ir, PR), l = rr_at(PR - 1 - tid, ir, PR);
        const double mjj = M[j * PLD + j], mll = M[l * PLD + l], mjl = M[j * PLD + l];
        const double den = sqrt(mjj * mll);
        double c = 1.0, sn = 0.0, tt = 0.0;
        if (den > 0.0 && fabs(mjl) > tol * den) {
          inner = fmax(inner, fabs(mjl) / den);
          const double th = (mll - mjj) / (2.0 * mjl);
          tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
          c = 1.0 / sqrt(1.0 + tt * tt);
          sn = c * tt;
        }
        // x_j' = c x_j - s x_l, x_l' = s x_j + c x_l
        cs_c[j] = c; cs_s[j] = -sn; cs_t[j] = -tt;
        cs_c[l] = c; cs_s[l] = sn;  cs_t[l] = tt;
      }
      __syncthreads();
      // 2 x 2 blocks (pair of i) x (pair of k), one per thread and step
      for (int bidx = tid; bidx < (PR / 2) * (PR / 2); bidx += RT) {
        const int qi = bidx / (PR / 2), qk = bidx % (PR / 2);
        const int i0 = rr_at(qi, ir, PR), i1 = rr_at(PR - 1 - qi, ir, PR);
        const int k0 = rr_at(qk, ir, PR), k1 = rr_at(PR - 1 - qk, ir, PR);
        if (qi == qk) {
          // the pair's own block: exact diagonal update, zero off-diagonal
          const double m01 = M[i0 * PLD + i1];
          if (cs_s[i0] != 0.0) {
            M[i0 * PLD + i0] += cs_t[i0] * m01;  // M_jj - t M_jl
            M[i1 * PLD + i1] += cs_t[i1] * m01;  // M_ll + t M_jl
            M[i0 * PLD + i1] = 0.0;
            M[i1 * PLD + i0] = 0.0;
          }
        } else {
          const double a00 = M[i0 * PLD + k0], a01 = M[i0 * PLD + k1], a10 = M[i1 * PLD + k0],
                       a11 = M[i1 * PLD + k1];
          // x_i' = c_i x_i + s_i x_(partner of i), on both sides
          const double ci0 = cs_c[i0], si0 = cs_s[i0], ci1 = cs_c[i1], si1 = cs_s[i1];
          const double ck0 = cs_c[k0], sk0 = cs_s[k0], ck1 = cs_c[k1], sk1 = cs_s[k1];
          const double r00 = ci0 * a00 + si0 * a10, r01 = ci0 * a01 + si0 * a11;
          const double r10 = ci1 * a10 + si1 * a00, r11 = ci1 * a11 + si1 * a01;
          M[i0 * PLD + k0] = ck0 * r00 + sk0 * r01;
          M[i0 * PLD + k1] = ck1 * r01 + sk1 * r00;
          M[i1 * PLD + k0] = ck0 * r10 + sk0 * r11;
          M[i1 * PLD + k1] = ck1 * r11 + sk1 * r10;
        }
      }
      // Q <- Q J: the two columns of each pair, row by row
      for (int e = tid; e < PR * (PR / 2); e += RT) {
        const int row = e / (PR / 2), qi = e % (PR / 2);
        const int i0 = rr_at(qi, ir, PR), i1 = rr_at(PR - 1 - qi, ir, PR);
        if (cs_s[i0] == 0.0) continue;
        const double q0 = Q[row * PLD + i0], q1 = Q[row * PLD + i1];
        Q[row * PLD + i0] = cs_c[i0] * q0 + cs_s[i0] * q1;
        Q[row * PLD + i1] = cs_c[i1] * q1 + cs_s[i1] * q0;
      }
      __syncthreads();
    }
    if (tid < PR / 2) red[tid] = inner;
    __syncthreads();
    if (tid == 0) {
      double m = 0.0;
      for (int q = 0; q < PR / 2; ++q) m = fmax(m, red[q]);
      red[0] = m;
    }
    __syncthreads();
    const bool done = !(red[0] > tol);
    __syncthreads();
    if (done) break;
  }
  double *out = Qg + (int64_t)pi * PR * PR;
  for (int e = tid; e < PR * PR; e += RT) out[e] = Q[(e / PR) * PLD + e % PR];
}

// Per mode a < n: lambda_a = |x_a|^2 and (S/N)^2_a = (x_a . y)^2 / lambda_a.
__global__ void k_pca_modes(const double *__restrict__ X, const double *__restrict__ y, int64_t n, int64_t n_pad,
                            double *__restrict__ lam, double *__restrict__ snr2) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t a = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  if (a >= n) return;
  const double *x = X + a * n_pad;
  double nn = 0.0, dy = 0.0;
  for (int64_t k = lane; k < n_pad; k += WAVE) {
    nn += x[k] * x[k];
    dy += x[k] * y[k];
  }
  nn = wave_sum(nn);
  dy = wave_sum(dy);
  if (lane == 0) {
    lam[a] = nn;
    snr2[a] = nn > 0.0 ? dy * dy / nn : 0.0;
  }
}

// Rank of each mode by ascending lambda (ties by index) and by descending
// (S/N)^2; outputs in those orders.
__global__ void k_pca_rank(const double *__restrict__ lam, const double *__restrict__ snr2, int64_t n,
                           int32_t *__restrict__ rank_lam, int32_t *__restrict__ rank_snr) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  const double la = lam[a], sa = snr2[a];
  int64_t rl = 0, rs = 0;
  for (int64_t b = 0; b < n; ++b) {
    const double lb = lam[b], sb = snr2[b];
    rl += (lb < la) || (lb == la && b < a);
    rs += (sb > sa) || (sb == sa && b < a);
  }
  rank_lam[a] = (int32_t)rl;
  rank_snr[a] = (int32_t)rs;
}

__global__ void k_pca_scatter(const double *__restrict__ lam, const double *__restrict__ snr2,
                              const int32_t *__restrict__ rank_lam, const int32_t *__restrict__ rank_snr, int64_t n,
                              double *__restrict__ lam_out, double *__restrict__ snr2_out,
                              double *__restrict__ desc) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  lam_out[rank_lam[a]] = lam[a];
  snr2_out[rank_lam[a]] = snr2[a];
  desc[rank_snr[a]] = snr2[a];
}

// Cumulative sum in place, in order, by one thread (n is at most a few 1e5).
__global__ void k_pca_cumsum(double *__restrict__ v, int64_t n) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int64_t a = 0; a < n; ++a) {
    s += v[a];
    v[a] = s;
  }
}

// Eigenvector rows in ascending-lambda order, first n entries, with the
// sign that makes the largest entry in magnitude positive.
__global__ void k_pca_vectors(const double *__restrict__ Vr, const int32_t *__restrict__ rank_lam, int64_t n,
                              int64_t n_pad, double *__restrict__ S) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const int64_t a = blockIdx.x;
  const double *v = Vr + a * n_pad;
  double best = -1.0;
  int64_t at = 0;
  for (int64_t k = threadIdx.x; k < n; k += blockDim.x)
    if (fabs(v[k]) > best) { best = fabs(v[k]); at = k; }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = at;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double o = bv[threadIdx.x + w];
      const int64_t oi = bi[threadIdx.x + w];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const double sg = v[bi[0]] < 0.0 ? -1.0 : 1.0;
  double *out = S + (int64_t)rank_lam[a] * n;
  for (int64_t k = threadIdx.x; k < n; k += blockDim.x) out[k] = sg * v[k];
}

void launch_pca_init(const double *Wm, int64_t ld, const int32_t *t, int64_t n, int64_t n_pad, double *X, double *V,
                     double *y, hipStream_t s) {
  const dim3 grid((unsigned)std::min<int64_t>((n_pad + 255) / 256, 64), (unsigned)n_pad);
  hipLaunchKernelGGL(k_pca_init, grid, dim3(256), 0, s, Wm, ld, t, n, n_pad, X, V, y);
}

// Rotation of a pair's rows.  Q's fragments stay in
// registers; the pair's 64 rows are copied from global memory straight into
// LDS (buffer loads with the LDS flag: lane l of a wavefront writes 16 bytes
// at the wavefront's LDS base + 16 l), one 64-column chunk ahead, into two
// buffers of [64 rows][64 doubles], unpadded, with the 16-byte chunk s of
// row l at slot s ^ (8 (l & 1)): the four rows one MFMA operand read touches
// fall on alternate halves of the banks.  A wavefront copy fills two rows.
constexpr int ACD = 8;  // 64-column chunks per workgroup

__device__ __forceinline__ int apply_slot(int l, int col) { return l * PR + 2 * ((col >> 1) ^ (8 * (l & 1))) + (col & 1); }

__global__ __launch_bounds__(256) void k_pca_apply(double *__restrict__ X, double *__restrict__ V, int64_t n_pad,
                                                     int n_blk, int r, const double *__restrict__ Qg,
                                                     const int32_t *__restrict__ rot) {
  __shared__ __attribute__((aligned(16))) double st0[PR * PR];
  __shared__ __attribute__((aligned(16))) double st1[PR * PR];
  const int pi = blockIdx.x;
  if (!rot[pi]) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int bp = rr_at(pi, r, n_blk), bq = rr_at(n_blk - 1 - pi, r, n_blk);
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  double *Y = blockIdx.z == 0 ? X : V;
  // Q fragments: step kk, block x: Q[kk + lane / 16][wr + 16 x + lane % 16]
  const double *q = Qg + (int64_t)pi * PR * PR;
  double qa[PR / 4][2];
#pragma unroll
  for (int kk = 0; kk < PR / 4; ++kk)
#pragma unroll
    for (int x = 0; x < 2; ++x) qa[kk][x] = q[(4 * kk + (lane >> 4)) * PR + wr + x * 16 + (lane & 15)];
  // copies: wavefront w fills LDS rows 2 (8 i + w) + lane / 32 ... for i < 8
  // copy i of this wavefront: rows l0 = 2 (4 i + w) and l0 + 1 of the pair
  // (one 32-row block, so consecutive rows of Y), one descriptor per copy
  const double *rows[8];
  uint32_t off[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int l0 = 2 * (i * 4 + wave), l = l0 + (lane >> 5);
    rows[i] = Y + pair_row(bp, bq, l0) * n_pad;
    off[i] = (uint32_t)(((lane >> 5) * n_pad + 2 * ((lane & 31) ^ (8 * (l & 1)))) * 8);
  }
  const int64_t cbase = (int64_t)blockIdx.y * ACD * PR;
  const int nch = (int)min((int64_t)ACD, (n_pad - cbase) / PR);
  auto issue = [&](int ci, double *buf) {
#pragma unroll
    for (int i = 0; i < 8; ++i)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          __builtin_amdgcn_make_buffer_rsrc((void *)rows[i], 0, (int)(2 * n_pad * 8), 0x00020000),
          (__attribute__((address_space(3))) void *)(buf + (i * 4 + wave) * 2 * PR), 16, off[i],
          (int)((cbase + (int64_t)ci * PR) * 8), 0, 0);
    __builtin_amdgcn_sched_barrier(0);
  };
  auto compute = [&](const double *buf, int ci) {
    f64x4 acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int z = 0; z < 2; ++z) acc[x][z] = f64x4{0.0, 0.0, 0.0, 0.0};
    // out[j][c] = sum_l Q[l][j] stage[l][c]
#pragma unroll
    for (int kk = 0; kk < PR / 4; ++kk) {
      const int l = 4 * kk + (lane >> 4);
      double b[2];
#pragma unroll
      for (int z = 0; z < 2; ++z) b[z] = buf[apply_slot(l, wc + z * 16 + (lane & 15))];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int z = 0; z < 2; ++z) acc[x][z] = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[kk][x], b[z], acc[x][z], 0, 0, 0);
    }
    const int64_t c0 = cbase + (int64_t)ci * PR;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int z = 0; z < 2; ++z)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = wr + x * 16 + (lane >> 4) + 4 * v, c = wc + z * 16 + (lane & 15);
          Y[pair_row(bp, bq, j) * n_pad + c0 + c] = acc[x][z][v];
        }
  };
  // the chunk written back is never one being copied (the copies run one
  // chunk ahead, on other columns)
  if (nch > 0) issue(0, st0);
  int ci = 0;
  for (; ci + 1 < nch; ci += 2) {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wavefront's copy of chunk ci
    __syncthreads();
    issue(ci + 1, st1);
    compute(st0, ci);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    if (ci + 2 < nch) issue(ci + 2, st0);
    compute(st1, ci + 1);
  }
  if (ci < nch) {
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    compute(st0, ci);
  }
}

// Column slices of the Gram: enough workgroups to cover the chip, each
// slice a multiple of 64 columns.
int pca_slices(int64_t n_pad) {
  const int pairs = (int)(n_pad / PB) / 2;
  int ks = 1;
  while (pairs * ks * 2 <= 1024 && n_pad % ((int64_t)ks * 2 * PR) == 0 && n_pad / (ks * 2) >= 256) ks *= 2;
  return ks;
}

void launch_pca_round(double *X, double *V, int64_t n_pad, int r, double tol, int max_inner, double *conv,
                      double *part, double *Qg, int32_t *rot, hipStream_t s) {
  const int n_blk = (int)(n_pad / PB), pairs = n_blk / 2, ks = pca_slices(n_pad);
  // slices are multiples of 64 columns
  hipLaunchKernelGGL(k_pca_gram, dim3((unsigned)pairs, (unsigned)ks), dim3(256), 0, s, X, n_pad, n_blk, r,
                     n_pad / ks, part);
  hipLaunchKernelGGL(k_pca_rot, dim3((unsigned)pairs), dim3(RT), 0, s, part, ks, tol, max_inner, Qg, rot, conv);
  hipLaunchKernelGGL(k_pca_apply, dim3((unsigned)pairs, (unsigned)((n_pad / PR + ACD - 1) / ACD), V ? 2u : 1u),
                     dim3(256), 0, s, X, V, n_pad, n_blk, r, Qg, rot);
}

void launch_pca_finish(const double *X, const double *y, const double *Vr, int64_t n, int64_t n_pad, double *lam,
                       double *snr2, int32_t *rank_lam, int32_t *rank_snr, double *lam_out, double *snr2_out,
                       double *desc, double *S, hipStream_t s) {
  hipLaunchKernelGGL(k_pca_modes, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, X, y, n, n_pad, lam, snr2);
  const unsigned g = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_pca_rank, dim3(g), dim3(256), 0, s, lam, snr2, n, rank_lam, rank_snr);
  hipLaunchKernelGGL(k_pca_scatter, dim3(g), dim3(256), 0, s, lam, snr2, rank_lam, rank_snr, n, lam_out, snr2_out,
                     desc);
  hipLaunchKernelGGL(k_pca_cumsum, dim3(1), dim3(64), 0, s, desc, n);
  if (S && Vr) hipLaunchKernelGGL(k_pca_vectors, dim3((unsigned)n), dim3(256), 0, s, Vr, rank_lam, n, n_pad, S);
}

}  // namespace wlc
