// 128 x 256 FP64 product tile for 512-thread workgroups (8 wavefronts on a
// 2 x 4 grid, 64 x 64 each on v_mfma_f64_16x16x4; the accumulator value v of
// lane l is row l / 16 + 4 v, column l % 16 of a 16 x 16 block):
//   acc[i][j] += sum_k R[i][k] S[j][k],  i < 128 (row side), j < 256 (column side),
// with R and S two row-major panels of one matrix (row pitch ld) read over
// n_st 16-wide k steps from column kb.
//
// Operands go from global memory straight into LDS (buffer loads with the LDS
// flag: lane l of a wavefront writes 16 bytes at the wavefront's LDS base +
// 16 l) through three buffers: step s + 2 is copied while step s is
// multiplied, one barrier per step.  A step holds 16 k of the 128 + 256 rows,
// 128 B per row, unpadded; the 16-byte chunk c of row r sits at slot
// c ^ ((r >> 1) & 7).  A wavefront copy fills 8 rows, lane l taking slot l & 7
// of row l >> 3 and fetching the chunk that the swizzle puts there.  Rows past
// nR / nS read as zero: each side's buffer descriptor ends at its last valid
// row.  Within a step, lane group g = l / 16 holds k = 4 g .. 4 g + 3 of its
// row in two halves (16-byte reads, free of bank conflicts): half 0 is
// k = 4 g, 4 g + 1, half 1 is k = 4 g + 2, 4 g + 3, and MFMA j takes k = 4 g + j
// from every group; both operands use the same map, so each k is summed once.
// Half 0 of step s + 1 is read into registers while step s is multiplied, so
// after each barrier the matrix cores start at once on registers that are
// already there; every accumulator still sums its k in increasing j order
// within a step.
//
// Requirements (checked by the callers on the host): ld and kb even (16-byte
// aligned chunks) and 256 ld 8 < 2^31 (a side within one descriptor).
#pragma once

#include <hip/hip_runtime.h>

#include "dev.h"

namespace wlc {

constexpr int FT_R = 128, FT_S = 256, FT_K = 16, FT_ROWS = FT_R + FT_S;

__device__ __forceinline__ int ft_slot(int r, int c) { return r * FT_K + 2 * (c ^ ((r >> 1) & 7)); }

__device__ __forceinline__ void f64_tile_product(const double *R, const double *S, int64_t ld, int64_t nR,
                                                 int64_t nS, int64_t kb, int64_t n_st, f64x4 (&acc)[4][4]) {
  __shared__ __attribute__((aligned(16))) double lds0[FT_ROWS * FT_K];
  __shared__ __attribute__((aligned(16))) double lds1[FT_ROWS * FT_K];
  __shared__ __attribute__((aligned(16))) double lds2[FT_ROWS * FT_K];
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = (wave / 4) * 64, wc = (wave % 4) * 64;
  // copies: wavefront w takes the 8-row groups q * 8 + w, q < 6 (groups 0-15
  // are the row side, 16-47 the column side)
  uint32_t off[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int r = (q * 8 + wave) * 8 + (lane >> 3);  // LDS row
    const int rs = q < 2 ? r : r - FT_R;             // row within its side
    const int c = (lane & 7) ^ ((r >> 1) & 7);
    off[q] = (uint32_t)(rs * ld * 8 + 16 * c);
  }
  auto issue = [&](int64_t k, double *buf) {
    const __amdgpu_buffer_rsrc_t rr =
        __builtin_amdgcn_make_buffer_rsrc((void *)(R + k), 0, (int)(nR * ld * 8), 0x00020000);
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)(S + k), 0, (int)(nS * ld * 8), 0x00020000);
#pragma unroll
    for (int q = 0; q < 6; ++q)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          q < 2 ? rr : rs, (__attribute__((address_space(3))) void *)(buf + (q * 8 + wave) * 8 * FT_K), 16, off[q],
          0, 0, 0);
    // the copies go out before the products that follow (the scheduler would
    // otherwise sink them next to the wait for them)
    __builtin_amdgcn_sched_barrier(0);
  };
  const int g = lane >> 4;
  // one half of a step's operands: a[x][j] = R row wr + 16 x + l % 16, b[y][j]
  // = S row wc + 16 y + l % 16, at k = 4 g + 2 h + j
  auto read_half = [&](const double *buf, int h, double (&a)[4][2], double (&b)[4][2]) {
#pragma unroll
    for (int blk = 0; blk < 4; ++blk) {
      const int ra = wr + blk * 16 + (lane & 15), rb = FT_R + wc + blk * 16 + (lane & 15);
      const double2 av = *(const double2 *)&buf[ft_slot(ra, 2 * g + h)];
      const double2 bv = *(const double2 *)&buf[ft_slot(rb, 2 * g + h)];
      a[blk][0] = av.x; a[blk][1] = av.y;
      b[blk][0] = bv.x; b[blk][1] = bv.y;
    }
    __builtin_amdgcn_sched_barrier(0);
  };
  auto mfma_half = [&](const double (&a)[4][2], const double (&b)[4][2]) {
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x][j], b[y][j], acc[x][y], 0, 0, 0);
    __builtin_amdgcn_sched_barrier(0);
  };
  double pa[4][2], pb[4][2], qa[4][2], qb[4][2];
  // step s: its half 0 is in (pa, pb); cur holds it, nxt step s + 1, fill
  // receives step s + 2 (the buffer of step s - 1)
  auto step = [&](int64_t s, const double *cur, const double *nxt, double *fill) {
    // this wavefront's copy of step s + 1 is complete; after the barrier every
    // wavefront's is, and no wavefront still reads step s - 1's buffer
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
    if (s + 2 < n_st) issue(kb + (s + 2) * FT_K, fill);
    read_half(cur, 1, qa, qb);
    mfma_half(pa, pb);
    if (s + 1 < n_st) read_half(nxt, 0, pa, pb);
    mfma_half(qa, qb);
  };
  if (n_st <= 0) return;
  issue(kb, lds0);
  if (n_st > 1) {
    issue(kb + FT_K, lds1);
    __builtin_amdgcn_s_waitcnt(0x0F76);  // vmcnt(6): step 0's copies are complete
  } else {
    __builtin_amdgcn_s_waitcnt(0x0F70);
  }
  __syncthreads();
  read_half(lds0, 0, pa, pb);
  // the three buffers are distinct arrays and the loop is unrolled by three,
  // so the compiler can tell the buffers being filled from those being read
  int64_t st = 0;
  for (; st + 2 < n_st; st += 3) {
    step(st, lds0, lds1, lds2);
    step(st + 1, lds1, lds2, lds0);
    step(st + 2, lds2, lds0, lds1);
  }
  if (st < n_st) step(st, lds0, lds1, lds2);
  if (st + 1 < n_st) step(st + 1, lds1, lds2, lds0);
}

}  // namespace wlc
