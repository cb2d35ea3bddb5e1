// 128 x 256 FP64 product tile for 512-thread workgroups (8 wavefronts on a
// 2 x 4 grid, 64 x 64 each on v_mfma_f64_16x16x4; the accumulator value v of
// lane l is row l / 16 + 4 v, column l % 16 of a 16 x 16 block):
//   acc[i][j] += sum_k R[i][k] S[j][k],  i < 128 (row side), j < 256 (column side),
// with R and S two row-major panels of one matrix (row pitch ld) read over
// n_st 16-wide k steps from column kb.
//
// Operands go from global memory straight into LDS (buffer loads with the LDS
// flag: lane l of a wavefront writes 16 bytes at the wavefront's LDS base +
// 16 l), two buffers, step s + 1 copied while step s is multiplied, one
// barrier per step.  A step holds 16 k of the 128 + 256 rows, 128 B per row,
// unpadded; the 16-byte chunk c of row r sits at slot c ^ ((r >> 1) & 7).  A
// wavefront copy fills 8 rows, lane l taking slot l & 7 of row l >> 3 and
// fetching the chunk that the swizzle puts there.  Rows past nR / nS read as
// zero: each side's buffer descriptor ends at its last valid row.  Within a
// step, lane group g = l / 16 holds k = 4 g .. 4 g + 3 of its row (two
// 16-byte reads, free of bank conflicts), and MFMA step j takes k = 4 g + j
// from every group; both operands use the same map, so each k is summed once.
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
  auto compute = [&](const double *buf) {
    const int g = lane >> 4;
    double a[4][4], b[4][4];
#pragma unroll
    for (int blk = 0; blk < 4; ++blk) {
      const int ra = wr + blk * 16 + (lane & 15), rb = FT_R + wc + blk * 16 + (lane & 15);
      const double2 a0 = *(const double2 *)&buf[ft_slot(ra, 2 * g)], a1 = *(const double2 *)&buf[ft_slot(ra, 2 * g + 1)];
      const double2 b0 = *(const double2 *)&buf[ft_slot(rb, 2 * g)], b1 = *(const double2 *)&buf[ft_slot(rb, 2 * g + 1)];
      a[blk][0] = a0.x; a[blk][1] = a0.y; a[blk][2] = a1.x; a[blk][3] = a1.y;
      b[blk][0] = b0.x; b[blk][1] = b0.y; b[blk][2] = b1.x; b[blk][3] = b1.y;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x][j], b[y][j], acc[x][y], 0, 0, 0);
  };
  // the two buffers are distinct arrays and the loop is unrolled by two, so
  // the compiler can tell the buffer being filled from the one being read
  if (n_st > 0) issue(kb, lds0);
  int64_t st = 0;
  for (; st + 1 < n_st; st += 2) {
    // this wavefront's copy of step st is complete; after the barrier every
    // wavefront's is, and no wavefront still reads the buffer refilled next
    __builtin_amdgcn_sched_barrier(0);  // the previous step's products stay ahead of the wait
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __syncthreads();
    issue(kb + (st + 1) * FT_K, lds1);
    compute(lds0);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    if (st + 2 < n_st) issue(kb + (st + 2) * FT_K, lds0);
    compute(lds1);
  }
  if (st < n_st) {  // odd step count: the last step sits in buffer 0
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __syncthreads();
    compute(lds0);
  }
}

}  // namespace wlc
