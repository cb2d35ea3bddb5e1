// Block update of the FP64 Cholesky factorisation:
//   W[i][j] -= sum_{q in [k0, k1)} W[i][q] W[j][q],  i in [c0, r1), j in [c0, c1), i >= j,
// on tiles of 128 rows by 128 or 256 columns: 128 x 256 tiles (8 wavefronts,
// k_update2d) span a whole 256-wide panel, so that each row slice is read
// once per launch (21.3 instead of 16 flops per operand byte); other shapes
// go on 128 x 128 tiles (4 wavefronts, k_update2<4>).  Each wavefront
// computes 64 x 64 on v_mfma_f64_16x16x4 (the accumulator value v of lane l
// is row l / 16 + 4 v, column l % 16).  K advances in 16-wide steps with one
// barrier per step: the wide kernel copies operands from global memory
// straight into three LDS buffers two steps ahead (the tile product of
// f64tile.h), the narrow one stages them through registers two steps ahead
// into two LDS buffers.  The register budget is capped at
// two wavefronts per SIMD.  A long k range may be split into slices whose
// partial products go to a scratch buffer and are subtracted in a fixed order
// by a second kernel, so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "f64tile.h"
#include "kernels.h"

namespace wlc {

constexpr int UT2 = 128;
constexpr int UBK = 16;
constexpr int ULDR = UBK + 1;

__device__ __forceinline__ void tile_of(int64_t t, int tri, int64_t tcols, int64_t &ti, int64_t &tj) {
  if (tri) {
    int64_t i = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    while (i * (i + 1) / 2 > t) --i;
    ti = i;
    tj = t - i * (i + 1) / 2;
  } else {
    ti = t / tcols;
    tj = t % tcols;
  }
}

// Write a wavefront's 64 x 64 result (rows i0 + wr.., columns j0 + wc..):
// into the split-k scratch (rows and columns relative to c0), or subtracted
// from W.  The subtraction reads W 16 entries at a time, all loads of a
// batch in flight together and from clamped addresses inside the block
// (their values are dropped where the entry is not written), instead of
// one load and wait per entry.
__device__ __forceinline__ void tile_epilogue(double *__restrict__ Wm, int64_t ld, int64_t i0, int64_t j0, int wr,
                                              int wc, int lane, int64_t c0, int64_t r1, int64_t c1,
                                              double *__restrict__ pdst, const f64x4 (&acc)[4][4]) {
  const int64_t pcols = c1 - c0;
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    double w[4][4];
    if (!pdst) {
#pragma unroll
      for (int y = 0; y < 4; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t i = min(i0 + wr + x * 16 + (lane >> 4) + 4 * v, r1 - 1);
          const int64_t j = min(j0 + wc + y * 16 + (lane & 15), c1 - 1);
          w[y][v] = Wm[i * ld + j];
        }
    }
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = i0 + wr + x * 16 + (lane >> 4) + 4 * v;
        const int64_t j = j0 + wc + y * 16 + (lane & 15);
        if (i < r1 && j < c1 && i >= j) {
          if (pdst) pdst[(i - c0) * pcols + (j - c0)] = acc[x][y][v];
          else Wm[i * ld + j] = w[y][v] - acc[x][y][v];
        }
      }
  }
}

// Register-staged form: in each 4-wide k step lane l holds row l % 16, k
// l / 16 of each operand; the LDS rows are padded by one element.
template <int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_update2(
    double *__restrict__ Wm, int64_t ld, int64_t c0, int64_t r1, int64_t c1, int64_t k0, int64_t k1, int tri_grid,
    int64_t tcols, int n_split, int64_t k_split, double *__restrict__ part) {
  constexpr int NT = 64 * NW;                // threads
  constexpr int TC = 32 * NW;                // tile columns
  constexpr int PR = UT2 * (UBK / 2) / NT;   // double2 chunks per thread, row side
  constexpr int PC = TC * (UBK / 2) / NT;    // double2 chunks per thread, column side
  __shared__ double lds[2][(UT2 + TC) * ULDR];  // [buffer][rows, then columns]
  int64_t ti, tj;
  tile_of(blockIdx.x / n_split, tri_grid, tcols, ti, tj);
  const int split = blockIdx.x % n_split;
  const int64_t i0 = c0 + ti * UT2, j0 = c0 + tj * TC;
  if (j0 > i0 + UT2 - 1) return;  // entirely above the diagonal
  const int64_t kb = k0 + (int64_t)split * k_split;
  const int64_t ke = min(k1, kb + k_split);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave / (NW / 2)) * 64, wc = (wave % (NW / 2)) * 64;
  f64x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};

  // each side: rows x 16 k as double2 chunks; chunk q is row q >> 3, pair q & 7
  double2 pr[PR], pc[PC];
  auto load_side = [&](double2 *dst, int per, int64_t base, int64_t lim, int64_t kq) {
    for (int q = 0; q < per; ++q) {
      const int ch = tid + NT * q;
      const int r = ch >> 3, c = ch & 7;
      const int64_t row = base + r, k = kq + 2 * c;
      double2 v = make_double2(0.0, 0.0);
      if (row < lim) {
        const double *src = Wm + row * ld + k;
        if (k + 1 < ke) v = *(const double2 *)src;
        else if (k < ke) v.x = src[0];
      }
      dst[q] = v;
    }
  };
  auto gload = [&](int64_t kq) {
    load_side(pr, PR, i0, r1, kq);
    load_side(pc, PC, j0, c1, kq);
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < PR; ++q) {
      const int ch = tid + NT * q;
      const int r = ch >> 3, c = ch & 7;
      lds[buf][r * ULDR + 2 * c] = pr[q].x;
      lds[buf][r * ULDR + 2 * c + 1] = pr[q].y;
    }
#pragma unroll
    for (int q = 0; q < PC; ++q) {
      const int ch = tid + NT * q;
      const int r = ch >> 3, c = ch & 7;
      lds[buf][(UT2 + r) * ULDR + 2 * c] = pc[q].x;
      lds[buf][(UT2 + r) * ULDR + 2 * c + 1] = pc[q].y;
    }
  };
  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < UBK; kk += 4) {
      const int kc = kk + (lane >> 4);
      double a[4], b[4];
#pragma unroll
      for (int blk = 0; blk < 4; ++blk) {
        a[blk] = lds[buf][(wr + blk * 16 + (lane & 15)) * ULDR + kc];
        b[blk] = lds[buf][(UT2 + wc + blk * 16 + (lane & 15)) * ULDR + kc];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
    }
  };

  // the last step may be partial: gload zero-fills k >= ke
  const int64_t n_st = (ke - kb + UBK - 1) / UBK;
  if (n_st > 0) {
    gload(kb);
    lstore(0);
    if (n_st > 1) gload(kb + UBK);
    __syncthreads();
  }
  // the next step's LDS copy and the global fetch of the one after are
  // issued before this step's products (measured 0.5 % faster than after)
  for (int64_t st = 0; st < n_st; ++st) {
    if (st + 1 < n_st) {
      lstore((int)((st + 1) & 1));  // that buffer was last read before the previous barrier
      if (st + 2 < n_st) gload(kb + (st + 2) * UBK);
    }
    compute((int)(st & 1));
    __syncthreads();
  }
  double *pdst = n_split > 1 ? part + (int64_t)split * (r1 - c0) * (c1 - c0) : nullptr;
  tile_epilogue(Wm, ld, i0, j0, wr, wc, lane, c0, r1, c1, pdst, acc);
}

// The 128 x 256 update: the tile product of f64tile.h on the row slice
// [i0, i0 + 128) and the panel's columns [c0, c0 + 256), then the subtraction
// (or the split-k partial store).
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_update2d(
    double *__restrict__ Wm, int64_t ld, int64_t c0, int64_t r1, int64_t c1, int64_t k0, int64_t k1, int n_split,
    int64_t k_split, double *__restrict__ part) {
  const int64_t ti = blockIdx.x / n_split;
  const int split = blockIdx.x % n_split;
  const int64_t i0 = c0 + ti * UT2, j0 = c0;
  const int64_t kb = k0 + (int64_t)split * k_split;
  const int64_t ke = min(k1, kb + k_split);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = (wave / 4) * 64, wc = (wave % 4) * 64;
  f64x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  // the host passes whole 16-wide steps only
  f64_tile_product(Wm + i0 * ld, Wm + j0 * ld, ld, min((int64_t)FT_R, r1 - i0), min((int64_t)FT_S, c1 - j0), kb,
                   (ke - kb) / FT_K, acc);
  double *pdst = n_split > 1 ? part + (int64_t)split * (r1 - c0) * (c1 - c0) : nullptr;
  tile_epilogue(Wm, ld, i0, j0, wr, wc, lane, c0, r1, c1, pdst, acc);
}

// W[i][j] -= sum_s part[s][i - c0][j - c0] for the lower part of the block.
__global__ void k_update_reduce(double *__restrict__ Wm, int64_t ld, int64_t c0, int64_t r1, int64_t c1, int n_split,
                                const double *__restrict__ part) {
  const int64_t pc = c1 - c0, rows = r1 - c0;
  const int64_t total = rows * pc;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = c0 + e / pc, j = c0 + e % pc;
    if (i < j) continue;
    double s = part[e];
    for (int q = 1; q < n_split; ++q) s += part[q * total + e];
    Wm[i * ld + j] -= s;
  }
}

// The most k slices the split rule below can choose for a k range of k_len:
// a slice keeps at least 32 k-steps, and there are at most 64 slices.
int64_t update2_max_slices(int64_t k_len) {
  const int64_t q = (k_len + UBK - 1) / UBK / 32;
  return q < 1 ? 1 : (q > 64 ? 64 : q);
}

void launch_update2(double *Wm, int64_t ld, int64_t c0, int64_t r1, int64_t c1, int64_t k0, int64_t k1,
                    double *part, int64_t part_rows, hipStream_t s, KernelProbe *probe) {
  if (c0 >= c1 || c0 >= r1 || k0 >= k1) return;
  const bool timed = probe && probe->ev && probe->count < probe->cap;
  if (probe) {
    const double cols = (double)(c1 - c0);
    const double lower = cols * (double)r1 - (double)(c0 + c1 - 1) * cols / 2.0;  // entries with i >= j
    probe->flops += 2.0 * lower * (double)(k1 - k0);
    ++probe->launches;
  }
  if (timed) (void)hipEventRecord(probe->ev[2 * probe->count], s);
  // a whole 256-wide panel below its diagonal block goes on 128 x 256 tiles
  // (k_update2d: whole 16-wide stages, 16-byte aligned rows and a 256-row
  // side within a buffer descriptor's 31-bit range, which the factorisation's
  // 64-multiple k ranges and 8-multiple row pitch always give); anything else,
  // and a k range of one inner block (64), where a tile is mostly its fill
  // and write-back and two workgroups per CU do better, on 128 x 128 tiles
  const bool wide = c1 - c0 > UT2 && c1 - c0 <= 2 * UT2 && r1 - c0 > 2 * UT2 && (k1 - k0) % UBK == 0 &&
                    k0 % 2 == 0 && ld % 2 == 0 && 2 * UT2 * ld * 8 < ((int64_t)1 << 31) && k1 - k0 > 64;
  const int64_t tcw = wide ? 2 * UT2 : UT2;
  const int64_t tr = (r1 - c0 + UT2 - 1) / UT2, tc = (c1 - c0 + tcw - 1) / tcw;
  const int tri = !wide && tr == tc;
  const int64_t tiles = tri ? tr * (tr + 1) / 2 : tr * tc;
  // Split the k range so that the workgroups fill whole rounds of the chip's
  // resident slots (two 4-wavefront or one 8-wavefront workgroup per CU): a
  // launch takes about ceil(tiles ns / slots) rounds of (ksteps / ns + 3)
  // k-steps, the 3 being a slice's pipeline fill and partial-tile traffic.
  // Each slice keeps at least 32 k-steps, and the scratch (slices x rows x
  // 256 doubles) stays within the part_rows x 256 doubles the caller
  // reserved.  The choice depends only on the shape, so results stay
  // deterministic.
  int ns = 1;
  if (part && c1 - c0 <= 256) {
    const int64_t ksteps = (k1 - k0 + UBK - 1) / UBK;
    const int64_t slots = wide ? 256 : 2 * 256;
    double best = (double)((tiles + slots - 1) / slots) * (double)(ksteps + 3);
    for (int q = 2; q <= 64; ++q) {
      if (ksteps / q < 32 || (int64_t)q * (r1 - c0) > part_rows) break;
      const double cost = (double)((tiles * q + slots - 1) / slots) * ((double)ksteps / q + 3.0);
      if (cost < best) {
        best = cost;
        ns = q;
      }
    }
  }
  const int64_t ksplit = ((k1 - k0 + UBK - 1) / UBK + ns - 1) / ns * UBK;
  if (wide)
    hipLaunchKernelGGL(k_update2d, dim3((unsigned)(tiles * ns)), dim3(512), 0, s, Wm, ld, c0, r1, c1, k0, k1, ns,
                       ksplit, part);
  else
    hipLaunchKernelGGL(k_update2<4>, dim3((unsigned)(tiles * ns)), dim3(256), 0, s, Wm, ld, c0, r1, c1, k0, k1, tri,
                       tc, ns, ksplit, part);
  if (ns > 1) {
    const int64_t total = (r1 - c0) * (c1 - c0);
    const unsigned g = (unsigned)std::min<int64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_update_reduce, dim3(g), dim3(256), 0, s, Wm, ld, c0, r1, c1, ns, part);
  }
  if (timed) (void)hipEventRecord(probe->ev[2 * probe->count++ + 1], s);
}

}  // namespace wlc
